"""Writes the stored reference values of tests/golden/ that come from the oracle
package (nothing here calls the GPU library).

    python tests/golden/make_golden.py            closed forms (seconds)
    python tests/golden/make_golden.py appd       App. D's example at L = 28, n = 14:
                                                  the four lowest states by deflated
                                                  Lanczos on the C oracle (about an
                                                  hour on 8 cores, ~4 GB of memory)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.closed_forms import bethe_e0  # noqa: E402


def appd(L=28, num=4):
    """Energies and site magnetisations of the num lowest states of App. D's open
    chain in the field h_k = k (synth.tilted_field_chain), n = L/2."""
    import time

    import numpy as np

    import synth
    from oracle import native
    from oracle.observables import lowest_by_deflation

    n = L // 2
    bonds, jxy, jz, h = synth.tilted_field_chain(L)
    ns = native.NativeSector(2, L, n, [L // 2, L - L // 2])
    t = native.NativeTerms(bonds, jxy, jz, h)
    v0 = synth.vector(ns.dim, synth.SEED_V0)
    t0 = time.time()
    found = lowest_by_deflation(lambda v: native.hx_range(ns, t, v), v0, num, 3000,
                                log=lambda m: print(m, f"({time.time() - t0:.0f} s)", flush=True))
    states = []
    for E, psi, steps, res in found:
        exy, ez, esz = native.bond_sums(ns, bonds, psi, psi, fields=True)
        states.append({"E": E, "lanczos_steps": steps, "residual_norm": res,
                       "sz": [float(v) for v in esz], "xy": [float(v) for v in exy],
                       "zz": [float(v) for v in ez]})
        del psi
    out = {"source": "oracle.observables.lowest_by_deflation on the C oracle's product, "
                     "written by tests/golden/make_golden.py appd",
           "model": "open chain, Jxy = Jz = 1 on bonds (k, k+1), field h_k = k on every site k",
           "L": L, "n": n, "dim": ns.dim, "start_vector": "synth.vector(dim, synth.SEED_V0)",
           "bonds": [list(b) for b in bonds], "states": states}
    with open(os.path.join(HERE, f"appd_L{L}.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def main():
    out = {"source": "Bethe ansatz of the periodic spin-1/2 Heisenberg chain (J = Delta = 1) at n = L/2, "
                     "written by tests/golden/make_golden.py from oracle.closed_forms.bethe_e0",
           "E0": {str(L): bethe_e0(L) for L in (8, 10, 12, 16, 20, 24, 28, 32, 34)}}
    with open(os.path.join(HERE, "bethe_e0.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "appd":
        appd(*[int(a) for a in sys.argv[2:]])
    else:
        main()
