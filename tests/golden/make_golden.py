"""Writes the stored reference values of tests/golden/ that come from closed forms
the oracle package evaluates (nothing here calls the GPU library).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.closed_forms import bethe_e0  # noqa: E402


def main():
    out = {"source": "Bethe ansatz of the periodic spin-1/2 Heisenberg chain (J = Delta = 1) at n = L/2, "
                     "written by tests/golden/make_golden.py from oracle.closed_forms.bethe_e0",
           "E0": {str(L): bethe_e0(L) for L in (8, 10, 12, 16, 20, 24, 28, 32, 34)}}
    with open(os.path.join(HERE, "bethe_e0.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
