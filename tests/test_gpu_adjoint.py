"""GPU adjoint of y = H(theta) x: parity with the oracle gradients, autograd
gradcheck, finite differences (exact for a linear map) and the Hellmann-Feynman
ground-energy gradient."""
import numpy as np
import pytest
import torch

import paper_2407_14591_amd as dq
import synth
from gpu_common import DEV, rel_err, say
from oracle import native
from oracle.gradients import adjoint as o_adjoint, chain_rule_j_delta
from oracle.hamiltonian import apply_h, full_basis_digit_sums, full_matrix
from oracle.sector import BruteSector

pytestmark = pytest.mark.gpu


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


@pytest.mark.parametrize("Q,L,n,split", [(2, 10, 5, [5, 5]), (2, 12, 4, [4, 4, 4]),
                                         (2, 9, 4, [1, 2, 3, 3]), (3, 6, 6, [2, 2, 2]),
                                         (4, 5, 7, [2, 3])])
def test_adjoint_matches_oracle(Q, L, n, split):
    rng = np.random.default_rng(L * Q)
    b = BruteSector(Q, L, n, split)
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
    x, g = rng.normal(size=b.dim), rng.normal(size=b.dim)
    gx, gj, gz, gh = o_adjoint(b, bonds, jxy, jz, x, g, h)
    s, t = dq.Sector(L, n, Q, split), dq.Terms(bonds)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        out = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz),
                                           torch.tensor(x, device=DEV).to(dt),
                                           torch.tensor(g, device=DEV).to(dt), h=dev_f64(h),
                                           want_grad_h=True)
        say("adjoint", Q, L, n, dt)
        assert rel_err(out[0].double().cpu().numpy(), gx) <= tol
        assert rel_err(out[1].cpu().numpy(), gj) <= tol
        assert rel_err(out[2].cpu().numpy(), gz) <= tol
        assert rel_err(out[3].cpu().numpy(), gh) <= tol


def test_gradcheck_autograd():
    L, n = 8, 4
    s = dq.Sector(L, n, 2, [4, 4])
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    t = dq.Terms(bonds)
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.normal(size=s.dim), device=DEV, requires_grad=True)
    jxy = torch.tensor(rng.uniform(0.5, 1.5, len(bonds)), device=DEV, requires_grad=True)
    jz = torch.tensor(rng.uniform(0, 2, len(bonds)), device=DEV, requires_grad=True)
    f = lambda x_, a_, b_: dq.HApply.apply(x_, a_, b_, s, t)
    assert torch.autograd.gradcheck(f, (x, jxy, jz), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_differentiable_workload_L24():
    """L=24, n=12, per-bond J_b, Delta_b: coupling gradients against the C oracle
    (g . H_b x with one unit bond at a time) and grad_x = H g."""
    L, n, sp = 24, 12, [8, 8, 8]
    bonds = synth.chain_bonds(L, 1)
    J, Dl = synth.random_couplings(len(bonds))
    jxy, jz = J, J * Dl
    ns = native.NativeSector(2, L, n, sp)
    x = synth.vector(ns.dim, synth.SEED_X)
    g = synth.vector(ns.dim, synth.SEED_G)
    ref_gx = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), g)
    ref_gj = np.array([g @ native.hx_range(ns, native.NativeTerms([bd], [1.0], [0.0]), x) for bd in bonds])
    ref_gz = np.array([g @ native.hx_range(ns, native.NativeTerms([bd], [0.0], [1.0]), x) for bd in bonds])
    s, t = dq.Sector(L, n, 2, sp), dq.Terms(bonds)
    gx, gj, gz, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz),
                                                 torch.tensor(x, device=DEV),
                                                 torch.tensor(g, device=DEV))
    assert rel_err(gx.cpu().numpy(), ref_gx) <= 1e-12
    assert rel_err(gj.cpu().numpy(), ref_gj) <= 1e-12
    assert rel_err(gz.cpu().numpy(), ref_gz) <= 1e-12
    # chain rule to (J, Delta) through autograd against the oracle's chain rule
    Jt = torch.tensor(J, device=DEV, requires_grad=True)
    Dt = torch.tensor(Dl, device=DEV, requires_grad=True)
    y = dq.HApply.apply(torch.tensor(x, device=DEV), Jt, Jt * Dt, s, t)
    (y * torch.tensor(g, device=DEV)).sum().backward()
    gJ, gD = chain_rule_j_delta(J, Dl, ref_gj, ref_gz)
    assert rel_err(Jt.grad.cpu().numpy(), gJ) <= 1e-12
    assert rel_err(Dt.grad.cpu().numpy(), gD) <= 1e-12
    # deterministic: a second call is bitwise equal
    _, gj2, gz2, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz),
                                                  torch.tensor(x, device=DEV),
                                                  torch.tensor(g, device=DEV), want_grad_x=False)
    assert torch.equal(gj, gj2) and torch.equal(gz, gz2)


def hf_gradient(s, t, jxy, jz, steps=150):
    v0 = torch.tensor(synth.vector(s.dim, synth.SEED_V0), device=DEV)
    res = dq.lanczos(s, t, dev_f64(jxy), dev_f64(jz), v0, steps, reorth="full", num_eig=2,
                     want_vector=True)
    psi = res["vector"]
    _, gj, gz, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), psi, psi,
                                                want_grad_x=False)
    return res["eig"], gj.cpu().numpy(), gz.cpu().numpy()


def test_hellmann_feynman_dense_L12():
    L, n = 12, 6
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    J, Dl = synth.random_couplings(len(bonds), seed=9)
    jxy, jz = J, J * Dl
    sel = np.nonzero(full_basis_digit_sums(2, L) == n)[0]
    w, v = np.linalg.eigh(full_matrix(2, L, bonds, jxy, jz)[np.ix_(sel, sel)])
    assert w[1] - w[0] > 1e-3
    b = BruteSector(2, L, n, [6, 6])
    # the dense ground vector in the full-space numbering -> canonical order
    from oracle.sector import unpack
    full_idx = [sum(q * 2 ** (L - 1 - i) for i, q in enumerate(unpack(int(st), 2, L))) for st in b.states]
    pos = {f: k for k, f in enumerate(sel)}
    psi = v[[pos[f] for f in full_idx], 0]
    ref_gj = np.array([psi @ apply_h(b, [bd], [1.0], [0.0], psi) for bd in bonds])
    ref_gz = np.array([psi @ apply_h(b, [bd], [0.0], [1.0], psi) for bd in bonds])
    s, t = dq.Sector(L, n, 2, [6, 6]), dq.Terms(bonds)
    eig, gj, gz = hf_gradient(s, t, jxy, jz)
    assert abs(eig[0] - w[0]) < 1e-10
    assert np.allclose(gj, ref_gj, atol=1e-8) and np.allclose(gz, ref_gz, atol=1e-8)


def test_hellmann_feynman_finite_differences_L24():
    """dE0/dtheta at the L=24 random-coupling workload: Hellmann-Feynman against
    central finite differences of the Lanczos ground energy (step 1e-4)."""
    L, n, sp = 24, 12, [8, 8, 8]
    bonds = synth.chain_bonds(L, 1)
    J, Dl = synth.random_couplings(len(bonds))
    jxy, jz = J, J * Dl
    s, t = dq.Sector(L, n, 2, sp), dq.Terms(bonds)
    eig, gj, gz = hf_gradient(s, t, jxy, jz)
    assert eig[1] - eig[0] > 1e-6          # non-degenerate ground state
    eps = 1e-4
    for b in (0, 7, 19):
        e = np.zeros(len(bonds))
        e[b] = eps
        ep = hf_gradient(s, t, jxy + e, jz)[0][0]
        em = hf_gradient(s, t, jxy - e, jz)[0][0]
        fd = (ep - em) / (2 * eps)
        say("HF jxy", b, gj[b], fd)
        assert abs(fd - gj[b]) <= 1e-6 * max(1.0, abs(gj[b]))
        ep = hf_gradient(s, t, jxy, jz + e)[0][0]
        em = hf_gradient(s, t, jxy, jz - e)[0][0]
        fd = (ep - em) / (2 * eps)
        assert abs(fd - gz[b]) <= 1e-6 * max(1.0, abs(gz[b]))


@pytest.mark.parametrize("autotune", ["0", "1"])
def test_adjoint_on_split_products(monkeypatch, autotune):
    """L=26, n=13.  Autotuner off: grad_x comes from the staged split product and
    equals the product H g bit for bit.  Autotuner on: the first call times the
    fused pass against split product plus sums pass; grad_x matches H g.  Either
    way the coupling and field sums equal those of the fused single-pass adjoint
    bit for bit, and three bonds' sums match the C oracle."""
    monkeypatch.setenv("DCS_AUTOTUNE", autotune)
    L, n = 26, 13
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)[:5]
    J, Dl = synth.random_couplings(len(bonds), seed=11)
    jxy, jz = J, J * Dl
    hf = np.random.default_rng(12).normal(size=L)
    s, t = dq.Sector(L, n, 2), dq.Terms(bonds)
    ns = native.NativeSector(2, L, n, s.split)
    x = synth.vector(ns.dim, synth.SEED_X)
    g = synth.vector(ns.dim, synth.SEED_G)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        xd, gd = torch.tensor(x, device=DEV).to(dt), torch.tensor(g, device=DEV).to(dt)
        args = (s, t, dev_f64(jxy), dev_f64(jz), xd, gd)
        gx, gj, gz, gh = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
        hg = dq.hamiltonian_apply(s, t, dev_f64(jxy), dev_f64(jz), gd, h=dev_f64(hf))
        if autotune == "0":
            assert torch.equal(gx, hg)
        assert rel_err(gx.double().cpu().numpy(), hg.double().cpu().numpy()) <= tol
        again = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
        assert all(torch.equal(a, b) for a, b in zip((gx, gj, gz, gh), again))
        monkeypatch.setenv("DCS_SPLIT", "0")
        gx1, gj1, gz1, gh1 = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
        monkeypatch.delenv("DCS_SPLIT")
        say("adjoint split", dt, rel_err(gx.double().cpu().numpy(), gx1.double().cpu().numpy()))
        if dt == torch.float64:  # the same per-row sums in the same order
            assert torch.equal(gj, gj1) and torch.equal(gz, gz1) and torch.equal(gh, gh1)
        else:  # FP32: the sums may come from the split product's own gathers (other order)
            for a, b in ((gj, gj1), (gz, gz1), (gh, gh1)):
                assert rel_err(a.cpu().numpy(), b.cpu().numpy()) <= tol
        assert rel_err(gx.double().cpu().numpy(), gx1.double().cpu().numpy()) <= tol
        if dt == torch.float64:
            xs, sel = xd.cpu().numpy(), [0, 13, len(bonds) - 1]
            rj = [g @ native.hx_range(ns, native.NativeTerms([bonds[b]], [1.0], [0.0]), xs) for b in sel]
            rz = [g @ native.hx_range(ns, native.NativeTerms([bonds[b]], [0.0], [1.0]), xs) for b in sel]
            assert rel_err(gj.cpu().numpy()[sel], np.array(rj)) <= 1e-12
            assert rel_err(gz.cpu().numpy()[sel], np.array(rz)) <= 1e-12


@pytest.mark.parametrize("way", ["0", "1", "2"])
def test_adjoint_ways_L26_f32(monkeypatch, way):
    """The three ways of the FP32 adjoint on a split sector (L=26, n=13, J1-J2 bonds,
    fields): 0 the fused single pass, 1 the split product of g plus a sums pass, 2 the
    sums formed inside the split product (per-run and per-tile values reduced in a
    fixed order).  Each against the C oracle's gradient sums over every row (FP64 on
    the FP64 draws) and grad_x = H g; repeated calls are bitwise equal."""
    monkeypatch.setenv("DCS_ADJOINT_WAY", way)
    L, n = 26, 13
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 0.8)
    rng = np.random.default_rng(31)
    jxy = jxy * rng.uniform(0.5, 1.5, len(bonds))
    hf = rng.normal(size=L)
    s, t = dq.Sector(L, n, 2, [6, 7, 6, 7]), dq.Terms(bonds)  # runs of <= 1716 rows: staged
    ns = native.NativeSector(2, L, n, s.split)
    x = synth.vector(ns.dim, synth.SEED_X)
    g = synth.vector(ns.dim, synth.SEED_G)
    xd, gd = torch.tensor(x, device=DEV).float(), torch.tensor(g, device=DEV).float()
    args = (s, t, dev_f64(jxy), dev_f64(jz), xd, gd)
    gx, gj, gz, gh = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
    ref_gx = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, hf), g)
    rxy, rz, rh = native.bond_sums(ns, bonds, x, g, fields=True)
    errs = [rel_err(gx.double().cpu().numpy(), ref_gx), rel_err(gj.cpu().numpy(), rxy),
            rel_err(gz.cpu().numpy(), rz), rel_err(gh.cpu().numpy(), rh)]
    say("adjoint way", way, errs)
    assert max(errs) <= 1e-5
    again = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
    assert all(torch.equal(a, b) for a, b in zip((gx, gj, gz, gh), again))


@pytest.mark.parametrize("Q,L,n,split,k", [(2, 10, 5, [5, 5], 2), (2, 12, 6, [4, 4, 4], 8),
                                           (3, 6, 6, [2, 2, 2], 4), (2, 9, 4, [1, 2, 3, 3], 4)])
def test_block_adjoint_matches_oracle(Q, L, n, split, k):
    """The adjoint of a block of k columns: grad_X = H G and the coupling and field sums
    over rows and columns, against the C oracle's sums (FP64 and FP32)."""
    rng = np.random.default_rng(L * Q + k)
    bonds = synth.chain_bonds(L, 1) + synth.chain_bonds(L, 2)
    jxy, jz, h = rng.normal(size=len(bonds)), rng.normal(size=len(bonds)), rng.normal(size=L)
    ns = native.NativeSector(Q, L, n, split)
    x, g = rng.normal(size=(ns.dim, k)), rng.normal(size=(ns.dim, k))
    ref_gx = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, h), g)
    rxy, rz, rh = native.bond_sums(ns, bonds, x, g, fields=True)
    s, t = dq.Sector(L, n, Q, split), dq.Terms(bonds)
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        out = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz), torch.tensor(x, device=DEV).to(dt),
                                           torch.tensor(g, device=DEV).to(dt), h=dev_f64(h), want_grad_h=True)
        errs = [rel_err(out[0].double().cpu().numpy(), ref_gx), rel_err(out[1].cpu().numpy(), rxy),
                rel_err(out[2].cpu().numpy(), rz), rel_err(out[3].cpu().numpy(), rh)]
        say("block adjoint", Q, L, n, k, dt, errs)
        assert max(errs) <= tol


def test_block_adjoint_L24_k8_and_autograd():
    """k = 8 FP32 block on the L=24 workload (per-bond couplings, split view): sums
    against the oracle over every row and column, grad_X against the oracle on every
    row; and autograd through HApply on a [dim, 2] FP64 block equals the oracle's
    column sums (gradcheck on a small block)."""
    L, n, sp = 24, 12, [8, 8, 8]
    bonds = synth.chain_bonds(L, 1)
    J, Dl = synth.random_couplings(len(bonds))
    jxy, jz = J, J * Dl
    ns = native.NativeSector(2, L, n, sp)
    x = synth.vector(ns.dim, synth.SEED_X, k=8)
    g = synth.vector(ns.dim, synth.SEED_G, k=8)
    s, t = dq.Sector(L, n, 2, sp), dq.Terms(bonds)
    gx, gj, gz, _ = dq.hamiltonian_apply_adjoint(s, t, dev_f64(jxy), dev_f64(jz),
                                                 torch.tensor(x, device=DEV).float(),
                                                 torch.tensor(g, device=DEV).float())
    rxy, rz, _ = native.bond_sums(ns, bonds, x, g)
    ref_gx = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz), g)
    errs = [rel_err(gx.double().cpu().numpy(), ref_gx), rel_err(gj.cpu().numpy(), rxy),
            rel_err(gz.cpu().numpy(), rz)]
    say("block adjoint L24 k8", errs)
    assert max(errs) <= 1e-5
    # autograd on a small block
    Ls, ns_ = 8, 4
    s8 = dq.Sector(Ls, ns_, 2, [4, 4])
    b8 = synth.chain_bonds(Ls, 1) + synth.chain_bonds(Ls, 2)
    t8 = dq.Terms(b8)
    rng = np.random.default_rng(5)
    xb = torch.tensor(rng.normal(size=(s8.dim, 2)), device=DEV, requires_grad=True)
    a = torch.tensor(rng.uniform(0.5, 1.5, len(b8)), device=DEV, requires_grad=True)
    bz = torch.tensor(rng.uniform(0, 2, len(b8)), device=DEV, requires_grad=True)
    f = lambda x_, a_, b_: dq.HApply.apply(x_, a_, b_, s8, t8)
    assert torch.autograd.gradcheck(f, (xb, a, bz), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("L,n,split,k,min_dim", [(24, 12, [6, 6, 6, 6], 8, None), (24, 12, [6, 6, 6, 6], 2, None),
                                                 (22, 11, [5, 6, 5, 6], 4, "0"), (20, 8, [5, 5, 5, 5], 8, "0")])
def test_block_adjoint_ways_split(monkeypatch, L, n, split, k, min_dim):
    """Both ways of the FP32 block adjoint on a split view (J1-J2 bonds, fields):
    1 the block product of G plus a sums pass, 2 the sums formed inside the split
    block product (per-tile values folded per run, then reduced in a fixed order).
    Each against the C oracle's sums over every row and column and grad_X = H G on
    every row; repeated calls are bitwise equal, and the two ways' sums are formed
    in different orders, so they are not bitwise equal (the forced way ran)."""
    if min_dim is not None:
        monkeypatch.setenv("DCS_SPLIT_MIN_DIM", min_dim)
    bonds, jxy, jz = synth.j1j2_chain(L, 1.0, 0.5, 0.8)
    rng = np.random.default_rng(L + k)
    jxy = jxy * rng.uniform(0.5, 1.5, len(bonds))
    hf = rng.normal(size=L)
    ns = native.NativeSector(2, L, n, split)
    x = synth.vector(ns.dim, synth.SEED_X, k=k)
    g = synth.vector(ns.dim, synth.SEED_G, k=k)
    ref_gx = native.hx_range(ns, native.NativeTerms(bonds, jxy, jz, hf), g)
    rxy, rz, rh = native.bond_sums(ns, bonds, x, g, fields=True)
    xd, gd = torch.tensor(x, device=DEV).float(), torch.tensor(g, device=DEV).float()
    outs = {}
    for way in ("1", "2"):
        monkeypatch.setenv("DCS_ADJOINT_WAY", way)
        s, t = dq.Sector(L, n, 2, split), dq.Terms(bonds)
        args = (s, t, dev_f64(jxy), dev_f64(jz), xd, gd)
        out = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
        errs = [rel_err(out[0].double().cpu().numpy(), ref_gx), rel_err(out[1].cpu().numpy(), rxy),
                rel_err(out[2].cpu().numpy(), rz), rel_err(out[3].cpu().numpy(), rh)]
        say("block adjoint way", way, L, n, split, k, errs)
        assert max(errs) <= 1e-5
        again = dq.hamiltonian_apply_adjoint(*args, h=dev_f64(hf), want_grad_h=True)
        assert all(torch.equal(a, b) for a, b in zip(out, again))
        outs[way] = out
    assert not torch.equal(outs["1"][1], outs["2"][1])
