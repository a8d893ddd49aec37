"""Oracle: the lowest few eigenpairs of H and expectation values of its terms.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  FP64.

App. D computes the lowest states of an open chain in a site-dependent field
with the Lanczos iteration and reports, for each state, its energy and the
magnetisation of site 0.  Here:

  lowest_states   Lanczos with full re-orthogonalisation (lanczos.py); the
                  Ritz pairs (theta_e, psi_e = V s_e / |V s_e|) of the num
                  lowest Ritz values, s_e the eigenvector of T for theta_e.
  lowest_by_deflation
                  the same pairs without a stored basis, for sectors whose
                  Lanczos basis does not fit host memory: the e-th pair is the
                  lowest pair of H + sigma sum_{f<e} psi_f psi_f^T (Wielandt
                  deflation, sigma above the spectrum's width, so psi_f moves
                  to the top), each from a three-term Lanczos run with no
                  re-orthogonalisation (the lowest Ritz value is not disturbed
                  by the ghosts that appear above it), stopped once that value
                  has settled; its vector comes from running the identical
                  recurrence a second time and summing s_j v_j, and its energy
                  is the Rayleigh quotient psi.H psi.
  expectations    for a real state psi and each term M of H,
                  <psi|M|psi> = sum_s psi_s (M psi)_s by definition:
                  A_b = (S+_i S-_j + S-_i S+_j)/2 through apply_h on that one
                  bond, and the diagonal terms as digit-weighted sums,
                  Z_b -> sum_s psi_s^2 m_i(s) m_j(s),  Sz_i -> sum_s psi_s^2 m_i(s)
                  (m_i(s) = digit_i(s) - S).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import apply_h, spin
from .lanczos import lanczos, ritz
from .sector import nbits_for


def lowest_states(apply, v0, steps: int, num: int, dim: int | None = None):
    """(theta[:num], psi [D, num]) from a fully re-orthogonalised Lanczos run."""
    alpha, beta, V = lanczos(apply, v0, steps, dim)
    evals, evecs = ritz(alpha, beta, vectors=True)
    num = min(num, len(evals))
    psi = V @ evecs[:, :num]
    psi /= np.linalg.norm(psi, axis=0)
    return np.asarray(evals[:num]), psi


def _three_term(apply, v0, steps, coef=None, stop=None):
    """Lanczos without re-orthogonalisation for at most `steps` steps: returns
    (alpha, beta, psi).  stop(alpha, beta), if given, is asked after every step
    whether to end the run.  With coef (length >= the steps taken) psi is
    sum_j coef_j v_j; a second run with the same arguments repeats the same
    arithmetic, so its v_j equal the first run's."""
    v = v0 / np.linalg.norm(v0)
    v_prev = None
    alpha, beta = [], []
    psi = coef[0] * v if coef is not None else None
    for j in range(steps):
        w = apply(v)
        if v_prev is not None:
            w -= beta[-1] * v_prev
        a = float(v @ w)
        w -= a * v
        alpha.append(a)
        if j + 1 == steps or (stop is not None and stop(alpha, beta)):
            break
        b = float(np.linalg.norm(w))
        beta.append(b)
        v_prev, v = v, w / b
        if psi is not None:
            psi += coef[j + 1] * v
    return np.array(alpha), np.array(beta[:len(alpha) - 1]), psi


def _lowest(alpha, beta):
    if len(alpha) == 1:
        return float(alpha[0])
    return float(scipy.linalg.eigh_tridiagonal(alpha, beta, eigvals_only=True,
                                               select="i", select_range=(0, 0))[0])


def lowest_by_deflation(apply, v0, num: int, max_steps: int, tol: float = 1e-14,
                        check: int = 10, log=None):
    """[(E_e, psi_e, steps_e, residual_e)] for the num lowest eigenpairs (see the
    module docstring).  A run stops when its lowest Ritz value moved by at most
    tol * max(1, |theta|) over the last `check` steps, twice in a row."""
    v0 = np.asarray(v0, dtype=np.float64)
    found = []
    sigma = None
    for e in range(num):
        P = [p for _, p, _, _ in found]

        def apply_e(v, P=P):
            y = apply(v)
            for p in P:
                y += (sigma * float(p @ v)) * p
            return y

        seen = {"theta": None, "settled": 0}

        def stop(alpha, beta):
            if len(alpha) % check:
                return False
            theta = _lowest(np.array(alpha), np.array(beta))
            prev = seen["theta"]
            seen["theta"] = theta
            if prev is not None and abs(theta - prev) <= tol * max(1.0, abs(theta)):
                seen["settled"] += 1
            else:
                seen["settled"] = 0
            return seen["settled"] >= 2

        alpha, beta, _ = _three_term(apply_e, v0, max_steps, stop=stop)
        if sigma is None:  # width of the spectrum from the first run's extreme Ritz values
            ev = scipy.linalg.eigh_tridiagonal(alpha, beta, eigvals_only=True)
            sigma = 2.0 * (ev[-1] - ev[0]) + 1.0
        if len(alpha) == 1:
            S = np.ones((1, 1))
        else:
            _, S = scipy.linalg.eigh_tridiagonal(alpha, beta, select="i", select_range=(0, 0))
        _, _, psi = _three_term(apply_e, v0, len(alpha), coef=S[:, 0])
        psi /= np.linalg.norm(psi)
        hp = apply(psi)
        E = float(psi @ hp)
        res = float(np.linalg.norm(hp - E * psi))
        if log:
            log(f"state {e}: E = {E!r} after {len(alpha)} steps, residual {res:.3e}")
        found.append((E, psi, len(alpha), res))
    return found


def site_m(bs, i: int) -> np.ndarray:
    """m_i(s) = digit_i(s) - S for every state of the brute sector, canonical order."""
    nb = nbits_for(bs.Q)
    d = (bs.states >> np.uint64(nb * (bs.L - 1 - i))) & np.uint64((1 << nb) - 1)
    return d.astype(np.float64) - spin(bs.Q)


def expectations(bs, bonds, psi):
    """(<A_b>, <Z_b>, <Sz_i>) of a real state psi on the brute sector (not
    normalised: a state of norm r gives r^2 times the expectation)."""
    psi = np.asarray(psi, dtype=np.float64)
    m = [site_m(bs, i) for i in range(bs.L)]
    p2 = psi * psi
    exy = np.array([float(psi @ apply_h(bs, [b], [1.0], [0.0], psi)) for b in bonds])
    ez = np.array([float(p2 @ (m[i] * m[j])) for (i, j) in bonds])
    esz = np.array([float(p2 @ m[i]) for i in range(bs.L)])
    return exy, ez, esz
