"""MI355X-native divide-and-conquer sector index and matrix-free H*x.

Python front of libdcs.so (C ABI in include/dcs.h).  PyTorch supplies device
memory and the current stream; every step of the computation runs in the
library's HIP kernels.  The names follow the ABI: ``sector_create`` ->
:class:`Sector`, ``rank`` / ``unrank`` / ``enumerate`` -> its methods,
``terms_create`` -> :class:`Terms`, ``hamiltonian_apply``,
``hamiltonian_apply_adjoint``, ``plan_create`` / ``plan_apply`` -> :class:`Plan`,
``lanczos``.

Method: R. Schaefer and D. J. Luitz, arXiv:2407.14591 (DanceQ).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import (DCS_F32, DCS_F64, DCS_INVALID_INDEX, DCS_REORTH_FULL, DCS_REORTH_LOCAL,
                   DCS_REORTH_NONE, DcsError, call)

__all__ = ["Sector", "Terms", "Plan", "hamiltonian_apply", "hamiltonian_apply_adjoint",
           "hamiltonian_form", "hamiltonian_apply_adjoint_noalloc",
           "HApply", "lanczos", "tridiag_eigvals", "lex_rank", "lex_unrank", "expectation_values", "DcsError", "DCS_INVALID_INDEX", "operator_expectation", "OperatorApply",
           "library_path", "Operator", "operator_apply", "local_operator", "operator_string",
           "lindbladian_terms"]


def library_path() -> str:
    _lib.lib()
    return _lib.LIB_PATH


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _dtype_code(dt) -> int:
    if dt == torch.float32:
        return DCS_F32
    if dt == torch.float64:
        return DCS_F64
    raise TypeError(f"vectors must be float32 or float64, not {dt}")


def _check_dev(t, device, name, dtype=None, shape=None, numel=None):
    """Device, contiguity, dtype and size of a tensor handed to the library; every
    pointer the C ABI receives is checked here against the extent the call reads or
    writes, so that a wrong-sized tensor raises instead of reaching a kernel."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be a CUDA tensor on device {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _block_shape(sector, x, name="x"):
    """Shape checks of a vector or a block of k columns: [dim] or [dim, k], k in {1, 2, 4, 8}."""
    if x.dim() not in (1, 2):
        raise ValueError(f"{name} must be [dim] or [dim, k], not {tuple(x.shape)}")
    if x.shape[0] != sector.dim:
        raise ValueError(f"{name} has {x.shape[0]} rows, sector dimension is {sector.dim}")
    k = 1 if x.dim() == 1 else x.shape[1]
    if k not in (1, 2, 4, 8):
        raise ValueError(f"{name} has {k} columns; k must be 1, 2, 4 or 8")
    return k


class Sector:
    """One particle-number sector with its divide-and-conquer index (dcs_sector_create).

    Q is one local dimension for every site, or a sequence of L local dimensions
    (dcs_sector_create_mixed: sites of different Q, Sec. 5); then ``Q`` holds the
    largest and ``local_dims`` the list."""

    def __init__(self, L: int, n: int, Q=2, split=None, device: int = 0):
        self._h = C.c_void_p()
        arr = None if split is None else (C.c_int * len(split))(*split)
        nsplit = 0 if split is None else len(split)
        if not hasattr(Q, "__len__"):
            call("dcs_sector_create", L, n, int(Q), nsplit, arr, device, C.byref(self._h))
        else:
            dims = [int(q) for q in Q]
            if len(dims) != L:
                raise ValueError(f"{len(dims)} local dimensions for {L} sites")
            call("dcs_sector_create_mixed", L, n, (C.c_int32 * L)(*dims), nsplit, arr, device,
                 C.byref(self._h))
        ld = (C.c_int32 * L)()
        call("dcs_sector_local_dims", self._h, ld)
        self.local_dims = [int(ld[i]) for i in range(L)]
        self.L, self.n, self.Q, self.device = L, n, max(self.local_dims), device
        d = C.c_uint64()
        call("dcs_sector_dim", self._h, C.byref(d))
        self.dim = int(d.value)
        num = C.c_int()
        sizes = (C.c_int * 64)()
        call("dcs_sector_split", self._h, C.byref(num), sizes)
        self.split = [sizes[i] for i in range(num.value)]
        gt, tb = C.c_int(), C.c_size_t()
        call("dcs_sector_tables", self._h, C.byref(gt), C.byref(tb))
        self.tables_in_device_memory = bool(gt.value)  # else staged in LDS by every kernel
        self.table_bytes = int(tb.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dcs_sector_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _counter(self, count_invalid):
        return torch.zeros(1, dtype=torch.int64, device=f"cuda:{self.device}") if count_invalid else None

    def rank(self, states: torch.Tensor, out: torch.Tensor | None = None, count_invalid=False):
        """Indices of packed states (int64/uint64 tensor); invalid -> DCS_INVALID_INDEX."""
        _check_dev(states, self.device, "states", (torch.int64, torch.uint64))
        out = torch.empty_like(states) if out is None else out
        _check_dev(out, self.device, "out", (torch.int64, torch.uint64), numel=states.numel())
        cnt = self._counter(count_invalid)
        call("dcs_rank", self._h, _ptr(states), _ptr(out), states.numel(), _ptr(cnt),
             _stream(self.device))
        return (out, cnt) if count_invalid else out

    def rank_search(self, states: torch.Tensor, out: torch.Tensor | None = None, count_invalid=False):
        """As ``rank``, with each subsystem's index found by binary search in its sorted
        list of valid words (the sorted-list container, dcs_rank_search)."""
        _check_dev(states, self.device, "states", (torch.int64, torch.uint64))
        out = torch.empty_like(states) if out is None else out
        _check_dev(out, self.device, "out", (torch.int64, torch.uint64), numel=states.numel())
        cnt = self._counter(count_invalid)
        call("dcs_rank_search", self._h, _ptr(states), _ptr(out), states.numel(), _ptr(cnt),
             _stream(self.device))
        return (out, cnt) if count_invalid else out

    def unrank(self, idx: torch.Tensor, out: torch.Tensor | None = None, count_invalid=False):
        _check_dev(idx, self.device, "idx", (torch.int64, torch.uint64))
        out = torch.empty_like(idx) if out is None else out
        _check_dev(out, self.device, "out", (torch.int64, torch.uint64), numel=idx.numel())
        cnt = self._counter(count_invalid)
        call("dcs_unrank", self._h, _ptr(idx), _ptr(out), idx.numel(), _ptr(cnt),
             _stream(self.device))
        return (out, cnt) if count_invalid else out

    def enumerate(self, first: int, count: int, out: torch.Tensor | None = None):
        if count < 0:
            raise ValueError("count must be >= 0")
        out = torch.empty(count, dtype=torch.int64, device=f"cuda:{self.device}") if out is None else out
        _check_dev(out, self.device, "out", (torch.int64, torch.uint64), numel=count)
        call("dcs_enumerate", self._h, first, count, _ptr(out), _stream(self.device))
        return out


class Terms:
    """Bond topology of an XXZ Hamiltonian (dcs_terms_create)."""

    def __init__(self, bonds):
        self.bonds = [(int(i), int(j)) for i, j in bonds]
        nb = len(self.bonds)
        si = (C.c_int32 * max(nb, 1))(*[b[0] for b in self.bonds])
        sj = (C.c_int32 * max(nb, 1))(*[b[1] for b in self.bonds])
        self._h = C.c_void_p()
        call("dcs_terms_create", nb, si, sj, C.byref(self._h))
        self.num_bonds = nb

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dcs_terms_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def local_operator(name: str, Q: int):
    """Single-site matrix on digits 0..Q-1 (spin S = (Q-1)/2, m = d - S): "Id", "Sz",
    "S+" (raises d by one, factor sqrt(S(S+1) - m(m+1))), "S-" (lowers it,
    sqrt(S(S+1) - m(m-1))), the ladder factors of the XXZ terms, or "Sx" = (S+ + S-)/2,
    "Sy" = (S+ - S-)/(2i) (complex)."""
    import numpy as np
    if name in ("Sx", "Sy"):
        sp, sm = local_operator("S+", Q), local_operator("S-", Q)
        return (sp + sm) / 2 if name == "Sx" else (sp - sm) / 2j
    S = (Q - 1) / 2.0
    M = np.zeros((Q, Q))
    for d in range(Q):
        m = d - S
        if name == "Id":
            M[d, d] = 1.0
        elif name == "Sz":
            M[d, d] = m
        elif name == "S+":
            if d + 1 < Q:
                M[d + 1, d] = np.sqrt(S * (S + 1) - m * (m + 1))
        elif name == "S-":
            if d > 0:
                M[d - 1, d] = np.sqrt(S * (S + 1) - m * (m - 1))
        else:
            raise ValueError(f"unknown local operator {name!r}")
    return M


def operator_string(coef: float, sites, names, Q):
    """The term coef * op_0(sites[0]) op_1(sites[1]) ... as (coef, sites, matrix): the
    Kronecker product of the named single-site matrices, first site most significant.
    Q is one local dimension, or the sequence of every site's (mixed dimensions)."""
    import numpy as np
    if len(sites) != len(names):
        raise ValueError("one local operator name per site")
    M = np.ones((1, 1))
    for st, nm in zip(sites, names):
        M = np.kron(M, local_operator(nm, int(Q[st]) if hasattr(Q, "__len__") else Q))
    return (float(coef), tuple(int(s) for s in sites), M)


def lindbladian_terms(L: int, hamiltonian, jumps):
    """Terms of the Lindblad superoperator (Sec. 4.1's Lindbladian operators) on the
    doubled chain of 2L sites: ket sites 0..L-1, bra sites L..2L-1, acting on
    vec(rho) with vec(rho)[(s, s')] = rho_ss' (the ket state the high digits):

        -i (H x I - I x H^T) + sum_k g_k (A_k x A_k^* - 1/2 A_k^+A_k x I - 1/2 I x (A_k^+A_k)^T)

    ``hamiltonian``: terms (coef, sites, M); ``jumps``: (g_k, (coef, sites, M)) with
    A_k = coef M.  Number-conserving H and A_k keep the ket and the bra particle
    numbers, so the doubled sector of 2n particles holds the (n, n) block of rho."""
    import numpy as np
    out = []
    for coef, sites, M in hamiltonian:
        M = np.asarray(M)
        bra = tuple(int(s) + L for s in sites)
        out.append((1.0, tuple(sites), -1j * coef * M))
        out.append((1.0, bra, 1j * coef * M.T))
    for g, (coef, sites, M) in jumps:
        A = coef * np.asarray(M, dtype=np.complex128)
        AdA = A.conj().T @ A
        bra = tuple(int(s) + L for s in sites)
        out.append((float(g), tuple(sites) + bra, np.kron(A, A.conj())))
        out.append((-0.5 * g, tuple(sites), AdA))
        out.append((-0.5 * g, bra, AdA.T))
    return out


class Operator:
    """A generic number-conserving operator (dcs_operator_create): terms (coef, sites,
    matrix) with a real or complex Q^m x Q^m matrix on the m listed sites, merged into
    clusters of at most ``cluster_sites`` sites and stored sparse on the device.  Q may
    be a sequence of L local dimensions (dcs_operator_create_mixed); a term's matrix
    then has the product of its sites' dimensions as size."""

    def __init__(self, Q, L: int, terms, cluster_sites: int = 4, device=None):
        import numpy as np
        self.L = int(L)
        mixed = hasattr(Q, "__len__")
        self.local_dims = [int(q) for q in Q] if mixed else [int(Q)] * self.L
        if len(self.local_dims) != self.L:
            raise ValueError(f"{len(self.local_dims)} local dimensions for {self.L} sites")
        self.Q = max(self.local_dims)
        self.device = torch.cuda.current_device() if device is None else int(device)
        terms = list(terms)
        cplx_in = any(np.iscomplexobj(M) for _, _, M in terms)
        nsites, sites, coefs, mats = [], [], [], []
        for coef, st, M in terms:
            st = [int(v) for v in st]
            M = np.ascontiguousarray(M, dtype=np.complex128 if cplx_in else np.float64)
            if any(v < 0 or v >= self.L for v in st):
                raise ValueError(f"term sites {st} outside [0, {self.L})")
            n = int(np.prod([self.local_dims[v] for v in st]))
            if M.shape != (n, n):
                raise ValueError(f"term on {len(st)} sites needs a {n} x {n} matrix, got {M.shape}")
            nsites.append(len(st))
            sites.extend(st)
            coefs.append(float(coef))
            mats.append(M.ravel().view(np.float64))  # complex: interleaved re, im
        nt = len(terms)
        a_ns = (C.c_int32 * max(nt, 1))(*nsites)
        a_st = (C.c_int32 * max(len(sites), 1))(*sites)
        a_cf = (C.c_double * max(nt, 1))(*coefs)
        flat = np.concatenate(mats) if mats else np.zeros(1)
        self._mats = flat  # kept alive for the call
        self._h = C.c_void_p()
        mat_p = flat.ctypes.data_as(C.POINTER(C.c_double))
        if mixed:
            dims = (C.c_int32 * self.L)(*self.local_dims)
            call("dcs_operator_create_mixed", self.L, dims, nt, a_ns, a_st, a_cf, mat_p, int(cplx_in),
                 int(cluster_sites), self.device, C.byref(self._h))
        else:
            call("dcs_operator_create", self.Q, self.L, nt, a_ns, a_st, a_cf, mat_p, int(cplx_in),
                 int(cluster_sites), self.device, C.byref(self._h))
        ncl, nnz, mx, cx = C.c_int(), C.c_uint64(), C.c_int(), C.c_int()
        call("dcs_operator_info", self._h, C.byref(ncl), C.byref(nnz), C.byref(mx), C.byref(cx))
        self.num_clusters, self.nnz, self.max_cluster_sites = ncl.value, nnz.value, mx.value
        self.is_complex = bool(cx.value)  # complex terms with real sums make a real operator
        self._spec = (list(terms), int(cluster_sites))

    def adjoint(self) -> "Operator":
        """O^+: every term (coef, sites, M) as (coef, sites, M^+) (the coefficients are
        real), built by the library like this operator (the Heisenberg-picture map of a
        Lindbladian, the transpose of a real operator)."""
        import numpy as np
        terms, cs = self._spec
        dims = self.local_dims if len(set(self.local_dims)) > 1 else self.Q
        return Operator(dims, self.L, [(c, st, np.conj(np.asarray(M)).T) for c, st, M in terms],
                        cluster_sites=cs, device=self.device)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dcs_operator_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def operator_expectation(sector: "Sector", op: Operator, x):
    """Expectation values without storing O x (dcs_operator_expectation): for real x of
    shape [dim] or [dim, k], a float64 tensor of the k sums sum_s x[s, c] (O x)[s, c];
    for complex x of shape [dim], the complex sum_s conj(x_s) (O x)_s (complex128)."""
    codes = {torch.float32: _lib.DCS_F32, torch.float64: _lib.DCS_F64, torch.complex64: _lib.DCS_C64,
             torch.complex128: _lib.DCS_C128}
    _check_dev(x, sector.device, "x", tuple(codes))
    k = _block_shape(sector, x)
    if x.is_complex() and k != 1:
        raise ValueError("complex vectors take one column")
    nb = C.c_size_t()
    call("dcs_operator_expectation_workspace_size", sector._h, op._h, k, C.byref(nb))
    ws = torch.empty(max(int(nb.value), 8), dtype=torch.uint8, device=x.device)
    out = torch.empty(2 if x.is_complex() else k, dtype=torch.float64, device=x.device)
    call("dcs_operator_expectation", sector._h, op._h, codes[x.dtype], k, _ptr(x), _ptr(out), _ptr(ws),
         ws.numel(), _stream(sector.device))
    if x.is_complex():
        return torch.complex(out[0], out[1])
    return out


def operator_apply(sector: "Sector", op: Operator, x, out=None):
    """y = O x on the sector (dcs_operator_apply): x of shape [dim] or, for float32 /
    float64, a block [dim, k] (k in 1, 2, 4, 8); complex64 / complex128 vectors of
    shape [dim] (required for a complex operator)."""
    codes = {torch.float32: _lib.DCS_F32, torch.float64: _lib.DCS_F64, torch.complex64: _lib.DCS_C64,
             torch.complex128: _lib.DCS_C128}
    _check_dev(x, sector.device, "x", tuple(codes))
    k = _block_shape(sector, x)
    if x.is_complex() and k != 1:
        raise ValueError("complex vectors take one column")
    out = torch.empty_like(x) if out is None else out
    _check_dev(out, sector.device, "out", x.dtype, shape=x.shape)
    dt = codes[x.dtype]
    call("dcs_operator_apply", sector._h, op._h, dt, k, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
         _stream(sector.device))
    return out


def _couplings(sector, terms, jxy, jz, h):
    for name, c, n in (("jxy", jxy, terms.num_bonds), ("jz", jz, terms.num_bonds)):
        _check_dev(c, sector.device, name, torch.float64)
        if c.numel() != n:
            raise ValueError(f"{name} has {c.numel()} entries, expected {n}")
    if h is not None:
        _check_dev(h, sector.device, "h", torch.float64)
        if h.numel() != sector.L:
            raise ValueError("h must hold one field per site")


def hamiltonian_apply(sector: Sector, terms: Terms, jxy, jz, x, h=None, out=None):
    """Y = H X (dcs_hamiltonian_apply); X is [dim] or [dim, k] float32/float64."""
    _couplings(sector, terms, jxy, jz, h)
    _check_dev(x, sector.device, "x", (torch.float32, torch.float64))
    k = _block_shape(sector, x)
    out = torch.empty_like(x) if out is None else out
    _check_dev(out, sector.device, "out", x.dtype, shape=x.shape)
    call("dcs_hamiltonian_apply", sector._h, terms._h, _ptr(jxy), _ptr(jz), _ptr(h),
         _dtype_code(x.dtype), k, _ptr(x), _ptr(out), _stream(sector.device))
    return out


def hamiltonian_form(sector: Sector, terms: Terms, dtype=torch.float32, k: int = 1) -> str:
    """Launch form of the product for (terms, dtype, k) on the sector (dcs_hamiltonian_form):
    "split_staged", "split_global", "split_fused", "split_tiled", "single", or "untuned"
    before the autotuner has timed that key."""
    f = C.c_int()
    call("dcs_hamiltonian_form", sector._h, terms._h, _dtype_code(dtype), k, C.byref(f))
    return _lib.FORM_NAMES[f.value]


def hamiltonian_apply_adjoint(sector: Sector, terms: Terms, jxy, jz, x, g, h=None,
                              want_grad_x=True, want_grad_h=False):
    """(H g, dL/dJxy, dL/dJz, dL/dh) for y = H x and dL/dy = g (dcs_hamiltonian_apply_adjoint);
    x and g are [dim] or [dim, k] blocks (the sums run over the columns too)."""
    _couplings(sector, terms, jxy, jz, h)
    _check_dev(x, sector.device, "x", (torch.float32, torch.float64))
    k = _block_shape(sector, x)
    _check_dev(g, sector.device, "g", x.dtype, shape=x.shape)
    dev = x.device
    gx = torch.empty_like(x) if want_grad_x else None
    gj = torch.empty(terms.num_bonds, dtype=torch.float64, device=dev)
    gz = torch.empty(terms.num_bonds, dtype=torch.float64, device=dev)
    gh = torch.empty(sector.L, dtype=torch.float64, device=dev) if want_grad_h else None
    nbytes = C.c_size_t()
    call("dcs_adjoint_workspace_size", sector._h, terms._h, k, C.byref(nbytes))
    ws = torch.empty(max(nbytes.value, 8), dtype=torch.uint8, device=dev)
    call("dcs_hamiltonian_apply_adjoint", sector._h, terms._h, _ptr(jxy), _ptr(jz), _ptr(h),
         _dtype_code(x.dtype), k, _ptr(x), _ptr(g), _ptr(gx), _ptr(gj), _ptr(gz), _ptr(gh), _ptr(ws),
         nbytes.value, _stream(sector.device))
    return gx, gj, gz, gh


def hamiltonian_apply_adjoint_noalloc(sector: Sector, terms: Terms, jxy, jz, x, g, grad_x, grad_jxy,
                                      grad_jz, h=None, grad_h=None):
    """The adjoint into caller-given outputs with no workspace
    (dcs_hamiltonian_apply_adjoint_noalloc): nothing is allocated, here or in the
    library.  grad_x may be None (coupling sums only); grad_h None skips the fields."""
    _couplings(sector, terms, jxy, jz, h)
    _check_dev(x, sector.device, "x", (torch.float32, torch.float64), shape=(sector.dim,))
    _check_dev(g, sector.device, "g", x.dtype, shape=x.shape)
    if grad_x is not None:
        _check_dev(grad_x, sector.device, "grad_x", x.dtype, shape=x.shape)
    _check_dev(grad_jxy, sector.device, "grad_jxy", torch.float64, numel=terms.num_bonds)
    _check_dev(grad_jz, sector.device, "grad_jz", torch.float64, numel=terms.num_bonds)
    if grad_h is not None:
        _check_dev(grad_h, sector.device, "grad_h", torch.float64, numel=sector.L)
    call("dcs_hamiltonian_apply_adjoint_noalloc", sector._h, terms._h, _ptr(jxy), _ptr(jz), _ptr(h),
         _dtype_code(x.dtype), _ptr(x), _ptr(g), _ptr(grad_x), _ptr(grad_jxy), _ptr(grad_jz),
         _ptr(grad_h), _stream(sector.device))
    return grad_x, grad_jxy, grad_jz, grad_h


class HApply(torch.autograd.Function):
    """y = H(jxy, jz) x with the fused hand-written backward; x is [dim] or a block [dim, k].

    backward: grad_x = H g (H is real symmetric), grad_jxy_b = g . (A_b x),
    grad_jz_b = g . (Z_b x) (dcs_hamiltonian_apply_adjoint: the sums formed inside the
    product of g, or in a pass that ranks every reached state once).
    """

    @staticmethod
    def forward(ctx, x, jxy, jz, sector, terms):
        ctx.sector, ctx.terms = sector, terms
        ctx.save_for_backward(x, jxy, jz)
        return hamiltonian_apply(sector, terms, jxy.detach().contiguous(),
                                 jz.detach().contiguous(), x.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        x, jxy, jz = ctx.saved_tensors
        gx, gj, gz, _ = hamiltonian_apply_adjoint(ctx.sector, ctx.terms, jxy.detach().contiguous(),
                                                  jz.detach().contiguous(),
                                                  x.detach().contiguous(), g.contiguous(),
                                                  want_grad_x=ctx.needs_input_grad[0])
        return gx, gj, gz, None, None


class OperatorApply(torch.autograd.Function):
    """y = O x for a generic operator (dcs_operator_apply); x is [dim], a real block
    [dim, k] or a complex vector.  backward: grad_x = O^+ g, the adjoint operator
    (Operator.adjoint, built once and kept on the operator) applied by the same kernel
    (for complex vectors this is torch's conjugate convention for a linear map)."""

    @staticmethod
    def forward(ctx, x, sector, op):
        ctx.sector, ctx.op = sector, op
        return operator_apply(sector, op, x.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        op = ctx.op
        if getattr(op, "_adjoint_op", None) is None:
            op._adjoint_op = op.adjoint()
        gx = operator_apply(ctx.sector, op._adjoint_op, g.contiguous()) if ctx.needs_input_grad[0] else None
        return gx, None, None


def lanczos(sector: Sector, terms, jxy, jz, v0, steps: int, reorth="auto",
            num_eig: int = 1, want_vector=False, h=None, hbm_fraction: float = 0.5,
            num_vec: int = 0):
    """Lanczos with FP64 scalars (dcs_lanczos; with an Operator in place of the terms,
    dcs_lanczos_operator, jxy / jz / h unused).  Returns a dict with alpha, beta,
    steps_done, eig (lowest num_eig Ritz values), reorth mode, "vector" (the ground
    Ritz vector) and "vectors" ([num_vec, D], the Ritz vectors of the num_vec lowest
    Ritz values; want_vector=True alone asks for one)."""
    is_op = isinstance(terms, Operator)
    if not is_op:
        _couplings(sector, terms, jxy, jz, h)
    _check_dev(v0, sector.device, "v0", (torch.float32, torch.float64), shape=(sector.dim,))
    if steps < 1:
        raise ValueError("steps must be >= 1")
    if num_vec < 0:
        raise ValueError("num_vec must be >= 0")
    nvec = max(num_vec, 1 if want_vector else 0)
    dtype = _dtype_code(v0.dtype)
    modes = {"none": DCS_REORTH_NONE, "local": DCS_REORTH_LOCAL, "full": DCS_REORTH_FULL}
    if reorth == "auto":
        # full re-orthogonalisation when the stored basis fits in the given share of free HBM
        free, _ = torch.cuda.mem_get_info(sector.device)
        need = C.c_size_t()
        call("dcs_lanczos_workspace_size", sector._h, dtype, steps, DCS_REORTH_FULL, nvec,
             C.byref(need))
        reorth = "full" if need.value <= hbm_fraction * free else "local"
    mode = modes[reorth]
    nbytes = C.c_size_t()
    call("dcs_lanczos_workspace_size", sector._h, dtype, steps, mode, nvec, C.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=v0.device)
    alpha = (C.c_double * steps)()
    beta = (C.c_double * steps)()
    done = C.c_int()
    ne = max(1, num_eig)
    eig = (C.c_double * ne)()
    psi = torch.zeros((nvec, sector.dim), dtype=v0.dtype, device=v0.device) if nvec else None
    if is_op:
        call("dcs_lanczos_operator", sector._h, terms._h, dtype, steps, mode, _ptr(v0), alpha, beta,
             C.byref(done), ne, eig, _ptr(psi), nvec, _ptr(ws), nbytes.value, _stream(sector.device))
    else:
        call("dcs_lanczos", sector._h, terms._h, _ptr(jxy), _ptr(jz), _ptr(h), dtype, steps, mode,
             _ptr(v0), alpha, beta, C.byref(done), ne, eig, _ptr(psi), nvec, _ptr(ws), nbytes.value,
             _stream(sector.device))
    m = done.value
    if psi is not None and m < nvec:
        psi = psi[:m]  # at most steps_done Ritz vectors exist
    return {"alpha": [alpha[i] for i in range(m)], "beta": [beta[i] for i in range(max(m - 1, 0))],
            "steps_done": m, "eig": [eig[i] for i in range(min(ne, m))], "reorth": reorth,
            "vector": psi[0] if psi is not None else None, "vectors": psi}


def expectation_values(sector: Sector, terms: Terms, psi, fields: bool = True):
    """<psi_e| term |psi_e> for every bond term and site field (dcs_expectation_values).
    psi: [D] or [num, D] device tensor (float32/float64).  Returns a dict of FP64
    tensors xy [num, B], z [num, B] and sz [num, L] (None unless fields)."""
    if psi.dim() == 1:
        psi = psi.unsqueeze(0)
    _check_dev(psi, sector.device, "psi", (torch.float32, torch.float64))
    if psi.dim() != 2 or psi.shape[1] != sector.dim:
        raise ValueError(f"psi must be [num, {sector.dim}], got {tuple(psi.shape)}")
    psi = psi.contiguous()
    num, nb = psi.shape[0], terms.num_bonds
    dev = psi.device
    exy = torch.zeros((num, nb), dtype=torch.float64, device=dev)
    ez = torch.zeros((num, nb), dtype=torch.float64, device=dev)
    esz = torch.zeros((num, sector.L), dtype=torch.float64, device=dev) if fields else None
    nbytes = C.c_size_t()
    call("dcs_expectation_workspace_size", sector._h, terms._h, C.byref(nbytes))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    call("dcs_expectation_values", sector._h, terms._h, _dtype_code(psi.dtype), num, _ptr(psi),
         _ptr(exy), _ptr(ez), _ptr(esz), _ptr(ws), nbytes.value, _stream(sector.device))
    return {"xy": exy, "z": ez, "sz": esz}


def lex_rank(L: int, n: int, states: torch.Tensor, out: torch.Tensor | None = None, count_invalid=False, Q: int = 2):
    """Ranks in the lexicographic (N = L, on-the-fly) order of the sector (dcs_lex_rank for
    Q = 2, dcs_lex_rank_q for any Q, dcs_lex_rank_mixed when Q is a list of L local
    dimensions)."""
    dev = states.device.index if states.is_cuda else 0
    _check_dev(states, dev, "states", (torch.int64, torch.uint64))
    out = torch.empty_like(states) if out is None else out
    _check_dev(out, dev, "out", (torch.int64, torch.uint64), numel=states.numel())
    cnt = torch.zeros(1, dtype=torch.int64, device=states.device) if count_invalid else None
    if hasattr(Q, "__len__"):
        if len(Q) != L:
            raise ValueError(f"{len(Q)} local dimensions for {L} sites")
        dims = (C.c_int32 * L)(*[int(q) for q in Q])
        call("dcs_lex_rank_mixed", L, n, dims, _ptr(states), _ptr(out), states.numel(), _ptr(cnt), _stream(dev))
    elif Q == 2:
        call("dcs_lex_rank", L, n, _ptr(states), _ptr(out), states.numel(), _ptr(cnt), _stream(dev))
    else:
        call("dcs_lex_rank_q", L, n, Q, _ptr(states), _ptr(out), states.numel(), _ptr(cnt), _stream(dev))
    return (out, cnt) if count_invalid else out


def lex_unrank(L: int, n: int, idx: torch.Tensor, out: torch.Tensor | None = None, count_invalid=False, Q: int = 2):
    """States at lexicographic (N = L, on-the-fly) positions of the sector (dcs_lex_unrank for
    Q = 2, dcs_lex_unrank_q for any Q, dcs_lex_unrank_mixed for a list of local dimensions)."""
    dev = idx.device.index if idx.is_cuda else 0
    _check_dev(idx, dev, "idx", (torch.int64, torch.uint64))
    out = torch.empty_like(idx) if out is None else out
    _check_dev(out, dev, "out", (torch.int64, torch.uint64), numel=idx.numel())
    cnt = torch.zeros(1, dtype=torch.int64, device=idx.device) if count_invalid else None
    if hasattr(Q, "__len__"):
        if len(Q) != L:
            raise ValueError(f"{len(Q)} local dimensions for {L} sites")
        dims = (C.c_int32 * L)(*[int(q) for q in Q])
        call("dcs_lex_unrank_mixed", L, n, dims, _ptr(idx), _ptr(out), idx.numel(), _ptr(cnt), _stream(dev))
    elif Q == 2:
        call("dcs_lex_unrank", L, n, _ptr(idx), _ptr(out), idx.numel(), _ptr(cnt), _stream(dev))
    else:
        call("dcs_lex_unrank_q", L, n, Q, _ptr(idx), _ptr(out), idx.numel(), _ptr(cnt), _stream(dev))
    return (out, cnt) if count_invalid else out


def tridiag_eigvals(alpha, beta, num: int, device: int = 0):
    m = len(alpha)
    a = (C.c_double * m)(*alpha)
    b = (C.c_double * max(m - 1, 1))(*(list(beta) or [0.0]))
    out = (C.c_double * num)()
    call("dcs_tridiag_eigvals", a, b, m, num, out, device)
    return [out[i] for i in range(num)]


class Plan:
    """Many sectors applied in one launch (dcs_plan_create / dcs_plan_apply)."""

    def __init__(self, items):
        """items: list of (Sector, Terms, jxy, jz) with jxy, jz float64 device tensors."""
        self.items = list(items)
        n = len(self.items)
        S = (C.c_void_p * n)(*[it[0]._h.value for it in self.items])
        T = (C.c_void_p * n)(*[it[1]._h.value for it in self.items])
        J = (C.c_void_p * n)(*[it[2].data_ptr() for it in self.items])
        Z = (C.c_void_p * n)(*[it[3].data_ptr() for it in self.items])
        for s, t, j, z in self.items:
            _couplings(s, t, j, z, None)
        self._h = C.c_void_p()
        call("dcs_plan_create", n, S, T, J, Z, C.byref(self._h))
        self.device = self.items[0][0].device if n else 0

    def apply(self, xs, ys=None):
        n = len(self.items)
        if len(xs) != n:
            raise ValueError("one vector per sector")
        dt = xs[0].dtype
        for (s, _, _, _), x in zip(self.items, xs):
            _check_dev(x, s.device, "x", dt)
            if x.numel() != s.dim:
                raise ValueError("vector length differs from its sector dimension")
        ys = [torch.empty_like(x) for x in xs] if ys is None else list(ys)
        if len(ys) != n:
            raise ValueError("one output vector per sector")
        for (s, _, _, _), x, y in zip(self.items, xs, ys):
            if x.dim() != 1:
                raise ValueError("plan vectors are one column per sector")
            _check_dev(y, s.device, "y", dt, shape=x.shape)
        X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        Y = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
        call("dcs_plan_apply", self._h, _dtype_code(dt), X, Y, _stream(self.device))
        return ys

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dcs_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
