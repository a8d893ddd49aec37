"""The C-ABI library loads and exports every entry point include/dcs.h declares;
host-side argument checks work without a GPU.  CPU only."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcs.h")
LIB = os.path.join(ROOT, "paper_2407_14591_amd", "libdcs.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dcs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2407_14591_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ["dcs_sector_create", "dcs_sector_destroy", "dcs_sector_dim", "dcs_rank",
                 "dcs_unrank", "dcs_enumerate", "dcs_terms_create", "dcs_hamiltonian_apply",
                 "dcs_hamiltonian_apply_adjoint", "dcs_adjoint_workspace_size",
                 "dcs_plan_create", "dcs_plan_apply", "dcs_lanczos", "dcs_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(dcs_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(lib, n)


def test_binding_covers_every_entry_point():
    from paper_2407_14591_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared()


def test_host_side_errors(lib):
    from paper_2407_14591_amd import _lib
    l = _lib.lib()
    out = C.c_void_p()
    assert l.dcs_sector_create(0, 0, 2, 1, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert b"L=0" in l.dcs_last_error()
    assert l.dcs_sector_create(70, 3, 2, 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_sector_create(10, 11, 2, 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    sizes = (C.c_int * 2)(4, 5)
    assert l.dcs_sector_create(10, 5, 2, 2, sizes, 0, C.byref(out)) == _lib.DCS_EINVAL
    # the table-free lexicographic rank: argument checks before any launch
    assert l.dcs_lex_rank(0, 0, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_rank(10, 11, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_unrank(64, 32, None, None, 0, None, None) == _lib.DCS_OK  # every count below 2^64
    assert l.dcs_lex_rank(40, 20, None, None, 0, None, None) == _lib.DCS_OK  # count 0: nothing to do
    sizes = (C.c_int * 2)(3, 17)  # a 17-bit subsystem word
    assert l.dcs_sector_create(20, 5, 2, 2, sizes, 0, C.byref(out)) == _lib.DCS_EUNSUPPORTED
    sizes = (C.c_int * 2)(4, 8)  # Q = 3: an 8-site word of 16 bits (at most 1,107 words per digit sum)
    assert l.dcs_sector_create(12, 5, 3, 2, sizes, 0, C.byref(out)) != _lib.DCS_EUNSUPPORTED
    si = (C.c_int32 * 2)(0, 1)
    sj = (C.c_int32 * 2)(1, 1)
    assert l.dcs_terms_create(2, si, sj, C.byref(out)) == _lib.DCS_EINVAL
    sj = (C.c_int32 * 2)(1, 2)
    assert l.dcs_terms_create(2, si, sj, C.byref(out)) == _lib.DCS_OK
    assert l.dcs_terms_destroy(out) == _lib.DCS_OK
    assert l.dcs_terms_create(300, None, None, C.byref(out)) == _lib.DCS_EUNSUPPORTED
    assert l.dcs_version() >= 100


def test_tables_fit_the_workloads():
    """The per-subsystem word widths of every workload split stay within the
    library's on-chip table limits (checked on the host, no GPU needed)."""
    from oracle.sector import default_split
    for Q, L, split in [(2, 32, [8, 8, 8, 8]), (2, 34, [8, 8, 9, 9]), (2, 16, [8, 8]),
                        (2, 24, [8, 8, 8]), (2, 28, [7, 7, 7, 7]), (3, 16, default_split(3, 16))]:
        nb = (Q - 1).bit_length()
        assert max(split) * nb <= 14


def test_operator_host_checks(lib):
    """dcs_operator_create checks its terms before any device call (CPU): a term that
    does not conserve the particle number, repeated or out-of-range sites, too many
    sites, a bad cluster size and bad Q / L are refused with their codes."""
    from paper_2407_14591_amd import _lib
    l = _lib.lib()
    out = C.c_void_p()

    def create(Q, L, nsites, sites, coefs, mats, cluster=4):
        ns = (C.c_int32 * max(len(nsites), 1))(*nsites)
        st = (C.c_int32 * max(len(sites), 1))(*sites)
        cf = (C.c_double * max(len(coefs), 1))(*coefs)
        mt = (C.c_double * max(len(mats), 1))(*mats)
        return l.dcs_operator_create(Q, L, len(nsites), ns, st, cf, mt, 0, cluster, 0, C.byref(out))

    sp = [0, 0, 1, 0]  # S+ of spin 1/2: <1|S+|0> = 1 (does not conserve)
    assert create(2, 4, [1], [2], [1.0], sp) == _lib.DCS_EINVAL
    assert b"conserve" in l.dcs_last_error()
    hop = [0] * 16
    hop[1 * 4 + 2] = hop[2 * 4 + 1] = 1.0  # S+S- + S-S+ on two sites: conserves
    assert create(2, 4, [2], [1, 1], [1.0], hop) == _lib.DCS_EINVAL  # site listed twice
    assert create(2, 4, [2], [1, 4], [1.0], hop) == _lib.DCS_EINVAL  # site outside [0, L)
    assert create(2, 4, [2], [1, 2], [1.0], hop, cluster=0) == _lib.DCS_EINVAL
    assert create(2, 4, [2], [1, 2], [1.0], hop, cluster=9) == _lib.DCS_EINVAL
    assert create(1, 4, [2], [1, 2], [1.0], hop) == _lib.DCS_EINVAL
    assert create(2, 0, [2], [1, 2], [1.0], hop) == _lib.DCS_EINVAL
    assert create(2, 12, [9], list(range(9)), [1.0], [0.0] * (512 * 512)) == _lib.DCS_EUNSUPPORTED
    assert create(2, 4, [2], [1, 2], [float("nan")], hop) == _lib.DCS_EINVAL
    assert l.dcs_operator_info(None, None, None, None, None) == _lib.DCS_EINVAL
    assert l.dcs_operator_destroy(None) == _lib.DCS_OK


def test_mixed_and_on_the_fly_host_checks(lib):
    """The per-site-dimension and any-Q calls check their arguments before any device
    call (CPU): NULL or out-of-range local dimensions, too many bits, n out of range;
    the on-the-fly calls with count 0 need no device; a mixed operator checks the size
    of each term's matrix against its sites' dimensions."""
    from paper_2407_14591_amd import _lib
    l = _lib.lib()
    out = C.c_void_p()
    i32 = lambda v: (C.c_int32 * len(v))(*v)
    assert l.dcs_sector_create_mixed(4, 1, None, 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_sector_create_mixed(4, 1, i32([2, 1, 2, 2]), 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_sector_create_mixed(4, 1, i32([2, 17, 2, 2]), 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_sector_create_mixed(4, 7, i32([2, 3, 2, 3]), 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL  # n > 6
    assert l.dcs_sector_create_mixed(33, 1, i32([3] + [2] * 32), 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL  # 66 bits
    assert l.dcs_sector_create_mixed(0, 0, i32([2]), 0, None, 0, C.byref(out)) == _lib.DCS_EINVAL
    # on the fly: bad Q / dims / n are refused; count 0 returns at once
    assert l.dcs_lex_rank_q(8, 2, 17, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_rank_q(33, 2, 3, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_rank_q(8, 17, 3, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_unrank_q(8, 4, 3, None, None, 0, None, None) == _lib.DCS_OK
    assert l.dcs_lex_rank_mixed(4, 2, None, None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_rank_mixed(4, 7, i32([2, 3, 2, 3]), None, None, 0, None, None) == _lib.DCS_EINVAL
    assert l.dcs_lex_unrank_mixed(4, 5, i32([2, 3, 2, 3]), None, None, 0, None, None) == _lib.DCS_OK
    # a mixed operator: a term on sites of dimensions 2 and 3 needs a 6 x 6 matrix; NULL dimensions refused
    ns, st, cf = i32([2]), i32([0, 1]), (C.c_double * 1)(1.0)
    mt = (C.c_double * 36)(*([0.0] * 36))
    assert l.dcs_operator_create_mixed(4, None, 1, ns, st, cf, mt, 0, 4, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_operator_create_mixed(4, i32([2, 3, 2, 3]), 1, ns, st, cf, mt, 0, 0, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert l.dcs_operator_create_mixed(4, i32([2, 1, 2, 3]), 1, ns, st, cf, mt, 0, 4, 0, C.byref(out)) == _lib.DCS_EINVAL
    bad = [0.0] * 36
    bad[0 * 6 + 1] = 1.0  # <0,0|M|0,1>: digit sums 0 and 1
    mb = (C.c_double * 36)(*bad)
    assert l.dcs_operator_create_mixed(4, i32([2, 3, 2, 3]), 1, ns, st, cf, mb, 0, 4, 0, C.byref(out)) == _lib.DCS_EINVAL
    assert b"conserve" in l.dcs_last_error()
