"""CPU tests of the library's host side: the cached symbolic analysis against
brute-force elimination, the C-ABI symbol table and its argument/state errors.
No GPU is touched (host-only plans)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_05388_amd import fdfd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(F.LIB_PATH):
        from paper_2307_05388_amd import build
        build.build()
    return F.load_library()


def test_library_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "fdfd.h")).read()
    declared = set(re.findall(r"\b(fdfd_[a-z_]+)\s*\(", hdr))
    assert declared == set(F.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def _brute_columns(nx, ny, perm):
    """Boolean Gaussian elimination of the 5-point pattern in the given order:
    struct(L[:, q]) for every elimination position q."""
    N = nx * ny
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    adj = [set() for _ in range(N)]
    for n in range(N):
        i, j = n % nx, n // nx
        for t, ok in ((n - 1, i > 0), (n + 1, i < nx - 1), (n - nx, j > 0), (n + nx, j < ny - 1)):
            if ok:
                adj[iperm[n]].add(int(iperm[t]))
    cols = []
    for q in range(N):
        s = {t for t in adj[q] if t > q}
        cols.append(s)
        for a in s:
            adj[a] |= s - {a}
    return cols


@pytest.mark.parametrize("nx,ny,leaf", [(9, 7, 4), (12, 12, 8), (16, 11, 6), (13, 16, 36), (5, 23, 4), (3, 3, 4)])
def test_analysis_matches_brute_force_elimination(lib, nx, ny, leaf):
    P = F.Plan(nx, ny, 1, host_only=True, leaf=leaf)
    perm = P.table(F.FDFD_TABLE_PERM)
    fr = P.table(F.FDFD_TABLE_FRONTS).reshape(-1, 4)
    up = P.table(F.FDFD_TABLE_UPDATE)
    N = nx * ny
    assert np.array_equal(np.sort(perm), np.arange(N))
    # pivot ranges partition [0, N) in postorder
    assert fr[0, 0] == 0 and np.all(fr[1:, 0] == fr[:-1, 0] + fr[:-1, 1])
    assert fr[-1, 0] + fr[-1, 1] == N and fr[-1, 3] == -1
    assert np.all((fr[:-1, 3] > np.arange(len(fr) - 1)))
    cols = _brute_columns(nx, ny, perm)
    off = 0
    for f, (pb, p, u, par) in enumerate(fr):
        U = up[off:off + u]
        off += u
        assert np.all(np.diff(U) > 0) and (u == 0 or U[0] >= pb + p)
        # exact update set: every fill row below the front, and nothing else
        union = set()
        for q in range(pb, pb + p):
            union |= {t for t in cols[q] if t >= pb + p}
        assert union == set(U.tolist())
        # every true column structure lies inside the dense front structure
        dense_tail = set(U.tolist())
        for q in range(pb, pb + p):
            assert cols[q] <= set(range(q + 1, pb + p)) | dense_tail
        # elimination-tree parent of the front's last pivot is in the parent front
        last = pb + p - 1
        if cols[last]:
            e_par = min(cols[last])
            ppb, pp = fr[par, 0], fr[par, 1]
            assert ppb <= e_par < ppb + pp
        # children's update rows all appear in this front
    for f, (pb, p, u, par) in enumerate(fr):
        if par < 0:
            continue
        s_child = set(up[fr[:f, 2].sum():fr[:f, 2].sum() + u].tolist())
        ppb, pp, pu = fr[par, 0], fr[par, 1], fr[par, 2]
        poff = fr[:par, 2].sum()
        s_par = set(range(ppb, ppb + pp)) | set(up[poff:poff + pu].tolist())
        assert s_child <= s_par
    info = P.query()
    nnz_front = int(sum(p * (p + 1) // 2 + u * p for _, p, u, _ in fr))
    assert info["nnz_factor"] == nnz_front
    assert nnz_front >= sum(len(c) + 1 for c in cols)


def test_analysis_statistics_match_estimator(lib):
    """The 300 x 300 grid with 64-cell leaves reproduces the nested-dissection estimate:
    3373 fronts, 12 levels, nnz(L) = 5.78e6, 2.57e9 refactor flops."""
    P = F.Plan(300, 300, 20, host_only=True, leaf=64)
    info = P.query()
    assert info["nfronts"] == 3373 and info["nlevels"] == 12
    assert abs(info["nnz_factor"] - 5.78e6) / 5.78e6 < 0.01
    assert abs(info["refactor_flops"] - 2.57e9) / 2.57e9 < 0.01
    assert info["max_front"] == 450 and info["max_pivots"] == 300


def test_analyze_reports_its_phase_times(lib):
    """fdfd_analyze times its two phases itself (symbolic analysis, then the
    rest), which the caching comparison reports as SF and set-up; the info
    struct's layout ends with them after an explicit pad."""
    assert ctypes.sizeof(F.Info) == 192 and F.Info.analyze_ms.offset == 176
    P = F.Plan(300, 300, 20, host_only=True, leaf=64)
    info = P.query()
    assert info["analyze_ms"] > 0.0 and info["setup_ms"] >= 0.0 and info["reserved3"] == 0


def test_nested_dissection_separators_are_grid_lines(lib):
    """Top separator of an nx x ny grid (nx >= ny) is the middle column."""
    nx, ny = 20, 14
    P = F.Plan(nx, ny, 2, host_only=True)
    perm = P.table(F.FDFD_TABLE_PERM)
    fr = P.table(F.FDFD_TABLE_FRONTS).reshape(-1, 4)
    root = fr[-1]
    nodes = perm[root[0]:root[0] + root[1]]
    assert root[1] == ny and np.all(nodes % nx == nx // 2)
    assert np.array_equal(nodes // nx, np.arange(ny))


def _desc(**kw):
    d = dict(nx=10, ny=10, npml_x=2, npml_y=2, nsys=1, max_rhs=1, prec=0, device=-1, leaf=0,
             flags=F.FDFD_ANALYZE_HOST_ONLY, mem_cap_bytes=0)
    d.update(kw)
    return F.Desc(**d)


@pytest.mark.parametrize("bad", [dict(nx=1), dict(ny=0), dict(npml_x=5), dict(npml_y=-1), dict(nsys=0),
                                 dict(nsys=65), dict(max_rhs=0), dict(prec=7), dict(leaf=-2),
                                 dict(mem_cap_bytes=-1), dict(flags=F.FDFD_ANALYZE_HOST_ONLY | 64),
                                 dict(flags=F.FDFD_ANALYZE_HOST_ONLY | F.FDFD_GRAPH | F.FDFD_PROFILE),
                                 dict(small_lds=-2), dict(reserved=1)])
def test_analyze_rejects_bad_descriptors(lib, bad):
    h = ctypes.c_void_p(123)
    st = lib.fdfd_analyze(ctypes.byref(_desc(**bad)), ctypes.byref(h))
    assert st == F.FDFD_ERR_ARG
    assert not h.value
    assert lib.fdfd_last_error(None).decode()


def test_null_arguments_and_state_errors(lib):
    h = ctypes.c_void_p()
    assert lib.fdfd_analyze(None, ctypes.byref(h)) == F.FDFD_ERR_ARG
    assert lib.fdfd_analyze(ctypes.byref(_desc()), None) == F.FDFD_ERR_ARG
    assert lib.fdfd_analyze(ctypes.byref(_desc()), ctypes.byref(h)) == F.FDFD_OK
    om = (ctypes.c_double * 1)(0.2)
    dummy = ctypes.c_void_p(0x1000)
    # host-only plans cannot factor or solve
    assert lib.fdfd_refactor(h, dummy, 0, om, None) == F.FDFD_ERR_STATE
    assert lib.fdfd_solve(h, dummy, dummy, 1, 0, 0.0, None) == F.FDFD_ERR_STATE
    assert lib.fdfd_adjoint_grad(h, dummy, dummy, 1, 0, 0.0, None, dummy, 0, None) == F.FDFD_ERR_STATE
    assert lib.fdfd_refactor(None, dummy, 0, om, None) == F.FDFD_ERR_ARG
    assert lib.fdfd_solve(None, dummy, dummy, 1, 0, 0.0, None) == F.FDFD_ERR_ARG
    info = F.Info()
    assert lib.fdfd_query(h, ctypes.byref(info)) == F.FDFD_OK
    assert info.n == 100 and info.nfronts > 1
    assert lib.fdfd_query(None, ctypes.byref(info)) == F.FDFD_ERR_ARG
    buf = (ctypes.c_int32 * 10)()
    assert lib.fdfd_get_table(h, F.FDFD_TABLE_PERM, buf, 10) == F.FDFD_ERR_ARG
    assert lib.fdfd_get_table(h, 9, buf, 10) == F.FDFD_ERR_ARG
    lib.fdfd_destroy(h)
    lib.fdfd_destroy(None)


def test_status_strings(lib):
    for code in range(7):
        assert lib.fdfd_status_str(code).decode()
    assert lib.fdfd_status_str(99).decode() == "unknown status"
