"""The bottom levels' sweep items (host analysis, CPU): every front of the
bottom levels swept exactly once, each item's fronts children first, an item
of several fronts a whole subtree (its last front the root), every item after
the items holding its fronts' children, and the subtree height chosen as the
highest level up to 3 that still has 16 fronts per CU (4096 on 256 CUs)."""
import numpy as np
import pytest

from paper_2307_05388_amd import problems as P
from paper_2307_05388_amd.fdfd import FDFD_TABLE_FRONTS, FDFD_TABLE_SWEEP_ITEMS, Plan


def _heights(parent):
    h = np.zeros(len(parent), int)
    for f in range(len(parent)):          # fronts are numbered children first
        if parent[f] >= 0:
            h[parent[f]] = max(h[parent[f]], h[f] + 1)
    return h


def _check(plan):
    info = plan.query()
    lw = info["small_levels"]
    F = plan.table(FDFD_TABLE_FRONTS).reshape(-1, 4)
    parent = F[:, 3]
    h = _heights(parent)
    H, ptr, seq = plan.table(FDFD_TABLE_SWEEP_ITEMS)
    wave = np.flatnonzero(h < lw)
    # every bottom-level front exactly once
    assert sorted(seq.tolist()) == sorted(wave.tolist())
    item_of = np.full(len(F), -1)
    pos = np.full(len(F), -1)
    for i in range(len(ptr) - 1):
        fr = seq[ptr[i]:ptr[i + 1]]
        assert len(fr) >= 1
        item_of[fr] = i
        pos[fr] = np.arange(len(fr))
        if len(fr) > 1:
            # a whole subtree of height <= H, its root last, every other
            # front's parent in the same item
            root = fr[-1]
            assert h[root] <= H
            assert parent[root] < 0 or h[parent[root]] > H
            assert np.all(np.isin(parent[fr[:-1]], fr))
        else:
            f = fr[0]
            assert h[f] > H or parent[f] < 0 or h[parent[f]] > H
    # every child of an item's front is in that item (earlier) or an earlier item
    c = np.flatnonzero((parent >= 0) & (h < lw))
    c = c[h[parent[c]] < lw]
    pf = parent[c]
    assert np.all((item_of[c] < item_of[pf]) | ((item_of[c] == item_of[pf]) & (pos[c] < pos[pf])))
    return H, lw, h


@pytest.mark.parametrize("nx,ny,npml,leaf,small_lds", [(90, 77, 10, 16, 98304), (150, 131, 12, 0, 0),
                                                       (300, 300, 20, 16, 32768), (500, 500, 20, 25, 32768)])
def test_sweep_items_cover_and_order(nx, ny, npml, leaf, small_lds):
    p = P.custom_problem(nx, ny, npml)
    plan = Plan(p.nx, p.ny, p.npml, nsys=1, max_rhs=1, prec="c128", host_only=True, leaf=leaf, small_lds=small_lds)
    H, lw, h = _check(plan)
    counts = np.bincount(h)
    expect = max([0] + [l for l in range(1, min(3, lw - 1) + 1) if counts[l] >= 16 * 256])
    assert H == expect


@pytest.mark.parametrize("group", ["0", "1", "2", "5"])
def test_sweep_items_forced_height(monkeypatch, group):
    monkeypatch.setenv("FDFD_SWEEP_GROUP", group)
    p = P.custom_problem(150, 131, 12)
    plan = Plan(p.nx, p.ny, p.npml, nsys=1, max_rhs=1, prec="c128", host_only=True, leaf=16, small_lds=98304)
    H, lw, _ = _check(plan)
    assert H == min(int(group), lw - 1)


def test_sweep_items_large2000():
    """2000 x 2000, the benchmark's layout: subtrees of height 3 (16384 level-3
    fronts), 16384 subtree items of 15 fronts each, then levels 4-6 one front
    per item."""
    p = P.make_problem("large2000")
    plan = Plan(p.nx, p.ny, p.npml, nsys=1, max_rhs=1, prec="c128", host_only=True, leaf=25, small_lds=131072)
    H, lw, h = _check(plan)
    assert H == 3 and lw == 7
    _, ptr, _ = plan.table(FDFD_TABLE_SWEEP_ITEMS)
    sizes = np.diff(ptr)
    assert (sizes == 15).sum() == 16384 and (sizes == 1).sum() == 8192 + 4096 + 2048
