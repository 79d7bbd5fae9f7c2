"""The tile task graph of the large-front factorisation, checked on the host.

The schedule (fdfd_get_table(FDFD_TABLE_TASKS)) is replayed in claim order with
the kernel's own wait rules (tile versions, update-tile completion counts).
Every wait must already be met, with exactly the awaited version, by the
tasks listed before it: then no workgroup of the persistent launch can wait
for a task that has not been claimed, and no task can read a tile that a later
task has already changed.  At the end every tile must hold every product
L_Ik D_k L_Jk^T (k < min(J, nbk)) exactly once, and every front's update tiles
must be complete.  Run for several grids, LDS budgets and Schur-complement
group sizes.
"""
from collections import defaultdict

import numpy as np
import pytest

from paper_2307_05388_amd.fdfd import FDFD_TABLE_FRONTS, FDFD_TABLE_TASKS, Plan

T = 64
ASM, DIAG, TRSM, UPD, INV, FUSED, SYRK = range(7)


def replay(tasks, fronts):
    npiv, nupd, parent = fronts[:, 1], fronts[:, 2], fronts[:, 3]
    children = defaultdict(list)
    for f, par in enumerate(parent):
        if par >= 0:
            children[int(par)].append(f)
    tiled = set(int(f) for f in tasks[:, 1])
    nb = lambda f: (-(-int(npiv[f]) // T), -(-int(nupd[f]) // T))
    state = defaultdict(int)
    done = defaultdict(int)
    applied = defaultdict(list)

    def children_done(f):
        for c in children[f]:
            if c in tiled:
                nut = nb(c)[1]
                assert done[c] == nut * (nut + 1) // 2, f"front {f} waits for child {c}"

    for n, (ty, f, k, I, J) in enumerate(tasks.tolist()):
        nbk, nut = nb(f)
        R = nbk + nut
        v = lambda i, j: state[(f, i, j)]
        where = f"task {n} {(ty, f, k, I, J)}"
        if ty == ASM:
            assert J < nbk and I >= J, where
            children_done(f)
            assert v(I, J) == 0, where
            state[(f, I, J)] = 1
        elif ty == DIAG:
            assert v(k, k) == k + 1, where
            state[(f, k, k)] = k + 2
        elif ty == TRSM:
            assert v(k, k) == k + 2 and v(I, k) == k + 1, where
            state[(f, I, k)] = k + 2
        elif ty == UPD:
            k0, k1 = k & 0xFFFF, k >> 16
            assert J < nbk and 0 <= k0 < k1 <= J <= I, where
            assert v(I, k1 - 1) == k1 + 1 and v(J, k1 - 1) == k1 + 1 and v(I, J) == k0 + 1, where
            state[(f, I, J)] = k1 + 1
            applied[(f, I, J)].extend(range(k0, k1))
        elif ty == INV:
            for i in range(k + 1, R):
                assert v(i, k) == k + 2, where
        elif ty == FUSED:
            assert v(k - 1, k - 1) == k + 1 and v(k, k - 1) == k and v(k, k) == k, where
            state[(f, k, k - 1)] = k + 1
            applied[(f, k, k)].append(k - 1)
            state[(f, k, k)] = k + 2
        elif ty == SYRK:
            k0, k1 = k & 0xFFFF, k >> 16
            assert nbk <= J <= I < R and 0 <= k0 < k1 <= nbk, where
            assert v(I, k1 - 1) == k1 + 1 and v(J, k1 - 1) == k1 + 1, where
            if k0 == 0:
                children_done(f)
                assert v(I, J) == 0, where
            else:
                assert v(I, J) == k0, where
            state[(f, I, J)] = k1
            applied[(f, I, J)].extend(range(k0, k1))
            if k1 == nbk:
                done[f] += 1
        else:
            raise AssertionError(where)
    for f in tiled:
        nbk, nut = nb(f)
        R = nbk + nut
        assert done[f] == nut * (nut + 1) // 2
        for I in range(R):
            for J in range(I + 1):
                assert sorted(applied[(f, I, J)]) == list(range(min(J, nbk))), (f, I, J)
                if J < nbk:
                    assert state[(f, I, J)] == J + 2, (f, I, J)
                else:
                    assert state[(f, I, J)] == nbk, (f, I, J)
    return len(tasks)


@pytest.mark.parametrize("nx,ny,small_lds,group", [
    (60, 60, -1, "8"), (150, 131, -1, "1"), (150, 131, -1, "2"), (150, 131, 0, "0"),
    (300, 300, 0, "8"), (300, 300, -1, "3"), (500, 500, 0, "8"), (520, 260, 0, "4"),
])
def test_schedule_replays_in_claim_order(monkeypatch, nx, ny, small_lds, group):
    monkeypatch.setenv("FDFD_SYRK_GROUP", group)
    plan = Plan(nx, ny, 10, host_only=True, small_lds=small_lds, tuned=False)
    tasks = plan.table(FDFD_TABLE_TASKS)
    fronts = plan.table(FDFD_TABLE_FRONTS).reshape(-1, 4)
    assert replay(tasks, fronts) == len(tasks) > 0
    plan.close()


def test_planted_order_mistake_is_caught():
    """The replay is not vacuous: moving a task before one it waits for fails."""
    plan = Plan(150, 131, 10, host_only=True, small_lds=-1, tuned=False)
    tasks = plan.table(FDFD_TABLE_TASKS).copy()
    fronts = plan.table(FDFD_TABLE_FRONTS).reshape(-1, 4)
    i = int(np.nonzero(tasks[:, 0] == SYRK)[0][0])
    bad = np.concatenate([tasks[i:i + 1], tasks[:i], tasks[i + 1:]])
    with pytest.raises(AssertionError):
        replay(bad, fronts)
    j = int(np.nonzero(tasks[:, 0] == UPD)[0][0])
    bad = np.delete(tasks, j, axis=0)
    with pytest.raises(AssertionError):
        replay(bad, fronts)
    plan.close()
