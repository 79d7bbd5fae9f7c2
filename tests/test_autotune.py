"""The autotuner's table and lookup (CPU).  The timing itself runs on the GPU
(tests/test_gpu_workloads.py uses the tuned layouts through Plan's default)."""
import json

from paper_2307_05388_amd import autotune
from paper_2307_05388_amd import problems as P


def test_committed_table_covers_standard_workloads():
    table = json.load(open(autotune.TABLE))
    for name in ("plain300", "diff500", "mux400"):
        p = P.make_problem(name)
        for prec in ("c128", "c64"):
            e = table[autotune.key(p.nx, p.ny, p.npml, p.nsys, p.nrhs, prec)]
            assert e["leaf"] >= 4 and e["small_lds"] >= -1
            # the choice is the fastest row the tuner measured
            ok = [r for r in e["table"] if r["status"] in ("ok", "pivots perturbed")]
            assert min(r["ms"] for r in ok) == e["ms"]
            assert any(r["leaf"] == e["leaf"] and r["small_lds"] == e["small_lds"] for r in ok)


def test_lookup(tmp_path):
    path = tmp_path / "t.json"
    k = autotune.key(10, 12, 2, 1, 1, "c128")
    path.write_text(json.dumps({k: {"leaf": 25, "small_lds": 32768, "ms": 1.0, "table": []}}))
    assert autotune.lookup(10, 12, 2, 1, 1, "c128", path=str(path)) == (25, 32768)
    assert autotune.lookup(10, 12, 2, 1, 1, "c64", path=str(path)) is None
    assert autotune.lookup(10, 12, 2, 1, 1, "c128", path=str(tmp_path / "missing.json")) is None
