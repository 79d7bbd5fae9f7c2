"""The inverse-design loop (Sec. III / IV) on the GPU: the objective's
gradient (port modes, filter, projection, batched FDFD over wavelengths and
input modes, normalised transmissions) against central differences, and a
short L-BFGS-B run that lowers the objective with every solve's status ok."""
import numpy as np
import pytest

from gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu


def _small():
    from paper_2307_05388_amd.optimize import MuxDevice
    return MuxDevice(nx=120, ny=100, npml=12, wavelengths_um=(1.52, 1.58), nmodes=3,
                     design=(40, 80, 25, 75))


def test_objective_gradient_matches_central_differences():
    torch_cuda()
    from paper_2307_05388_amd.optimize import MuxObjective
    dev = _small()
    obj = MuxObjective(dev, max_ir=2, tol=1e-14)
    shape = obj._shape()
    theta = np.random.default_rng([1, 32]).uniform(0.2, 0.8, size=shape).reshape(-1)
    f0, g = obj(theta)
    rng = np.random.default_rng([1, 33])
    h = 1e-5
    fd, ad = [], []
    for _ in range(8):
        k = int(rng.integers(0, theta.size))
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd.append((obj(tp)[0] - obj(tm)[0]) / (2 * h))
        ad.append(g[k])
    e = np.linalg.norm(np.array(ad) - np.array(fd)) / np.linalg.norm(fd)
    say(f"mux objective F = {f0:.6f}: gradient vs central differences {e:.2e}")
    assert e < 1e-5
    obj.close()


def test_lbfgsb_lowers_the_objective():
    torch_cuda()
    from paper_2307_05388_amd.optimize import run_lbfgsb
    r = run_lbfgsb(_small(), iters=6, callback=lambda k, f: say(f"  eval {k}: F = {f:.6f}"))
    say(f"L-BFGS-B: {r['iterations']} iterations, {r['evals']} evaluations, F {r['F'][0]:.4f} -> {min(r['F']):.4f}, "
        f"{r['seconds_in_objective'] / r['evals'] * 1e3:.1f} ms per evaluation")
    assert min(r["F"]) < 0.9 * r["F"][0]
    assert np.all(r["theta"] >= 0) and np.all(r["theta"] <= 1)
