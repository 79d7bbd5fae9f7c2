"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element on the same seeded inputs.

Tolerances.  complex128 factors: the field error is bounded by kappa(A) u with
u = 1.1e-16; these grids have kappa well below 1e5, so 1e-10 on the relative
field error leaves margin.  The relative residual is held to 1e-10, the bar for
the FP64 form (the solves apply explicit inverses of 64 x 64 unit-lower diagonal
blocks, which adds rounding of order cond(L_kk) u; measured ~1e-12).  complex64 factors
with FP64 refinement: refinement continues until the FP64 relative residual is
below 1e-12, which bounds the field error by about kappa * 1e-12, tested at 1e-8
here (the metric's gate is 1e-6).
"""
import numpy as np
import pytest

from paper_2307_05388_amd import problems as P
from gpu_util import entry_err, gpu_iteration, make_plan, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle(oracle, p, eps, b, c=None, g=None):
    return oracle.design_iteration(p.nx, p.ny, p.npml, P.omegas(p), eps, b, c=c, g=g)


CASES = [
    # (nx, ny, npml, leaf, small_lds)   small_lds=0 forces the blocked large-front path
    (12, 10, 3, 0, None),
    (37, 29, 6, 0, None),
    (60, 60, 10, 0, None),
    (37, 29, 6, 0, 0),
    (60, 60, 10, 16, 0),
    (150, 131, 12, 0, None),
]


@pytest.mark.parametrize("nx,ny,npml,leaf,small_lds", CASES)
def test_c128_forward_adjoint_gradient(oracle, nx, ny, npml, leaf, small_lds):
    say(f"case c128 {nx}x{ny} npml={npml} leaf={leaf} small_lds={small_lds}")
    p = P.custom_problem(nx, ny, npml)
    eps = P.design_eps(p, t=1)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, "c128", leaf=leaf, small_lds=small_lds)
    out = gpu_iteration(plan, p, eps, b, c=c)
    ref = _oracle(oracle, p, eps, b, c=c)
    assert rel(out["x"], ref["x"]) < 1e-10
    assert rel(out["lam"], ref["lam"]) < 1e-10
    assert rel(out["grad"], ref["grad"]) < 1e-9
    r = oracle.relative_residual(nx, ny, npml, P.omegas(p)[0], eps, out["x"][0, 0], b[0, 0])
    say("  rel residual", r)
    assert r < 1e-10
    assert out["info"]["status"] in (0, 6)
    plan.close()


def test_small60_full_iteration_c128(oracle):
    """60x60 grid (N = 3600): one factorisation + forward + adjoint in complex128."""
    p = P.make_problem("small60")
    eps = P.design_eps(p)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, "c128")
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=1, tol=1e-14)
    ref = _oracle(oracle, p, eps, b, c=c)
    say("60x60 rel x", rel(out["x"], ref["x"]), "grad", rel(out["grad"], ref["grad"]), out["info"])
    assert rel(out["x"], ref["x"]) < 1e-10
    assert rel(out["grad"], ref["grad"]) < 1e-9
    assert out["info"]["rel_residual_solve"] < 1e-10
    plan.close()


@pytest.mark.parametrize("nx,ny,npml,small_lds", [(37, 29, 6, None), (60, 60, 10, None), (60, 60, 10, 0),
                                                  (150, 131, 12, None)])
def test_c64_with_refinement(oracle, nx, ny, npml, small_lds):
    say(f"case c64 {nx}x{ny}")
    p = P.custom_problem(nx, ny, npml)
    eps = P.design_eps(p, t=2)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, "c64", small_lds=small_lds)
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=10, tol=1e-12)
    ref = _oracle(oracle, p, eps, b, c=c)
    info = out["info"]
    say("  rel x", rel(out["x"], ref["x"]), "steps", info["ir_steps_solve"], info["ir_steps_adjoint"],
        "res", info["rel_residual_solve"], info["rel_residual_adjoint"], "pert", info["n_perturbed"])
    assert info["status"] in (0, 6)
    assert info["rel_residual_solve"] <= 1e-12 and info["rel_residual_adjoint"] <= 1e-12
    assert rel(out["x"], ref["x"]) < 1e-8
    assert rel(out["grad"], ref["grad"]) < 1e-8
    plan.close()


def test_c64_without_refinement_is_single_precision(oracle):
    p = P.custom_problem(40, 34, 6)
    eps = P.design_eps(p)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, "c64")
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=0)
    ref = _oracle(oracle, p, eps, b, c=c)
    e = rel(out["x"], ref["x"])
    say("c64 no IR rel", e)
    assert 1e-9 < e < 1e-3
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_multi_system_multi_rhs(oracle, prec):
    """Batched wavelengths (one analysis, per-system factors) and two source
    profiles per factor, against independent oracle factorisations."""
    p = P.custom_problem(44, 38, 6, wavelengths_um=(1.50, 1.533, 1.567, 1.60),
                         src_profiles=("gauss", "alt_gauss"))
    eps = P.design_eps(p, t=3)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, prec)
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=10 if prec == "c64" else 0, tol=1e-12)
    ref = _oracle(oracle, p, eps, b, c=c)
    tol = 1e-10 if prec == "c128" else 1e-8
    for s in range(p.nsys):
        for r in range(p.nrhs):
            assert rel(out["x"][s, r], ref["x"][s, r]) < tol
            assert rel(out["lam"][s, r], ref["lam"][s, r]) < tol
        assert rel(out["grad"][s], ref["grad"][s]) < tol * 10
    plan.close()


def test_per_system_eps(oracle):
    """eps_sys_stride > 0: every system has its own permittivity map."""
    torch = torch_cuda()
    p = P.custom_problem(30, 26, 5, wavelengths_um=(1.52, 1.58))
    eps = np.stack([P.design_eps(p, t=5), P.design_eps(p, t=6)])
    b = P.sources(p)
    plan = make_plan(p, "c128")
    dev = torch.device("cuda:0")
    plan.refactor(torch.from_numpy(eps).to(dev), P.omegas(p))
    x = plan.solve(torch.from_numpy(b).to(dev)).cpu().numpy()
    for s in range(2):
        ref = oracle.design_iteration(p.nx, p.ny, p.npml, P.omegas(p)[s:s + 1], eps[s], b[s:s + 1],
                                      c=P.objective_vector(p))
        assert rel(x[s], ref["x"][0]) < 1e-10
    plan.close()


def test_reciprocity_on_gpu():
    """b_b^T A^-1 b_a = (A^-T b_b)^T b_a with the cached factor (adjoint reuse)."""
    torch = torch_cuda()
    p = P.custom_problem(48, 40, 8)
    plan = make_plan(p, "c128")
    dev = torch.device("cuda:0")
    plan.refactor(torch.from_numpy(P.design_eps(p)).to(dev), P.omegas(p))
    ba, bb = P.random_complex((2, p.N), seed=11)
    xa = plan.solve(torch.from_numpy(ba.reshape(1, 1, -1).copy()).to(dev))
    lam = torch.empty_like(xa)
    plan.adjoint_grad(xa, torch.from_numpy(bb.reshape(1, 1, -1).copy()).to(dev), lam=lam)
    lhs = bb @ xa.cpu().numpy().reshape(-1)
    rhs = lam.cpu().numpy().reshape(-1) @ ba
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    plan.close()


def test_refactor_is_deterministic():
    torch = torch_cuda()
    p = P.custom_problem(70, 64, 8)
    plan = make_plan(p, "c64")
    dev = torch.device("cuda:0")
    eps = torch.from_numpy(P.design_eps(p)).to(dev)
    b = torch.from_numpy(P.sources(p)).to(dev)
    xs = []
    for _ in range(2):
        plan.refactor(eps, P.omegas(p))
        xs.append(plan.solve(b, max_ir=2).cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
    plan.close()


def test_state_errors_on_device():
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import FDFDError, FDFD_ERR_STATE, FDFD_ERR_NOMEM, Plan
    p = P.custom_problem(20, 20, 3)
    plan = make_plan(p, "c128")
    b = torch.zeros((1, 1, p.N), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(FDFDError) as e:
        plan.solve(b)
    assert e.value.status == FDFD_ERR_STATE
    plan.close()
    with pytest.raises(FDFDError) as e:
        Plan(200, 200, 10, mem_cap_bytes=1 << 20)
    assert e.value.status == FDFD_ERR_NOMEM


@pytest.mark.parametrize("group", ["1", "2", "0"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_schur_groups_forced(oracle, monkeypatch, group, prec):
    """Every level in the tile graph, with the Schur-complement tiles
    accumulated one, two or all pivot blocks per task (FDFD_SYRK_GROUP, read at
    analysis): the grouping changes only the order of the sums."""
    monkeypatch.setenv("FDFD_SYRK_GROUP", group)
    say(f"case schur group {group} {prec} 150x131")
    p = P.custom_problem(150, 131, 12, wavelengths_um=(1.52, 1.58), src_profiles=("gauss", "alt_gauss"))
    eps = np.stack([P.design_eps(p, t=13), P.design_eps(p, t=14)])
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, prec, small_lds=0)
    ir = (10, 1e-12) if prec == "c64" else (0, 0.0)
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=ir[0], tol=ir[1])
    ref = _oracle(oracle, p, eps, b, c=c)
    bar = 1e-10 if prec == "c128" else 1e-8
    say(f"  x {rel(out['x'], ref['x']):.2e} entry {entry_err(out['x'], ref['x']):.2e} "
        f"grad {rel(out['grad'], ref['grad']):.2e}", out["info"]["status_str"])
    assert out["info"]["status"] in (0, 6)
    assert rel(out["x"], ref["x"]) < bar and rel(out["lam"], ref["lam"]) < bar
    assert entry_err(out["x"], ref["x"]) < 1e3 * bar
    assert rel(out["grad"], ref["grad"]) < 10 * bar
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("wave_levels", ["0", "1", "2", "64"])
@pytest.mark.parametrize("leaf", [16, 36])
def test_wave_fronts_all_paths(oracle, monkeypatch, prec, wave_levels, leaf):
    """The bottom levels factored one wavefront per front (k_wave_fronts: none,
    the leaves only, two levels, every level that qualifies, two rows per
    lane included) and the rest in the one-workgroup kernel: all against the
    oracle."""
    monkeypatch.setenv("FDFD_WAVE_FRONTS", wave_levels)
    # fronts of up to 128 rows qualify at this size too (two rows per lane)
    monkeypatch.setenv("FDFD_WAVE_MIN_FRONTS", "0")
    p = P.custom_problem(90, 77, 10, wavelengths_um=(1.50, 1.60), src_profiles=("gauss", "alt_gauss"))
    say(f"case wave-front levels <= {wave_levels}, leaf={leaf} {prec}")
    eps = P.design_eps(p, t=6)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, prec, leaf=leaf)
    ir = (10, 1e-12) if prec == "c64" else (0, 0.0)
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=ir[0], tol=ir[1])
    ref = _oracle(oracle, p, eps, b, c=c)
    tol = 1e-10 if prec == "c128" else 1e-8
    say(f"  x {rel(out['x'], ref['x']):.2e} lam {rel(out['lam'], ref['lam']):.2e} grad {rel(out['grad'], ref['grad']):.2e}")
    assert out["info"]["status"] in (0, 6)
    assert rel(out["x"], ref["x"]) < tol and rel(out["lam"], ref["lam"]) < tol
    assert entry_err(out["x"], ref["x"]) < 1e3 * tol
    assert rel(out["grad"], ref["grad"]) < 10 * tol
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("group", ["0", "1", "2", "4", "99"])
def test_sweep_subtree_items(oracle, monkeypatch, prec, group):
    """The bottom-level sweeps with each wavefront taking a whole subtree of
    height <= FDFD_SWEEP_GROUP (children first, parents first backwards; 0 =
    one front per item, 99 = every bottom level), with three right-hand sides
    and two systems: against the oracle."""
    monkeypatch.setenv("FDFD_SWEEP_GROUP", group)
    p = P.custom_problem(90, 77, 10, wavelengths_um=(1.50, 1.60), src_profiles=("gauss", "alt_gauss", "line"))
    say(f"case sweep subtree items of height <= {group}, {prec}")
    eps = P.design_eps(p, t=7)
    b = P.sources(p)
    c = P.objective_vector(p)
    plan = make_plan(p, prec, leaf=16, small_lds=98304)
    assert plan.query()["small_levels"] >= 3
    ir = (10, 1e-12) if prec == "c64" else (0, 0.0)
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=ir[0], tol=ir[1])
    ref = _oracle(oracle, p, eps, b, c=c)
    tol = 1e-10 if prec == "c128" else 1e-8
    say(f"  x {rel(out['x'], ref['x']):.2e} lam {rel(out['lam'], ref['lam']):.2e} grad {rel(out['grad'], ref['grad']):.2e}")
    assert out["info"]["status"] in (0, 6)
    assert rel(out["x"], ref["x"]) < tol and rel(out["lam"], ref["lam"]) < tol
    assert entry_err(out["x"], ref["x"]) < 1e3 * tol
    assert rel(out["grad"], ref["grad"]) < 10 * tol
    plan.close()
