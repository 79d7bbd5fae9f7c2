"""The design parametrisation kernels (conic smoothing filter + tanh
projection, Sec. III / IV) against the CPU oracle, element by element, from
degenerate blocks to the full 1600 x 1600 design block; and the whole chain
theta -> filter -> projection -> FDFD solve -> |c^H x|^2 -> adjoint ->
dF/dtheta against central differences and against the oracle's composition."""
import numpy as np
import pytest

from oracle import param_oracle as po
from paper_2307_05388_amd import problems as P
from gpu_util import entry_err, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [
    # (h, w, radius, beta, eta, embed) embed: the block sits inside a larger map
    (1, 1, 3.0, 8.0, 0.5, False),
    (1, 37, 2.5, 8.0, 0.5, False),
    (20, 20, 1.5, 4.0, 0.5, False),
    (33, 47, 5.0, 16.0, 0.4, True),
    (120, 160, 8.0, 32.0, 0.5, True),
    (50, 70, 0.7, 8.0, 0.5, False),
    (1600, 1600, 5.0, 8.0, 0.5, False),
]


@pytest.mark.parametrize("h,w,radius,beta,eta,embed", CASES)
def test_param_forward_backward_match_oracle(h, w, radius, beta, eta, embed):
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import param_backward, param_desc, param_forward
    say(f"case param {h}x{w} R={radius} beta={beta} eta={eta} embed={embed}")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng([h, w, 17])
    theta = rng.uniform(0, 1, size=(h, w))
    g_blk = rng.standard_normal((h, w))
    i0, j0, nx, ny = (7, 5, w + 19, h + 11) if embed else (0, 0, w, h)
    d = param_desc(w, h, radius, beta, eta, i0=i0, j0=j0, nx=nx, ny=ny)
    eps_map = torch.full((ny, nx), -1.0, dtype=torch.float64, device=dev)
    th = torch.from_numpy(theta).to(dev)
    rho = torch.empty_like(th)
    param_forward(d, th, rho, eps_map)
    gmap = torch.zeros((ny, nx), dtype=torch.float64, device=dev)
    gmap[j0:j0 + h, i0:i0 + w] = torch.from_numpy(g_blk).to(dev)
    work, gt = torch.empty_like(th), torch.empty_like(th)
    param_backward(d, rho, gmap, work, gt)
    torch.cuda.synchronize()
    r_ref, e_ref = po.design_eps(theta, radius, beta, eta, 2.085, 12.11)
    g_ref = po.design_eps_backward(r_ref, g_blk, radius, beta, eta, 2.085, 12.11)
    em = eps_map.cpu().numpy()
    say(f"  rho {entry_err(rho.cpu().numpy(), r_ref, 0):.2e} eps {entry_err(em[j0:j0 + h, i0:i0 + w], e_ref, 0):.2e} "
        f"grad {rel(gt.cpu().numpy(), g_ref):.2e} entry {entry_err(gt.cpu().numpy(), g_ref):.2e}")
    assert entry_err(rho.cpu().numpy(), r_ref, 0) < 1e-13
    assert entry_err(em[j0:j0 + h, i0:i0 + w], e_ref, 0) < 1e-13
    assert rel(gt.cpu().numpy(), g_ref) < 1e-12 and entry_err(gt.cpu().numpy(), g_ref) < 1e-9
    if embed:   # the rest of the map is not touched
        mask = np.ones((ny, nx), bool)
        mask[j0:j0 + h, i0:i0 + w] = False
        assert np.all(em[mask] == -1.0)


def test_param_rejects_bad_arguments():
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import FDFD_ERR_ARG, FDFDError, param_desc, param_forward
    t = torch.zeros((4, 4), dtype=torch.float64, device="cuda:0")
    for d in (param_desc(4, 4, 13.0, 8.0), param_desc(4, 4, 2.0, 8.0, eta=1.0), param_desc(4, 4, 2.0, 8.0, i0=1)):
        with pytest.raises(FDFDError) as e:
            param_forward(d, t, t, t)
        assert e.value.status == FDFD_ERR_ARG


def _chain_problem():
    p = P.custom_problem(60, 60, 10)
    i0, i1, j0, j1 = p.design
    theta = np.random.default_rng([3, 21]).uniform(0, 1, size=(j1 - j0, i1 - i0))
    return p, theta, dict(radius=2.5, beta=4.0, eta=0.5, eps_min=2.085, eps_max=12.11)


def test_chain_gradient_matches_oracle_and_central_differences(oracle):
    torch = torch_cuda()
    from paper_2307_05388_amd.autograd import design_map, fdfd_fields, mode_overlap
    from paper_2307_05388_amd.fdfd import Plan
    dev = torch.device("cuda:0")
    p, theta, a = _chain_problem()
    i0, i1, j0, j1 = p.design
    om = P.omegas(p)
    base = torch.from_numpy(P.base_eps(p)).to(dev)
    b = torch.from_numpy(P.sources(p)).to(dev)
    c = torch.from_numpy(P.objective_vector(p)).to(dev)
    plan = Plan(p.nx, p.ny, p.npml, prec="c128")
    th = torch.from_numpy(theta).to(dev).requires_grad_(True)
    x = fdfd_fields(design_map(th, **a), plan, base, p.design, om, b, max_ir=2, tol=1e-14)
    F = mode_overlap(x, c)
    F.backward()
    g_gpu = th.grad.cpu().numpy()
    # the oracle's composition: parametrisation, banded-LU design iteration, chain rule
    rho, eps_blk = po.design_eps(theta, **a)
    eps = P.base_eps(p)
    eps[j0:j1, i0:i1] = eps_blk
    ref = oracle.design_iteration(p.nx, p.ny, p.npml, om, eps, P.sources(p), c=P.objective_vector(p))
    g_eps = ref["grad"][0].reshape(p.ny, p.nx)[j0:j1, i0:i1]
    g_ref = po.design_eps_backward(rho, g_eps, **a)
    say(f"chain: F {F.item():.6e} vs oracle {ref['F'].sum():.6e}; dF/dtheta vs oracle {rel(g_gpu, g_ref):.2e}")
    assert abs(F.item() - ref["F"].sum()) <= 1e-10 * abs(ref["F"].sum())
    assert rel(g_gpu, g_ref) < 1e-9

    def F_at(t):
        with torch.no_grad():
            xx = fdfd_fields(design_map(torch.from_numpy(t).to(dev), **a), plan, base, p.design, om, b,
                             max_ir=2, tol=1e-14)
            return float(mode_overlap(xx, c).item())

    h = 1e-5
    rng = np.random.default_rng([3, 22])
    fd, ad = [], []
    for _ in range(12):
        j, i = rng.integers(0, theta.shape[0]), rng.integers(0, theta.shape[1])
        tp, tm = theta.copy(), theta.copy()
        tp[j, i] += h
        tm[j, i] -= h
        fd.append((F_at(tp) - F_at(tm)) / (2 * h))
        ad.append(g_gpu[j, i])
    e = np.linalg.norm(np.array(ad) - np.array(fd)) / np.linalg.norm(fd)
    say(f"chain: dF/dtheta vs central differences {e:.2e}")
    assert e < 1e-5
    plan.close()
