"""The adjoint sweep as a torch.autograd.Function: gradients against the
oracle, torch.autograd.gradcheck, and central finite differences of the GPU
cost itself at the d = 240 configuration (sampled components)."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import relerr, say
from oracle import rk

pytestmark = pytest.mark.gpu


def _dev():
    import torch

    return torch.device("cuda", 0)


def test_autograd_matches_oracle_exact():
    import torch

    from paper_1609_03170_amd import Problem, open_grape_cost

    w = wl.config_c1()
    u_np = w.u[:50]
    say("[case] autograd C1[:50] f64 exact")
    p = Problem.from_workload(w, prec="f64", gmode="exact")
    u = torch.tensor(u_np, device=_dev(), requires_grad=True)
    rho0 = torch.tensor(w.rho0, device=_dev())
    sigma = torch.tensor(w.sigma, device=_dev())
    phi = open_grape_cost(u, p, rho0, sigma, w.dt)
    (3.0 * phi).backward()
    m = rk.Model.from_workload(w)
    rhos = rk.forward(m, u_np, w.rho0, w.dt)
    g_ref, _ = rk.gradient_exact(m, u_np, rhos, w.sigma, w.dt)
    assert abs(phi.item() - rk.cost(w.sigma, rhos[-1])) < 1e-12
    assert relerr(u.grad.cpu().numpy(), 3.0 * g_ref) < 1e-10
    p.close()


def test_autograd_batched_grad_output():
    import torch

    from paper_1609_03170_amd import Problem, open_grape_cost

    w = wl.config_c3(batch=3, n_t=12)
    say("[case] autograd C3-shape B=3 f32 exact, weighted sum")
    p = Problem.from_workload(w, prec="f32", gmode="exact")
    u = torch.tensor(w.u, device=_dev(), requires_grad=True)
    rho0 = torch.tensor(w.rho0, device=_dev())
    sigma = torch.tensor(w.sigma, device=_dev())
    phi = open_grape_cost(u, p, rho0, sigma, w.dt)
    wts = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=_dev())
    (phi * wts).sum().backward()
    m = rk.Model.from_workload(w, sparse=True)
    for b in range(3):
        rhos = rk.forward(m, w.u[b], w.rho0, w.dt)
        g_ref, _ = rk.gradient_exact(m, w.u[b], rhos, w.sigma, w.dt)
        assert relerr(u.grad[b].cpu().numpy(), float(wts[b]) * g_ref) < 1e-5
    p.close()


def test_gradcheck_tiny():
    import torch

    from paper_1609_03170_amd import Problem, open_grape_cost

    w = wl.resonator_problem(4, 0.5, 1.0, 0.7, wl.controls_uniform(60, 6, 2), 0.1)
    say("[case] gradcheck d=4 N_t=6 f64 exact")
    p = Problem.from_workload(w, prec="f64", gmode="exact")
    rho0 = torch.tensor(w.rho0, device=_dev())
    sigma = torch.tensor(w.sigma, device=_dev())
    u = torch.tensor(w.u, device=_dev(), requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: open_grape_cost(x, p, rho0, sigma, w.dt), (u,),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)
    p.close()


@pytest.mark.parametrize("n_t", [200])
def test_finite_differences_d240(n_t):
    """Central differences of the GPU float64 cost against the GPU exact
    gradient, sampled components, transmon(3) x resonator(80)."""
    import torch

    from paper_1609_03170_amd import Problem

    w = wl.config_c3(batch=1, n_t=n_t)
    say(f"[case] FD d=240 N_t={n_t} f64 exact")
    p = Problem.from_workload(w, prec="f64", gmode="exact")
    rho0 = torch.tensor(w.rho0, device=_dev())
    sigma = torch.tensor(w.sigma, device=_dev())
    u = torch.tensor(w.u, device=_dev())
    phi, g = p.cost_and_grad(u, rho0, sigma, w.dt)
    g = g.cpu().numpy()[0]
    idx = [(0, 0), (7, 1), (50, 2), (123, 3), (199, 0), (199, 3)]
    s = 1e-5
    fd = []
    for j, k in idx:
        up = u.clone()
        up[j, k] += s
        dn = u.clone()
        dn[j, k] -= s
        p.forward(up, rho0, w.dt)
        fp = p.cost(sigma).item()
        p.forward(dn, rho0, w.dt)
        fm = p.cost(sigma).item()
        fd.append((fp - fm) / (2 * s))
    got = np.array([g[j, k] for j, k in idx])
    say(f"   FD {np.array(fd)}\n   AD {got}")
    assert relerr(got, np.array(fd)) < 1e-7
    p.close()


def test_two_applications_before_backward():
    """loss = f(u1) + f(u2) on one Problem: the second forward sweep replaces
    the first in the workspace; backward of the first application notices
    (og_generation) and runs its forward sweep again, so both gradients are
    the oracle's."""
    import torch

    from paper_1609_03170_amd import Problem, open_grape_cost

    w = wl.config_c1()
    u1_np, u2_np = w.u[:30], -0.5 * w.u[30:60]
    say("[case] autograd C1 f64 exact, two applications then backward")
    p = Problem.from_workload(w, prec="f64", gmode="exact")
    u1 = torch.tensor(u1_np, device=_dev(), requires_grad=True)
    u2 = torch.tensor(u2_np, device=_dev(), requires_grad=True)
    rho0 = torch.tensor(w.rho0, device=_dev())
    sigma = torch.tensor(w.sigma, device=_dev())
    loss = open_grape_cost(u1, p, rho0, sigma, w.dt) + 2.0 * open_grape_cost(u2, p, rho0, sigma, w.dt)
    loss.backward()
    m = rk.Model.from_workload(w)
    for u, u_np, wt in ((u1, u1_np, 1.0), (u2, u2_np, 2.0)):
        rhos = rk.forward(m, u_np, w.rho0, w.dt)
        g_ref, _ = rk.gradient_exact(m, u_np, rhos, w.sigma, w.dt)
        assert relerr(u.grad.cpu().numpy(), wt * g_ref) < 1e-10
    p.close()
