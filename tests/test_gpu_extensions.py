"""GPU parity of the extensions: photon-number penalty (Eqs. (24)-(25),
App. B), multi-state index (Eq. (22)), Gaussian control filter (App. A)."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, phi_err, grad_err, relerr, say
from oracle import extensions as ext
from oracle import rk

pytestmark = pytest.mark.gpu


def _dev():
    import torch

    return torch.device("cuda", 0)


def _t(x):
    import torch

    return torch.tensor(np.ascontiguousarray(x), device=_dev())


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("gmode", ["grape1", "exact"])
@pytest.mark.parametrize("case", ["c1", "c3shape"])
def test_penalty(prec, gmode, case):
    from paper_1609_03170_amd import Problem

    if case == "c1":
        w = wl.config_c1()
        u = w.u[:80]
        A = w.sigma
        sparse = False
    else:
        w = wl.config_c3(batch=1, n_t=16)
        u = w.u
        N = 80
        a = np.kron(np.eye(3), wl.destroy(N))
        A = a.conj().T @ a
        sparse = True
    beta = 0.35
    say(f"[case] penalty {case} prec={prec} gmode={gmode}")
    p = Problem.from_workload(w, prec=prec, gmode=gmode)
    p.set_penalty(A, beta)
    phi, g = p.cost_and_grad(_t(u), _t(w.rho0), _t(w.sigma), w.dt)
    phi, g = phi.cpu().numpy()[0], g.cpu().numpy()[0]
    p.close()
    m = rk.Model.from_workload(w, sparse=sparse)
    phi_r, rhos = ext.penalty_cost(m, u, w.rho0, w.sigma, A, beta, w.dt)
    g_r = ext.penalty_gradient(m, u, rhos, w.sigma, A, beta, w.dt, mode=gmode)
    e_phi, e_g = phi_err(phi, phi_r), grad_err(g, g_r)
    say(f"   phi {e_phi:.2e} grad {e_g:.2e}")
    assert e_phi < TOL[prec]["phi"] and e_g < TOL[prec]["grad"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_multi_state_two_contexts_and_batch(prec):
    """Qubit-conditioned resonator problems (Delta -> +-chi, QND reading of
    Sec. IV.B) in two contexts, plus a batch of input states in one."""
    from paper_1609_03170_amd import Problem

    n_t, dt = 60, 0.05
    u = wl.controls_uniform(21, n_t, 2)
    ws = [wl.resonator_problem(14, s * 1.5, 1.0, 1.0, u, dt) for s in (+1, -1)]
    vac = np.zeros((14, 14), complex)
    vac[0, 0] = 1.0
    say(f"[case] multi-state two contexts prec={prec}")
    g = None
    phi = 0.0
    for w in ws:
        p = Problem.from_workload(w, prec=prec, gmode="exact")
        p.forward(_t(u), _t(w.rho0), dt)
        phi += float(p.cost(_t(vac)).cpu()[0])
        p.adjoint(_t(vac))
        g = p.gradient_sum(g)
        g.cpu()
        p.close()
    ms = [rk.Model.from_workload(w) for w in ws]
    phi_r, g_r = ext.multi_state_cost_and_grad(ms, u, [w.rho0 for w in ws], vac, dt, mode="exact")
    e_phi, e_g = phi_err(phi, phi_r), grad_err(g.cpu().numpy(), g_r)
    say(f"   phi {e_phi:.2e} grad {e_g:.2e}")
    assert e_phi < TOL[prec]["phi"] and e_g < TOL[prec]["grad"]
    # one context, three input states (coherent amplitudes 0.5, 1, 1.5)
    w = ws[0]
    rho0s = np.stack([np.outer(k, k.conj()) for k in (wl.coherent_ket(14, a) for a in (0.5, 1.0, 1.5))])
    p = Problem.from_workload(w, prec=prec, gmode="grape1")
    p.forward(_t(np.broadcast_to(u, (3, n_t, 2))), _t(rho0s), dt)
    p.cost(_t(vac))
    p.adjoint(_t(vac))
    gs = p.gradient_sum().cpu().numpy()
    p.close()
    ref = sum(rk.cost_and_grad(ms[0], u, r0, vac, dt)[1] for r0 in rho0s)
    assert grad_err(gs, ref) < TOL[prec]["grad"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gaussian_filter_end_to_end(prec):
    import torch

    from paper_1609_03170_amd import Problem
    from paper_1609_03170_amd.api import filter_apply, filter_grad

    w = wl.config_c1()
    N, dtu, dts = 12, 0.25, 0.025
    M = int(round(N * dtu / dts))
    w0 = ext.omega0_from_bandwidth(8.0)
    u = wl.controls_uniform(4, N, 2)
    say(f"[case] filter N={N} M={M} prec={prec}")
    s = filter_apply(_t(u[None]), N, M, dtu, dts, w0)
    T = ext.transfer_matrix(N, M, dtu, dts, w0)
    s_ref = ext.filtered_controls(u, T)
    assert np.max(np.abs(s.cpu().numpy()[0] - s_ref)) < 1e-13
    p = Problem.from_workload(w, prec=prec, gmode="exact")
    phi, g_s = p.cost_and_grad(s, _t(w.rho0), _t(w.sigma), dts)
    g_u = filter_grad(g_s, N, M, dtu, dts, w0, fix_ends=True)
    torch.cuda.synchronize()
    p.close()
    m = rk.Model.from_workload(w)
    rhos = rk.forward(m, s_ref, w.rho0, dts)
    gs_ref, _ = rk.gradient_exact(m, s_ref, rhos, w.sigma, dts)
    gu_ref = ext.chain_rule(gs_ref, T, fix_ends=True)
    e = relerr(g_u.cpu().numpy()[0], gu_ref)
    say(f"   grad_u {e:.2e}")
    assert e < TOL[prec]["grad"]
    assert np.all(g_u.cpu().numpy()[0][[0, -1]] == 0.0)
