"""og_evaluate_static: the evaluation without any device allocation by the
library (its workspace is the library's static device buffer), for callers
that cannot allocate.  Called through the C ABI and compared with the
regular entry points (og_forward, og_cost, og_adjoint, og_gradient with a
caller workspace) on the same inputs: two calls in a row, the second with a
smaller input (the buffer keeps the first call's contents), in both
precisions, on the fused banded path and the dense path; bitwise equal
(same kernels in the same order), and within the float64 oracle's
tolerance.  Sizes beyond the buffer are refused with nothing enqueued."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, grad_err, oracle_eval, phi_err, say

pytestmark = pytest.mark.gpu


def _static(p, u, rho0, sigma, dt):
    """og_evaluate_static through the C ABI on caller-allocated outputs."""
    import torch

    B, n_t = u.shape[0], u.shape[1]
    phi = torch.full((B,), float("nan"), dtype=torch.float64, device=u.device)
    g = torch.full((B, n_t, p.K), float("nan"), dtype=torch.float64, device=u.device)
    st = p._lib.og_evaluate_static(p._ctx, B, n_t, float(dt), u.data_ptr(), rho0.data_ptr(), sigma.data_ptr(),
                                   phi.data_ptr(), g.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, phi, g


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", ["banded_fused", "dense"])
def test_static_matches_regular_entry_points(case, prec):
    import torch

    from paper_1609_03170_amd import Problem

    dev = torch.device("cuda", 0)
    if case == "banded_fused":
        w = wl.config_c3(batch=3, n_t=31, N=20)
        p = Problem.from_workload(w, prec=prec, path="banded")
        assert p.fused
    else:
        w = wl.dense_random_problem(d=40, K=2, J=2, n_t=31, dt=0.005, seeds=(3, 4, 5, 6, 7, 8))
        w.u = np.stack([wl.controls_uniform(8 + b, 31, 2) for b in range(3)])
        p = Problem.from_workload(w, prec=prec, path="dense")
    sigma = torch.tensor(w.sigma, device=dev)
    # two calls in a row, the second smaller (fewer problems, fewer slices)
    for B, n_t in ((3, 31), (2, 17)):
        say(f"[case] og_evaluate_static {case} prec={prec} B={B} n_t={n_t}")
        u = torch.tensor(np.ascontiguousarray(w.u[:B, :n_t]), device=dev)
        rho0 = torch.tensor(np.broadcast_to(w.rho0, (B, w.d, w.d)).copy(), device=dev)
        assert p.workspace_bytes(B, n_t) <= 256 << 20
        st, phi_s, g_s = _static(p, u, rho0, sigma, w.dt)
        assert st == 0, p._lib.og_last_error()
        torch.cuda.synchronize()
        phi_s, g_s = phi_s.cpu().numpy(), g_s.cpu().numpy()
        phi_r, g_r = p.cost_and_grad(u, rho0, sigma, w.dt)
        torch.cuda.synchronize()
        assert np.array_equal(phi_s, phi_r.cpu().numpy()) and np.array_equal(g_s, g_r.cpu().numpy())
        po, go, _ = oracle_eval(w, w.u[B - 1, :n_t])
        e_phi, e_g = phi_err(phi_s[B - 1], po), grad_err(g_s[B - 1], go)
        say(f"   bitwise equal to the regular entry points; problem {B - 1} vs oracle: phi {e_phi:.2e} grad {e_g:.2e}")
        assert e_phi < TOL[prec]["phi"] and e_g < TOL[prec]["grad"]
    p.close()


def test_static_refuses_sizes_beyond_its_buffer():
    import torch

    from paper_1609_03170_amd import Problem

    dev = torch.device("cuda", 0)
    w = wl.config_c3(batch=1, n_t=10000)
    p = Problem.from_workload(w, prec="f64", path="banded")
    B = 4
    assert p.workspace_bytes(B, w.n_t) > 256 << 20
    u = torch.zeros((B, w.n_t, w.K), dtype=torch.float64, device=dev)
    rho0 = torch.tensor(np.broadcast_to(w.rho0, (B, w.d, w.d)).copy(), device=dev)
    sigma = torch.tensor(w.sigma, device=dev)
    say("[case] og_evaluate_static beyond its buffer")
    st, phi, g = _static(p, u, rho0, sigma, w.dt)
    torch.cuda.synchronize()
    assert st == -5 and b"static workspace" in p._lib.og_last_error()
    assert torch.isnan(phi).all()  # nothing ran
    p.close()
