"""Edge cases of the boundary: the largest dimension the library accepts
(d = 4096, banded), the largest numbers of controls and collapse operators
(K = J = 16, dense: more collapse operators than the per-operator product
split handles, so the single-product fallback runs), and empty inputs."""
import os

import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, oracle_eval, phi_err, grad_err, relerr, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_max_dimension_d4096_banded(prec):
    """A damped driven resonator truncated at N = 4096 (coherent amplitude 8),
    two slices: Phi, the gradient and sampled rows of rho_T against the
    stored oracle values (tests/golden/make_golden.py d4096); trace and exact
    Hermiticity of the whole state."""
    path = os.path.join(GOLDEN, "resonator_d4096_nt2.npz")
    if not os.path.exists(path):
        pytest.skip("resonator_d4096_nt2.npz not generated")
    gd = dict(np.load(path))
    n_t, dt = 2, 2e-4
    w = wl.resonator_problem(4096, 0.5, 1.0, 8.0, wl.controls_uniform(61, n_t, 2), dt, name="resonator4096")
    say(f"[case] d=4096 banded prec={prec} N_t={n_t}")
    phi, g, rhoT, p = gpu_eval(w, w.u, prec=prec, path="banded", gmode="grape1")
    p.close()
    tol = TOL[prec]
    rows = list(gd["rows"])
    e_phi, e_g = phi_err(phi[0], float(gd["phi"])), grad_err(g[0], gd["g_grape1"])
    e_rows = relerr(rhoT[0][rows], gd["rhoT_rows"])
    say(f"   phi {e_phi:.2e} grad {e_g:.2e} rows {e_rows:.2e}")
    assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rows < tol["rho"]
    assert abs(np.trace(rhoT[0]).real - 1.0) < (1e-12 if prec == "f64" else 1e-5)
    assert np.array_equal(rhoT[0], rhoT[0].conj().T)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("J", [8, 16])
def test_max_controls_and_collapses_dense(prec, J):
    """K = 16 controls and J = 8 (one product per collapse operator) or
    J = 16 (a single product over all of them) on the dense path."""
    w = wl.dense_random_problem(d=24, K=16, J=J, n_t=6, dt=0.002, seeds=(71, 72, 73, 74, 75, 76))
    say(f"[case] dense d=24 K=16 J={J} prec={prec}")
    for gmode in ("grape1", "exact"):
        phi, g, rhoT, p = gpu_eval(w, w.u, prec=prec, path="dense", gmode=gmode)
        p.close()
        phi_r, g_r, rho_r = oracle_eval(w, w.u, mode=gmode)
        tol = TOL[prec]
        e_phi, e_g, e_rho = phi_err(phi[0], phi_r), grad_err(g[0], g_r), relerr(rhoT[0], rho_r)
        say(f"   {gmode}: phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
        assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]


def test_empty_inputs_rejected():
    """No problems or no slices is an argument error, reported before any
    device work; the context stays usable."""
    import torch

    from paper_1609_03170_amd import Problem

    w = wl.config_c1()
    p = Problem.from_workload(w)
    dev = torch.device("cuda", 0)
    ws = torch.empty(p.workspace_bytes(1, 4), dtype=torch.uint8, device=dev)
    u = torch.tensor(w.u[:4], device=dev)
    r0 = torch.tensor(w.rho0, device=dev)
    lib, ctx = p._lib, p._ctx
    assert lib.og_forward(ctx, 0, 4, w.dt, u.data_ptr(), r0.data_ptr(), None, ws.data_ptr(), ws.numel(), None) == -1
    assert lib.og_forward(ctx, 1, 0, w.dt, u.data_ptr(), r0.data_ptr(), None, ws.data_ptr(), ws.numel(), None) == -1
    assert lib.og_workspace_bytes(ctx, 0, 4) == 0 and lib.og_workspace_bytes(ctx, 1, 0) == 0
    phi, g, _, _ = gpu_eval(w, w.u[:4], problem=p)
    p.close()
    phi_r, g_r, _ = oracle_eval(w, w.u[:4])
    assert phi_err(phi[0], phi_r) < 1e-12 and grad_err(g[0], g_r) < 1e-10
