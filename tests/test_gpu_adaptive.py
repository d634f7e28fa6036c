"""GPU parity of the adaptive-step path (Dormand-Prince 5(4) with step-size
control per problem, the adaptive integrator of Sec. III.A) against the
float64 oracle on the same seeded inputs: the same accepted / rejected step
counts per problem and sweep, then states, Phi and the Eq. (13) gradient to
the precision's tolerance.  Plus the invariants of the implementation
(checkpoint stride, batch position) and its argument errors.

The accept / reject decision compares a floating-point error norm with 1.
In float64 both sides compute it to ~1e-15 and take the same decisions.  In
float32 the stage derivatives carry ~6e-8 relative rounding, which enters
the norm as ~6e-8 h|L| / rtol; the float32 cases use rtol = 1e-4 so that
this stays near 1e-4 of the norm.  A decision that still flips (an error
norm within that distance of 1) is allowed once per sweep; both step
sequences are then valid adaptive solutions, and the GPU result is held to
be as close to the exact dynamics (a run of the oracle at rtol = 1e-10) as
the oracle's own result at the same tolerance."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, phi_err, grad_err, relerr, say
from oracle import adaptive as ad
from oracle import rk

pytestmark = pytest.mark.gpu


def _run(w, u, prec, rtol, atol, path="auto", ckpt_stride=0, problem=None):
    import torch

    from paper_1609_03170_amd import Problem

    dev = torch.device("cuda", 0)
    uu = np.asarray(u, dtype=np.float64)
    if uu.ndim == 2:
        uu = uu[None]
    B = uu.shape[0]
    p = problem or Problem.from_workload(w, prec=prec, path=path, gmode="grape1", ckpt_stride=ckpt_stride)
    p.set_adaptive(rtol, atol)
    ut = torch.tensor(uu, device=dev)
    r0 = torch.tensor(np.broadcast_to(w.rho0, (B, w.d, w.d)).copy(), device=dev)
    st = torch.tensor(w.sigma, device=dev)
    rhoT = p.forward(ut, r0, w.dt, want_rho_T=True)
    phi = p.cost(st)
    p.adjoint(st)
    g = p.gradient()
    torch.cuda.synchronize()
    counts = p.adaptive_stats(B)
    return phi.cpu().numpy(), g.cpu().numpy(), rhoT.cpu().numpy(), counts, p


F32_TOL = (1e-4, 1e-6)


def _check(w, u, prec, rtol, atol, path="auto", sparse=False, tag=""):
    if prec == "f32":
        rtol, atol = F32_TOL
    say(f"[case] adaptive {tag} d={w.d} N_t={np.asarray(u).shape[-2]} prec={prec} path={path} rtol={rtol}")
    phi, g, rhoT, counts, p = _run(w, u, prec, rtol, atol, path=path)
    p.close()
    uu = np.asarray(u)
    if uu.ndim == 2:
        uu = uu[None]
    m = rk.Model.from_workload(w, sparse=sparse)
    tol = TOL[prec]
    for b in range(uu.shape[0]):
        phi_r, g_r, rhos_r, (cf, cb) = ad.cost_and_grad(m, uu[b], w.rho0, w.sigma, w.dt, rtol, atol)
        ref = (cf.accepted, cf.rejected, cb.accepted, cb.rejected)
        say(f"   b={b} steps gpu {tuple(counts[b])} oracle {ref}")
        e_rho, e_phi, e_g = relerr(rhoT[b], rhos_r[-1]), phi_err(phi[b], phi_r), grad_err(g[b], g_r)
        say(f"   b={b} rho {e_rho:.2e} phi {e_phi:.2e} grad {e_g:.2e}")
        if prec == "f64" or tuple(counts[b]) == ref:
            assert tuple(counts[b]) == ref
            assert e_rho < tol["rho"] and e_phi < tol["phi"] and e_g < tol["grad"]
        else:
            assert max(abs(int(a) - int(r)) for a, r in zip(counts[b], ref)) <= 1
            phi_x, g_x, rhos_x, _ = ad.cost_and_grad(m, uu[b], w.rho0, w.sigma, w.dt, 1e-10, 1e-12)
            for mine, theirs, exact in ((rhoT[b], rhos_r[-1], rhos_x[-1]), (g[b], g_r, g_x)):
                e_me, e_or = relerr(mine, exact), relerr(theirs, exact)
                say(f"   decision flipped: distance to rtol=1e-10 gpu {e_me:.2e} oracle {e_or:.2e}")
                assert e_me <= 3.0 * e_or + 1e-5
        assert np.array_equal(rhoT[b], rhoT[b].conj().T)
    return counts


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("path", ["banded", "dense"])
def test_resonator_d10(prec, path):
    w = wl.config_c1()
    _check(w, w.u[:60], prec, 1e-7, 1e-9, path=path, tag="C1[:60]")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_long_slices_reject_and_refine(prec):
    """Slices of 0.5/kappa: the first attempt of a slice (h = dt or the
    carried proposal) is often rejected and the slice takes several steps."""
    w = wl.config_c1()
    w.dt = 0.5
    counts = _check(w, w.u[:12], prec, 1e-7, 1e-9, path="banded", tag="C1 dt=0.5")
    assert counts[0, 1] >= 1 and counts[0, 0] > 12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cqed_batch_diverging_steps(prec):
    """Two transmon x resonator problems with different controls (seeds 2, 3)
    in one batch: each keeps its own step sequence."""
    w = wl.config_c3(batch=2, n_t=8)
    w.dt = 0.05
    _check(w, w.u * 4.0, prec, 1e-6, 1e-8, path="banded", sparse=True, tag="C3-shape B=2 dt=0.05")


def test_stride_and_batch_position_bitwise():
    """The checkpoint recompute restarts from the stored controller state, so
    the stride does not change a bit; a problem alone equals itself in a
    batch."""
    w = wl.config_c1()
    w.dt = 0.25
    u = np.stack([w.u[:20], -w.u[20:40]])
    outs = []
    for s in (1, 3, 0):
        say(f"[case] adaptive ckpt_stride={s}")
        phi, g, _, counts, p = _run(w, u, "f32", 1e-6, 1e-8, path="banded", ckpt_stride=s)
        p.close()
        outs.append((phi, g, counts))
    for phi, g, counts in outs[1:]:
        assert np.array_equal(phi, outs[0][0]) and np.array_equal(g, outs[0][1])
        assert np.array_equal(counts, outs[0][2])
    phi1, g1, _, c1, p = _run(w, u[1], "f32", 1e-6, 1e-8, path="banded")
    p.close()
    assert np.array_equal(phi1[0], outs[0][0][1]) and np.array_equal(g1[0], outs[0][1][1])
    assert np.array_equal(c1[0], outs[0][2][1])


def test_argument_errors_and_switching_off():
    from paper_1609_03170_amd import OgError, Problem

    w = wl.config_c1()
    pe = Problem.from_workload(w, gmode="exact")
    with pytest.raises(OgError) as e:
        pe.set_adaptive(1e-6)
    assert e.value.name == "OG_ERR_ARG"
    pe.close()
    p = Problem.from_workload(w)
    with pytest.raises(OgError) as e:
        p.set_adaptive(-1.0)
    assert e.value.name == "OG_ERR_ARG"
    with pytest.raises(OgError) as e:
        p.adaptive_stats(1)
    assert e.value.name == "OG_ERR_ORDER"
    # on, then off again: the fixed-step results are those of a fresh context
    phi_a, _, _, _, p = _run(w, w.u[:30], "f64", 1e-8, 1e-10, problem=p)
    p.set_adaptive(0.0)
    import torch

    dev = torch.device("cuda", 0)
    u = torch.tensor(w.u[:30], device=dev)
    r0 = torch.tensor(w.rho0, device=dev)
    st = torch.tensor(w.sigma, device=dev)
    phi_f, g_f = p.cost_and_grad(u, r0, st, w.dt)
    p.close()
    phi_r, g_r, _ = rk.cost_and_grad(rk.Model.from_workload(w), w.u[:30], w.rho0, w.sigma, w.dt)
    assert phi_err(float(phi_f.cpu()[0]), phi_r) < 1e-12
    assert grad_err(g_f.cpu().numpy()[0], g_r) < 1e-10
