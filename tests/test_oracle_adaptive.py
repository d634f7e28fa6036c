"""Pins of the adaptive-step oracle (Dormand-Prince 5(4) with step-size
control, Sec. III.A's adaptive integrator): order conditions of the
coefficient table, the fifth-order convergence of the propagated solution
against the exact propagator, accuracy at tight tolerances against the
exact propagator and the undriven closed form, the behaviour of the
controller, and the first-order gradient against its exact-propagator
counterpart.  CPU only."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import workloads as wl
from oracle import adaptive as ad
from oracle import rk, superop


def _relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def test_table_order_conditions():
    """Row sums give the nodes; the propagated weights satisfy the order
    conditions up to order 5 and the embedded weights up to order 4 (exact
    rational arithmetic), so a mistyped coefficient fails here."""
    for i in range(1, 7):
        assert sum(ad.A[i], F(0)) == ad.C[i]
    c = ad.C
    # bushy-tree conditions sum_i b_i c_i^(q-1) = 1/q
    for q in range(1, 6):
        assert sum(b * c[i] ** (q - 1) for i, b in enumerate(ad.B)) == F(1, q)
    for q in range(1, 5):
        assert sum(b * c[i] ** (q - 1) for i, b in enumerate(ad.BHAT)) == F(1, q)
    # conditions with one inner sum: sum_i b_i c_i^m sum_l a_il c_l = 1/((m+3)(m+2)) ... (m = 0, 1, 2)
    def ac(i):
        return sum((a * c[l] for l, a in enumerate(ad.A[i])), F(0)) if i < 7 else F(0)
    assert sum(b * ac(i) for i, b in enumerate(ad.B)) == F(1, 6)
    assert sum(b * c[i] * ac(i) for i, b in enumerate(ad.B)) == F(1, 8)
    assert sum(b * c[i] ** 2 * ac(i) for i, b in enumerate(ad.B)) == F(1, 10)
    # the fourth-order companion reproduces the same first three conditions
    assert sum(b * ac(i) for i, b in enumerate(ad.BHAT)) == F(1, 6)
    # first-same-as-last: the last row of A is the propagated weights
    assert ad.A[6] + [F(0)] == ad.B
    assert sum(ad.E, F(0)) == 0


def test_fifth_order_convergence_against_exact_propagator():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:1]
    H = m.hamiltonian(u[0])
    f = lambda Y: rk.lindblad(m, H, Y)  # noqa: E731
    E = superop.slice_propagators(m, u, 0.4)[0]
    exact = superop.unvec(E @ superop.vec(w.rho0), w.d)
    # halving h divides the error by 2^5 in the asymptotic range (a fourth-
    # order table would give 2^4)
    errs = [_relerr(ad.dopri_fixed(f, w.rho0, 0.4 / n, n), exact) for n in (16, 32, 64)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 28 < r1 < 38 and 28 < r2 < 38, errs


def test_tight_tolerance_matches_exact_propagation():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:40]
    rhos, ctl = ad.forward(m, u, w.rho0, w.dt, rtol=1e-11, atol=1e-13)
    ex = superop.forward(m, u, w.rho0, w.dt)
    assert _relerr(rhos[-1], ex[-1]) < 1e-9
    assert ctl.accepted >= 40


def test_undriven_photon_number_closed_form():
    """u = 0: <a^dag a>(t) = n0 exp(-kappa t) for the damped resonator,
    exactly in truncation; adaptive steps follow it to the tolerance."""
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = np.zeros((50, 2))
    rhos, _ = ad.forward(m, u, w.rho0, w.dt, rtol=1e-10, atol=1e-12)
    a = wl.destroy(w.d)
    n_op = a.conj().T @ a
    n0 = np.trace(n_op @ w.rho0).real
    for j in (10, 30, 50):
        n = np.trace(n_op @ rhos[j]).real
        assert abs(n - n0 * math.exp(-1.0 * j * w.dt)) < 1e-8 * n0


def test_controller_behaviour():
    """Looser tolerances take no more steps; a long first slice is rejected
    and refined; the trace is preserved to the tolerance."""
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:20]
    counts = []
    for rtol in (1e-4, 1e-7, 1e-10):
        rhos, ctl = ad.forward(m, u, w.rho0, 10 * w.dt, rtol=rtol, atol=1e-3 * rtol)
        counts.append(ctl.accepted)
        assert abs(np.trace(rhos[-1]).real - 1.0) < 100 * rtol
    assert counts[0] <= counts[1] <= counts[2]
    assert counts[2] > counts[0]
    # a slice far longer than the stable RK step: the first attempts are rejected
    ctl = ad.Controller(5.0, 1e-8, 1e-10)
    H = m.hamiltonian(u[0])
    ctl.slice(lambda Y: rk.lindblad(m, H, Y), w.rho0, 5.0)
    assert ctl.rejected >= 1 and ctl.accepted >= 2


def test_grape1_gradient_matches_exact_propagator_form():
    """With tight tolerances the adaptive first-order gradient (Eq. (13) on
    adaptive rho_j, lambda_j) equals Eq. (13) on exactly propagated states."""
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:30]
    phi, g, rhos, _ = ad.cost_and_grad(m, u, w.rho0, w.sigma, w.dt, rtol=1e-11, atol=1e-13)
    ex_r = superop.forward(m, u, w.rho0, w.dt)
    ex_l = superop.backward(m, u, w.sigma, w.dt)
    g_ex = rk.gradient_grape1(m, u, ex_r, ex_l, w.dt)
    assert _relerr(g, g_ex) < 1e-8
    assert abs(phi - rk.cost(w.sigma, ex_r[-1])) < 1e-9


@pytest.mark.parametrize("sparse", [False, True])
def test_cqed_shape_runs_and_is_consistent(sparse):
    """The transmon x resonator shape (small N): adaptive and fine fixed-step
    RK4 agree to the tolerance; sparse and dense operators agree."""
    w = wl.transmon_resonator_problem(3, 8, alpha=1.0, qubit_drive=True, u=wl.controls_uniform(3, 6, 4), dt=0.01)
    m = rk.Model.from_workload(w, sparse=sparse)
    phi, g, rhos, (cf, cb) = ad.cost_and_grad(m, w.u, w.rho0, w.sigma, w.dt, rtol=1e-10, atol=1e-12)
    phi_r, g_r, _ = rk.cost_and_grad(m, w.u, w.rho0, w.sigma, w.dt, n_sub=16)
    assert abs(phi - phi_r) < 1e-8 * max(1.0, abs(phi_r))
    assert _relerr(g, g_r) < 1e-6
    assert cf.accepted >= w.u.shape[0] and cb.accepted >= w.u.shape[0]
