"""Pins of the oracle's extensions: Gaussian filter transfer matrix (App. A),
photon-number penalty (Eqs. (24)-(25), App. B), multi-state index
(Eq. (22)).  CPU only."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import extensions as ext
from oracle import rk


def _relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def test_filter_bandwidth_constant():
    # the paper quotes omega_0 ~ omega_B / 0.5887
    assert abs(ext.omega0_from_bandwidth(1.0) - 1 / 0.5887) < 1e-4


def test_transfer_matrix_erf_equals_integral_form():
    T = ext.transfer_matrix(4, 18, 1.0, 0.25, 3.0)
    Ti = ext.transfer_matrix_integral(4, 18, 1.0, 0.25, 3.0)
    assert np.max(np.abs(T - Ti)) < 1e-8


def test_transfer_matrix_partition_of_unity_and_sharp_limit():
    N, M, dtu, dts = 10, 100, 1.0, 0.1
    T = ext.transfer_matrix(N, M, dtu, dts, 8.0)
    # sum over j telescopes to (erf(w0 t/2) - erf(w0 (t - N dtu)/2)) / 2, ~1 inside
    inner = T[20:80].sum(axis=1)
    assert np.max(np.abs(inner - 1.0)) < 1e-12
    # w0 -> infinity: the piecewise-constant controls themselves
    Ts = ext.transfer_matrix(N, M, dtu, dts, 1e6)
    ref = np.zeros((M, N))
    for n in range(M):
        t = n * dts
        for j in range(N):
            if j * dtu < t < (j + 1) * dtu:
                ref[n, j] = 1.0
            elif abs(t - j * dtu) < 1e-12 or abs(t - (j + 1) * dtu) < 1e-12:
                ref[n, j] = 0.5
    assert np.max(np.abs(Ts - ref)) < 1e-12


def test_filter_chain_rule_vs_finite_differences():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    N, dtu, dts = 6, 0.25, 0.05
    M = int(round(N * dtu / dts))
    T = ext.transfer_matrix(N, M, dtu, dts, 12.0)
    u = wl.controls_uniform(3, N, 2)

    def phi(uu):
        s = ext.filtered_controls(uu, T)
        return rk.cost(w.sigma, rk.forward(m, s, w.rho0, dts)[-1])

    s = ext.filtered_controls(u, T)
    g_s, _ = rk.gradient_exact(m, s, rk.forward(m, s, w.rho0, dts), w.sigma, dts)
    g_u = ext.chain_rule(g_s, T, fix_ends=False)
    eps = 1e-6
    for j, k in [(0, 0), (2, 1), (3, 0), (5, 1)]:
        up = u.copy()
        up[j, k] += eps
        dn = u.copy()
        dn[j, k] -= eps
        fd = (phi(up) - phi(dn)) / (2 * eps)
        assert abs(fd - g_u[j, k]) < 1e-7 * max(1.0, abs(fd))
    assert np.all(ext.chain_rule(g_s, T)[[0, -1]] == 0.0)


@pytest.mark.parametrize("mode", ["exact"])
def test_penalty_gradient_vs_finite_differences(mode):
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:25]
    A = w.sigma
    beta = 0.7
    phi, rhos = ext.penalty_cost(m, u, w.rho0, w.sigma, A, beta, w.dt)
    g = ext.penalty_gradient(m, u, rhos, w.sigma, A, beta, w.dt, mode=mode)
    eps = 1e-5
    for j, k in [(0, 0), (7, 1), (24, 0), (12, 1)]:
        up = u.copy()
        up[j, k] += eps
        dn = u.copy()
        dn[j, k] -= eps
        fd = (ext.penalty_cost(m, up, w.rho0, w.sigma, A, beta, w.dt)[0]
              - ext.penalty_cost(m, dn, w.rho0, w.sigma, A, beta, w.dt)[0]) / (2 * eps)
        assert abs(fd - g[j, k]) < 1e-8 * max(1.0, abs(fd))


def test_penalty_recursion_equals_sum_of_backward_evolutions():
    """App. B: the modified backward sweep equals the sum of backward
    evolutions started at every time step (first-order gradient)."""
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:15]
    A = w.sigma
    rhos = rk.forward(m, u, w.rho0, w.dt)
    g_pen = ext.penalty_gradient(m, u, rhos, np.zeros_like(A), A, 1.0, w.dt)
    ref = np.zeros_like(g_pen)
    for n in range(1, len(u) + 1):  # Tr(A rho_n) depends on slices 0..n-1
        lams = rk.backward(m, u[:n], A, w.dt)
        ref[:n] += rk.gradient_grape1(m, u[:n], rhos[:n + 1], lams, w.dt)
    assert _relerr(g_pen, -w.dt * ref) < 1e-12


@pytest.mark.parametrize("n_sub", [1, 2])
def test_penalty_cost_value_closed_form(n_sub):
    """The value of the penalised index (Eq. (24), with the integral of
    Eq. (25) as the sum over n = 0 .. N of App. B), pinned by a closed form:
    for the undriven damped resonator, Tr(a^dag a rho_n) = n0 P(-kappa h)^(n n_sub)
    exactly in truncation (the adjoint generator maps a^dag a to -kappa a^dag a),
    P the RK4 stability polynomial, so
        Phi_p = dt n0 sum_{n=0}^{N} P(-kappa h)^(n n_sub).
    A sum without the n = 0 term, one that stops at N - 1 or one without dt
    misses it by at least 0.4 * dt * n0 * P^(N n_sub) (about 1e-2 here)."""
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    n_t, beta = 37, 0.4
    u = np.zeros((n_t, 2))
    a = wl.destroy(10)
    A = a.conj().T @ a
    n0 = np.trace(A @ w.rho0).real
    kappa = float(w.gammas[0])
    z = -kappa * w.dt / n_sub
    P = (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24) ** n_sub
    pen = w.dt * n0 * sum(P ** n for n in range(n_t + 1))
    # sigma = I: Tr(rho_N) = 1 (the trace is conserved), so Phi = 1 - beta Phi_p
    phi, rhos = ext.penalty_cost(m, u, w.rho0, np.eye(10, dtype=complex), A, beta, w.dt, n_sub)
    assert len(rhos) == n_t + 1
    assert abs(phi - (1.0 - beta * pen)) < 1e-13
    assert beta * w.dt * n0 * P ** n_t > 1e-3


def test_penalty_beta_zero_is_the_plain_index():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:12]
    phi, rhos = ext.penalty_cost(m, u, w.rho0, w.sigma, w.sigma, 0.0, w.dt)
    g = ext.penalty_gradient(m, u, rhos, w.sigma, w.sigma, 0.0, w.dt, mode="exact")
    ge, _ = rk.gradient_exact(m, u, rhos, w.sigma, w.dt)
    assert abs(phi - rk.cost(w.sigma, rhos[-1])) == 0.0
    assert _relerr(g, ge) < 1e-14


def test_multi_state_sum_vs_finite_differences():
    """Eq. (22): qubit-conditioned resonator problems (chi -> +-chi) summed."""
    n_t, dt = 10, 0.05
    u = wl.controls_uniform(21, n_t, 2)
    ws = [wl.resonator_problem(12, s * 1.5, 1.0, 1.0, u, dt) for s in (+1, -1)]
    ms = [rk.Model.from_workload(w) for w in ws]
    vac = np.zeros((12, 12), complex)
    vac[0, 0] = 1.0
    phi, g = ext.multi_state_cost_and_grad(ms, u, [w.rho0 for w in ws], vac, dt, mode="exact")
    eps = 1e-6
    for j, k in [(0, 1), (5, 0), (9, 1)]:
        up = u.copy()
        up[j, k] += eps
        dn = u.copy()
        dn[j, k] -= eps
        fp = sum(rk.cost(vac, rk.forward(m, up, w.rho0, dt)[-1]) for m, w in zip(ms, ws))
        fm = sum(rk.cost(vac, rk.forward(m, dn, w.rho0, dt)[-1]) for m, w in zip(ms, ws))
        assert abs((fp - fm) / (2 * eps) - g[j, k]) < 1e-8
    assert phi == pytest.approx(sum(rk.cost(vac, rk.forward(m, u, w.rho0, dt)[-1]) for m, w in zip(ms, ws)))
