"""Pins of the float64 oracle against facts fixed by the paper and by the
mathematics: closed forms, invariants, special cases that reduce to library
routines, brute-force finite differences, convergence orders.  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads as wl
from oracle import closed, rk, superop


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_herm(rng, d, scale=1.0):
    X = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return scale * 0.5 * (X + X.conj().T)


def _rand_dm(rng, d, rank=3):
    W = rng.standard_normal((d, rank)) + 1j * rng.standard_normal((d, rank))
    r = W @ W.conj().T
    return r / np.trace(r).real


def _rand_model(rng, d, K=2, J=2):
    H0 = _rand_herm(rng, d)
    Hk = [_rand_herm(rng, d, 0.3) for _ in range(K)]
    cs = [(rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * 0.3 for _ in range(J)]
    gs = rng.uniform(0.1, 0.5, size=J)
    return rk.Model(H0, Hk, cs, gs)


def _relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


# --------------------------------------------------------------------------
# Matrix exponential (Sec. II.B, Eq. (7)) against an independent library
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [0.01, 1.0, 7.0, 60.0])
def test_expm_matches_scipy(scale):
    rng = _rng(1)
    A = scale * (rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24))) / 5
    ref = sl.expm(A)
    assert _relerr(superop.expm(A), ref) < 1e-12


def test_expm_special_cases():
    d = np.array([0.3, -2.0 + 1j, 5.0, 0.0])
    assert np.allclose(superop.expm(np.diag(d)), np.diag(np.exp(d)), rtol=1e-14, atol=0)
    N = np.triu(_rng(2).standard_normal((5, 5)), 1)  # nilpotent
    ref = np.eye(5) + N + N @ N / 2 + N @ N @ N / 6 + N @ N @ N @ N / 24
    assert _relerr(superop.expm(N), ref) < 1e-14


def test_frechet_van_loan_vs_fd():
    rng = _rng(3)
    A = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    E = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    M = np.zeros((12, 12), dtype=complex)
    M[:6, :6] = A
    M[6:, 6:] = A
    M[:6, 6:] = E
    L = superop.expm(M)[:6, 6:]
    s = 1e-6
    fd = (sl.expm(A + s * E) - sl.expm(A - s * E)) / (2 * s)
    assert _relerr(L, fd) < 1e-8


# --------------------------------------------------------------------------
# Master equation: superoperator form, adjoint definition
# --------------------------------------------------------------------------

def test_liouvillian_matches_rhs():
    rng = _rng(4)
    m = _rand_model(rng, 7)
    H = m.hamiltonian([0.4, -0.7])
    Y = _rand_herm(rng, 7)
    L = superop.liouvillian(H, m.c_ops, m.gammas)
    assert _relerr(superop.unvec(L @ superop.vec(Y), 7), rk.lindblad(m, H, Y)) < 1e-14


def test_adjoint_definition():
    rng = _rng(5)
    m = _rand_model(rng, 8)
    H = m.hamiltonian([0.2, 0.9])
    X = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    Y = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    lhs = np.trace(X @ rk.lindblad(m, H, Y))
    rhs = np.trace(rk.lindblad_adjoint(m, H, X) @ Y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_trace_preserving_and_identity_fixed():
    rng = _rng(6)
    m = _rand_model(rng, 6)
    H = m.hamiltonian([1.0, -1.0])
    Y = _rand_herm(rng, 6)
    assert abs(np.trace(rk.lindblad(m, H, Y))) < 1e-13
    assert np.max(np.abs(rk.lindblad_adjoint(m, H, np.eye(6)))) < 1e-14


# --------------------------------------------------------------------------
# Closed forms of the damped resonator
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_sub", [1, 3])
def test_undriven_photon_number_discrete_and_continuous(n_sub):
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = np.zeros((200, 2))
    rhos = rk.forward(m, u, w.rho0, w.dt, n_sub)
    na = w.sigma
    n0 = np.trace(na @ w.rho0).real
    h = w.dt / n_sub
    for j in (1, 17, 100, 200):
        nj = np.trace(na @ rhos[j]).real
        # <a^dag a> obeys L^dag(a^dag a) = -kappa a^dag a exactly in truncation
        assert abs(nj - n0 * closed.rk4_poly(-h) ** (j * n_sub)) < 1e-13 * n0
        assert abs(nj - n0 * math.exp(-j * w.dt)) < 2e-6 * n0 / n_sub ** 4


def test_amplitude_damping_full_state():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    n_t = 20
    u = np.zeros((n_t, 2))
    t = n_t * w.dt
    ref = closed.amplitude_damping(w.rho0, 0.5, 1.0, t)
    ex = superop.forward(m, u, w.rho0, w.dt)[-1]
    assert _relerr(ex, ref) < 1e-12
    rkT = rk.forward(m, u, w.rho0, w.dt)[-1]
    assert _relerr(rkT, ref) < 1e-5
    assert _relerr(rkT, ref) > 1e-12  # RK4 is not exact: the check is not vacuous


def test_moment_recursion_matches_rk_d40():
    delta, kappa, alpha = 0.5, 1.0, 1.2
    rng = _rng(7)
    n_t, dt = 40, 0.05
    u = rng.uniform(-1, 1, size=(n_t, 2))
    w = wl.resonator_problem(40, delta, kappa, alpha, u, dt)
    m = rk.Model.from_workload(w)
    for n_sub in (1, 2):
        rhos = rk.forward(m, u, w.rho0, dt, n_sub)
        phi = rk.cost(w.sigma, rhos[-1])
        a = wl.destroy(40)
        A0 = np.trace(a @ w.rho0)
        n0 = np.trace(w.sigma @ w.rho0).real
        nT, AT, traj = closed.moment_recursion(u, dt, n_sub, delta, kappa, n0, A0)
        assert abs(phi - nT) < 1e-12 * abs(nT)
        assert abs(np.trace(a @ rhos[-1]) - AT) < 1e-12 * abs(AT)
        g, _ = rk.gradient_exact(m, u, rhos, w.sigma, dt, n_sub)
        gfd = closed.moment_fd_gradient(u, dt, n_sub, delta, kappa, n0, A0)
        assert _relerr(g, gfd) < 1e-7


def test_driven_steady_state_eq20():
    delta, kappa = 0.5, 1.0
    ux, uy = 0.3, -0.2
    n_t, dt = 1200, 0.05
    u = np.tile([ux, uy], (n_t, 1))
    w = wl.resonator_problem(16, delta, kappa, 0.0, u, dt)
    m = rk.Model.from_workload(w)
    rhoT = rk.forward(m, u, w.rho0, dt)[-1]
    a = wl.destroy(16)
    alpha_ss, n_ss = closed.steady_state(ux, uy, delta, kappa)
    assert abs(np.trace(a @ rhoT) - alpha_ss) < 1e-11
    assert abs(np.trace(w.sigma @ rhoT).real - n_ss) < 1e-11
    # the steady state is a coherent state |alpha_ss>
    ket = wl.coherent_ket(16, alpha_ss)
    assert _relerr(rhoT, np.outer(ket, ket.conj())) < 1e-9


def test_continuous_gradient_closed_form():
    delta, kappa, alpha = 0.5, 1.0, 0.5
    rng = _rng(8)
    n_t, dt = 12, 0.1
    u = rng.uniform(-0.3, 0.3, size=(n_t, 2))
    w = wl.resonator_problem(14, delta, kappa, alpha, u, dt)
    m = rk.Model.from_workload(w)
    rhos = superop.forward(m, u, w.rho0, dt)
    lams = superop.backward(m, u, w.sigma, dt)
    a = wl.destroy(14)
    AT = np.trace(a @ rhos[-1])
    g = superop.gradient_frechet(m, u, rhos, lams, dt)
    ref = closed.continuous_gradient_photon_number(u, dt, delta, kappa, AT)
    assert _relerr(g, ref) < 1e-9
    # first-order GRAPE with exact propagators against its closed form
    g1 = rk.gradient_grape1(m, u, rhos, lams, dt)
    ref1 = closed.continuous_gradient_photon_number(u, dt, delta, kappa, AT, first_order=True)
    assert _relerr(g1, ref1) < 1e-9


# --------------------------------------------------------------------------
# cQED sector invariants (Sec. IV)
# --------------------------------------------------------------------------

def test_cqed_qubit_sector_exact():
    rng = _rng(9)
    n_t, dt = 60, 0.01
    u = rng.uniform(-1, 1, size=(n_t, 2))
    w = wl.transmon_resonator_problem(3, 8, alpha=1.0, u=u, dt=dt)
    m = rk.Model.from_workload(w)
    rhos = rk.forward(m, u, w.rho0, dt)
    b = np.kron(wl.destroy(3), np.eye(8))
    nb = b.conj().T @ b
    pf = np.kron(np.diag([0, 0, 1.0]), np.eye(8))
    for j in (10, 60):
        assert abs(np.trace(nb @ rhos[j]).real - closed.rk4_poly(-0.01 * dt) ** j) < 1e-14
        assert abs(np.trace(pf @ rhos[j])) < 1e-15
    g_leak, _ = rk.gradient_exact(m, u, rhos, pf, dt)
    assert np.max(np.abs(g_leak)) < 1e-15


# --------------------------------------------------------------------------
# Adjoint sweep and gradients
# --------------------------------------------------------------------------

def test_adjoint_identity_every_slice():
    rng = _rng(10)
    m = _rand_model(rng, 6)
    n_t, dt = 25, 0.05
    u = rng.uniform(-1, 1, size=(n_t, 2))
    rho0 = _rand_dm(rng, 6)
    sigma = _rand_herm(rng, 6)
    rhos = rk.forward(m, u, rho0, dt)
    lams = rk.backward(m, u, sigma, dt)
    phi = rk.cost(sigma, rhos[-1])
    for j in range(n_t + 1):
        assert abs(np.trace(lams[j] @ rhos[j]).real - phi) < 1e-13 * max(1, abs(phi))
    _, lam0 = rk.gradient_exact(m, u, rhos, sigma, dt)
    assert _relerr(lam0, lams[0]) < 1e-13


def test_sigma_identity():
    rng = _rng(11)
    m = _rand_model(rng, 5)
    n_t, dt = 10, 0.05
    u = rng.uniform(-1, 1, size=(n_t, 2))
    rho0 = _rand_dm(rng, 5)
    phi, g, _ = rk.cost_and_grad(m, u, rho0, np.eye(5), dt)
    assert abs(phi - 1.0) < 1e-13
    assert np.max(np.abs(g)) < 1e-14
    lams = rk.backward(m, u, np.eye(5), dt)
    assert np.max(np.abs(lams[0] - np.eye(5))) < 1e-14
    ge, _ = rk.gradient_exact(m, u, rk.forward(m, u, rho0, dt), np.eye(5), dt)
    assert np.max(np.abs(ge)) < 1e-14


def test_unitary_reduction():
    rng = _rng(12)
    d = 6
    H0 = _rand_herm(rng, d)
    Hk = [_rand_herm(rng, d, 0.5)]
    m = rk.Model(H0, Hk, [], [])
    u = rng.uniform(-1, 1, size=(5, 1))
    dt = 0.1
    rho0 = _rand_dm(rng, d)
    ex = superop.forward(m, u, rho0, dt)[-1]
    r = rho0
    for j in range(5):
        U = sl.expm(-1j * dt * m.hamiltonian(u[j]))
        r = U @ r @ U.conj().T
    assert _relerr(ex, r) < 1e-13


def test_rk4_global_order():
    rng = _rng(13)
    m = _rand_model(rng, 5)
    n_t, dt = 10, 0.2
    u = rng.uniform(-1, 1, size=(n_t, 2))
    rho0 = _rand_dm(rng, 5)
    ex = superop.forward(m, u, rho0, dt)[-1]
    e1 = np.linalg.norm(rk.forward(m, u, rho0, dt, 1)[-1] - ex)
    e2 = np.linalg.norm(rk.forward(m, u, rho0, dt, 2)[-1] - ex)
    assert 14.0 < e1 / e2 < 18.0


@pytest.mark.parametrize("n_sub", [1, 2])
def test_exact_gradient_vs_finite_differences(n_sub):
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:30]
    rhos = rk.forward(m, u, w.rho0, w.dt, n_sub)
    g, _ = rk.gradient_exact(m, u, rhos, w.sigma, w.dt, n_sub)
    s = 1e-5
    idx = [(0, 0), (3, 1), (11, 0), (17, 1), (29, 0), (29, 1)]
    fd = []
    for j, k in idx:
        up = u.copy()
        up[j, k] += s
        dn = u.copy()
        dn[j, k] -= s
        fp = rk.cost(w.sigma, rk.forward(m, up, w.rho0, w.dt, n_sub)[-1])
        fm = rk.cost(w.sigma, rk.forward(m, dn, w.rho0, w.dt, n_sub)[-1])
        fd.append((fp - fm) / (2 * s))
    got = np.array([g[j, k] for j, k in idx])
    assert _relerr(got, np.array(fd)) < 1e-7


def test_grape1_is_first_order():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    u = w.u[:20]
    dt = w.dt

    def gap(u_, dt_):
        phi, g1, rhos = rk.cost_and_grad(m, u_, w.rho0, w.sigma, dt_)
        ge, _ = rk.gradient_exact(m, u_, rhos, w.sigma, dt_)
        return g1, ge

    g1a, gea = gap(u, dt)
    # split each slice in two half-slices with the same control
    u2 = np.repeat(u, 2, axis=0)
    g1b, geb = gap(u2, dt / 2)
    # derivative with respect to the shared control of both halves
    g1b = g1b[0::2] + g1b[1::2]
    geb = geb[0::2] + geb[1::2]
    ratio = np.linalg.norm(g1a - gea) / np.linalg.norm(g1b - geb)
    assert 1.7 < ratio < 2.3


def test_trace_hermiticity_positivity():
    w = wl.config_c1()
    m = rk.Model.from_workload(w)
    rhos = rk.forward(m, w.u, w.rho0, w.dt)
    for r in rhos[::20]:
        assert abs(np.trace(r) - 1.0) < 1e-13
        assert np.max(np.abs(r - r.conj().T)) < 1e-13
        assert np.min(np.linalg.eigvalsh(0.5 * (r + r.conj().T))) > -1e-4


def test_sparse_and_dense_operators_agree():
    w = wl.transmon_resonator_problem(3, 6, qubit_drive=True, alpha=1.0,
                                      u=_rng(14).uniform(-1, 1, size=(8, 4)), dt=0.01)
    md = rk.Model.from_workload(w)
    ms = rk.Model.from_workload(w, sparse=True)
    pd, gd, _ = rk.cost_and_grad(md, w.u, w.rho0, w.sigma, w.dt, mode="exact")
    ps, gs, _ = rk.cost_and_grad(ms, w.u, w.rho0, w.sigma, w.dt, mode="exact")
    assert abs(pd - ps) < 1e-13 * abs(pd)
    assert _relerr(gs, gd) < 1e-12
