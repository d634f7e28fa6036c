"""Exponential-free open GRAPE, plain float64 reference (test infrastructure).

Written from Secs. II.B and III of the paper.  Notation follows the paper:
H(t) = H0 + sum_k u_k(t) H_k (Eq. (1)); piecewise-constant controls u_k(j)
on slices of length dt (Sec. II.A); master equation
    d rho/dt = L rho = -i[H, rho] + sum_j gamma_j D[a_j] rho,
    D[a] rho = a rho a^dag - {a^dag a, rho}/2                (Eqs. (3), (4));
performance index Phi = Tr(sigma rho(T)) (Eq. (8)); forward states rho_j
(Eq. (10)); backward states lambda_j = L_{j+1}^dag ... L_N^dag sigma
(Eq. (11)); first-order gradient
    dPhi/du_k(j) = -i dt Tr{ lambda_j [H_k, rho_j] }        (Eq. (13)).
The propagation is classical fourth-order Runge-Kutta, slice by slice
(Eq. (14)), and the adjoint is integrated with L^dag from lambda_N = sigma
(Eq. (15)).

Indexing is 0-based: u[j] acts on [j dt, (j+1) dt) and maps rho[j] to
rho[j+1] (the paper's u_k(j+1), rho_{j+1}).  The first-order gradient of
slice j therefore pairs rho[j+1] with lambda[j+1].

Readings of points the paper leaves open (listed with the design notes):
  * The backward integration follows Eq. (11): lambda_j = P(h L_j^dag)
    lambda_{j+1}, i.e. integrate d lambda/ds = +L^dag lambda in reversed
    time s = T - t.  The printed step of Eq. (15) has the opposite sign and
    is read as a typo (it would integrate the anti-dissipative direction).
  * "Standard Runge-Kutta" is read as classical RK4 with a fixed step
    h = dt / n_sub.
  * The "higher-order" gradient the paper mentions is provided as the exact
    derivative of the RK4-discretised Phi (reverse mode through the four
    stages of every step), alongside the paper's first-order Eq. (13).

Operators may be dense numpy arrays or scipy.sparse matrices; only "@",
".conj()" and ".T" are used on them.  Plain, slow, obviously correct: no
blocking, fusion or reordering.

PARITY PINS: see the tests that start with test_oracle.
"""
from __future__ import annotations

import numpy as np


def _dag(A):
    return A.conj().T


def _dense(X):
    return np.asarray(X.todense()) if hasattr(X, "todense") else np.asarray(X)


class Model:
    """Operator set of Eq. (1) and Eq. (4): H0, control Hamiltonians H_k,
    collapse operators a_j with rates gamma_j."""

    def __init__(self, H0, Hk, c_ops, gammas):
        self.H0 = H0
        self.Hk = list(Hk)
        self.c_ops = list(c_ops)
        self.gammas = [float(g) for g in gammas]
        self.d = H0.shape[0]
        self.K = len(self.Hk)
        # a_j^dag a_j appears in the anticommutator of D[a_j]
        self.cdc = [_dag(c) @ c for c in self.c_ops]

    @classmethod
    def from_workload(cls, w, sparse: bool = False):
        if sparse:
            import scipy.sparse as sp
            conv = lambda A: sp.csr_matrix(A)  # noqa: E731
            return cls(conv(w.H0), [conv(h) for h in w.Hk], [conv(c) for c in w.c_ops], w.gammas)
        return cls(w.H0, list(w.Hk), list(w.c_ops), w.gammas)

    def hamiltonian(self, u_j):
        """H_j = H0 + sum_k u_k(j) H_k (Eq. (1) on slice j)."""
        H = self.H0
        for k in range(self.K):
            H = H + float(u_j[k]) * self.Hk[k]
        return H


def lindblad(model: Model, H, Y):
    """L Y = -i[H, Y] + sum_j gamma_j (a_j Y a_j^dag - {a_j^dag a_j, Y}/2), Eqs. (3)-(4)."""
    out = -1j * (H @ Y - Y @ H)
    for c, cdc, g in zip(model.c_ops, model.cdc, model.gammas):
        out = out + g * (c @ Y @ _dag(c) - 0.5 * (cdc @ Y + Y @ cdc))
    return np.asarray(out)


def lindblad_adjoint(model: Model, H, X):
    """L^dag X, defined by Tr(X (L Y)) = Tr((L^dag X) Y):
    i[H, X] + sum_j gamma_j (a_j^dag X a_j - {a_j^dag a_j, X}/2)."""
    out = 1j * (H @ X - X @ H)
    for c, cdc, g in zip(model.c_ops, model.cdc, model.gammas):
        out = out + g * (_dag(c) @ X @ c - 0.5 * (cdc @ X + X @ cdc))
    return np.asarray(out)


def rk4_step(f, Y, h):
    """One classical RK4 step of dY/dt = f(Y)."""
    k1 = f(Y)
    k2 = f(Y + 0.5 * h * k1)
    k3 = f(Y + 0.5 * h * k2)
    k4 = f(Y + h * k3)
    return Y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def forward(model: Model, u, rho0, dt, n_sub: int = 1):
    """Stepwise RK4 integration of Eq. (14), saving every rho_j.

    Returns the list [rho_0, rho_1, ..., rho_{N_t}]."""
    u = np.asarray(u, dtype=np.float64)
    h = dt / n_sub
    rhos = [np.array(rho0, dtype=np.complex128)]
    rho = rhos[0]
    for j in range(u.shape[0]):
        H = model.hamiltonian(u[j])
        f = lambda Y, H=H: lindblad(model, H, Y)  # noqa: E731
        for _ in range(n_sub):
            rho = rk4_step(f, rho, h)
        rhos.append(rho)
    return rhos


def cost(sigma, rho_T):
    """Phi = Tr(sigma rho(T)) (Eq. (8)); real for Hermitian sigma and rho."""
    val = np.trace(_dense(sigma) @ rho_T)
    return float(val.real)


def backward(model: Model, u, sigma, dt, n_sub: int = 1):
    """Backward states of Eq. (11) by RK4 integration with L^dag from
    lambda_N = sigma (Eq. (15), sign read from Eq. (11)).

    Returns [lambda_0, ..., lambda_{N_t}]."""
    u = np.asarray(u, dtype=np.float64)
    h = dt / n_sub
    n_t = u.shape[0]
    lams = [None] * (n_t + 1)
    lam = np.array(_dense(sigma), dtype=np.complex128)
    lams[n_t] = lam
    for j in range(n_t - 1, -1, -1):
        H = model.hamiltonian(u[j])
        f = lambda X, H=H: lindblad_adjoint(model, H, X)  # noqa: E731
        for _ in range(n_sub):
            lam = rk4_step(f, lam, h)
        lams[j] = lam
    return lams


def gradient_grape1(model: Model, u, rhos, lams, dt):
    """First-order gradient of Eq. (13), 0-based: slice j pairs rho[j+1]
    with lambda[j+1]:  g[j, k] = -i dt Tr(lambda_{j+1} [H_k, rho_{j+1}])."""
    n_t = len(rhos) - 1
    g = np.zeros((n_t, model.K))
    for j in range(n_t):
        rho, lam = rhos[j + 1], lams[j + 1]
        for k in range(model.K):
            Hk = model.Hk[k]
            comm = Hk @ rho - rho @ Hk
            val = -1j * dt * np.trace(lam @ comm)
            g[j, k] = val.real
    return g


def gradient_exact(model: Model, u, rhos, sigma, dt, n_sub: int = 1):
    """Exact derivative of the RK4-discretised Phi with respect to u[j, k].

    For one RK4 step Y1 = rho, Y2 = rho + h/2 k1, Y3 = rho + h/2 k2,
    Y4 = rho + h k3, k_s = L(Y_s), rho' = rho + h/6 (k1 + 2k2 + 2k3 + k4),
    reverse mode with the incoming cotangent lam' gives
        kb4 = h/6 lam',            Yb4 = L^dag kb4
        kb3 = h/3 lam' + h Yb4,    Yb3 = L^dag kb3
        kb2 = h/3 lam' + h/2 Yb3,  Yb2 = L^dag kb2
        kb1 = h/6 lam' + h/2 Yb2,  Yb1 = L^dag kb1
        lam = lam' + Yb1 + Yb2 + Yb3 + Yb4
    and, since dk_s/du_k = -i[H_k, Y_s],
        g[j, k] += sum_s Re Tr(kb_s (-i [H_k, Y_s])).
    Returns (g, lambda_0)."""
    u = np.asarray(u, dtype=np.float64)
    h = dt / n_sub
    n_t = u.shape[0]
    g = np.zeros((n_t, model.K))
    lam = np.array(_dense(sigma), dtype=np.complex128)
    for j in range(n_t - 1, -1, -1):
        H = model.hamiltonian(u[j])
        f = lambda Y, H=H: lindblad(model, H, Y)  # noqa: E731
        fa = lambda X, H=H: lindblad_adjoint(model, H, X)  # noqa: E731
        # start states of the n_sub substeps of slice j
        starts = [rhos[j]]
        for _ in range(n_sub - 1):
            starts.append(rk4_step(f, starts[-1], h))
        for s in range(n_sub - 1, -1, -1):
            rho = starts[s]
            Y1 = rho
            k1 = f(Y1)
            Y2 = rho + 0.5 * h * k1
            k2 = f(Y2)
            Y3 = rho + 0.5 * h * k2
            k3 = f(Y3)
            Y4 = rho + h * k3
            kb4 = (h / 6.0) * lam
            Yb4 = fa(kb4)
            kb3 = (h / 3.0) * lam + h * Yb4
            Yb3 = fa(kb3)
            kb2 = (h / 3.0) * lam + 0.5 * h * Yb3
            Yb2 = fa(kb2)
            kb1 = (h / 6.0) * lam + 0.5 * h * Yb2
            Yb1 = fa(kb1)
            for k in range(model.K):
                Hk = model.Hk[k]
                acc = 0.0
                for kb, Y in ((kb1, Y1), (kb2, Y2), (kb3, Y3), (kb4, Y4)):
                    acc += np.trace(kb @ (-1j * (Hk @ Y - Y @ Hk))).real
                g[j, k] += acc
            lam = lam + Yb1 + Yb2 + Yb3 + Yb4
    return g, lam


def cost_and_grad(model: Model, u, rho0, sigma, dt, n_sub: int = 1, mode: str = "grape1"):
    """Phi and dPhi/du for one control array u[N_t, K].

    mode = "grape1": the paper's Eq. (13) with RK4 forward/backward states.
    mode = "exact":  the exact derivative of the RK4-discretised Phi."""
    rhos = forward(model, u, rho0, dt, n_sub)
    phi = cost(sigma, rhos[-1])
    if mode == "grape1":
        lams = backward(model, u, sigma, dt, n_sub)
        g = gradient_grape1(model, u, rhos, lams, dt)
    elif mode == "exact":
        g, _ = gradient_exact(model, u, rhos, sigma, dt, n_sub)
    else:
        raise ValueError(mode)
    return phi, g, rhos
