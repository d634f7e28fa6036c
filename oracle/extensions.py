"""Extensions of the basic index (test infrastructure): Gaussian control
filter (App. A), photon-number penalty (Sec. IV.C, Eqs. (24)-(25), App. B)
and multi-state index (Eq. (22)).  Plain float64, written from the paper.

Readings:
  * Filter (Eq. (A4)), 1-based indices n (subpixel) and j (control):
        T[n, j] = ( erf(w0 ((n-1) dts - (j-1) dtu) / 2) - erf(w0 ((n-1) dts - j dtu) / 2) ) / 2,
    evaluated at the subpixel start (n-1) dts as printed; w0 = wB / sqrt(-ln(1/sqrt 2)).
    s_k(n) = sum_j T[n, j] u_k(j) (Eq. (A1)); dPhi/du = T^T dPhi/ds (Eq. (A2)).
    The first and last controls are held fixed (Fig. 1): their gradient is
    zero.
  * Penalty: Phi = Tr(sigma rho_N) - beta sum_{n=0}^{N} dt Tr(A rho_n)
    (Eq. (24) with the integral of Eq. (25) as the sum of App. B).  The
    garbled recursion of App. B is read as mu_n = A + L_{n+1}^dag mu_{n+1},
    mu_N = A; by linearity the combined adjoint is
        lam_N = sigma - beta dt A,  lam_n = P(h L_n^dag) lam_{n+1} - beta dt A.
  * Multi-state: Eq. (22) sums (not averages) over the input states.
"""
from __future__ import annotations

import math

import numpy as np

from . import rk


def omega0_from_bandwidth(omega_b):
    """Reference bandwidth of the Gaussian filter from the 3 dB bandwidth."""
    return omega_b / math.sqrt(-math.log(1.0 / math.sqrt(2.0)))


def transfer_matrix(n_ctrl, n_sub_px, dtu, dts, w0):
    """T[n, j] of Eq. (A4), shape (M, N) (0-based storage of the 1-based formula)."""
    T = np.zeros((n_sub_px, n_ctrl))
    for n in range(1, n_sub_px + 1):
        for j in range(1, n_ctrl + 1):
            a = math.erf(w0 * ((n - 1) * dts - (j - 1) * dtu) / 2.0)
            b = math.erf(w0 * ((n - 1) * dts - j * dtu) / 2.0)
            T[n - 1, j - 1] = 0.5 * (a - b)
    return T


def transfer_matrix_integral(n_ctrl, n_sub_px, dtu, dts, w0):
    """Eq. (A4) in its integral form, by quadrature (independent check)."""
    from scipy.integrate import quad

    T = np.zeros((n_sub_px, n_ctrl))
    for n in range(1, n_sub_px + 1):
        for j in range(1, n_ctrl + 1):
            x = (2 * (n - 1) * dts - (2 * j - 1) * dtu) / 2.0

            def f(w):
                if w == 0.0:
                    return dtu / (2.0 * math.pi)
                return math.exp(-(w / w0) ** 2) * math.cos(w * x) * math.sin(w * dtu / 2.0) / (math.pi * w)

            val, _ = quad(f, -40 * w0, 40 * w0, limit=400, points=[0.0])
            T[n - 1, j - 1] = val
    return T


def filtered_controls(u, T):
    """s = T u per control channel (Eq. (A1)); u (N, K) -> s (M, K)."""
    return T @ np.asarray(u)


def chain_rule(g_s, T, fix_ends=True):
    """dPhi/du = T^T dPhi/ds (Eq. (A2)); zero for the held first / last control."""
    g = T.T @ np.asarray(g_s)
    if fix_ends:
        g[0, :] = 0.0
        g[-1, :] = 0.0
    return g


def penalty_cost(model, u, rho0, sigma, A, beta, dt, n_sub=1):
    rhos = rk.forward(model, u, rho0, dt, n_sub)
    phi0 = rk.cost(sigma, rhos[-1])
    pen = sum(dt * np.trace(A @ r).real for r in rhos)
    return phi0 - beta * pen, rhos


def penalty_gradient(model, u, rhos, sigma, A, beta, dt, n_sub=1, mode="grape1"):
    """Gradient of the penalised index with the combined adjoint."""
    u = np.asarray(u, dtype=np.float64)
    n_t = u.shape[0]
    h = dt / n_sub
    g = np.zeros((n_t, model.K))
    lam = np.array(sigma, dtype=np.complex128) - beta * dt * A
    for j in range(n_t - 1, -1, -1):
        H = model.hamiltonian(u[j])
        fa = lambda X, H=H: rk.lindblad_adjoint(model, H, X)  # noqa: E731
        if mode == "grape1":
            for k in range(model.K):
                Hk = model.Hk[k]
                comm = Hk @ rhos[j + 1] - rhos[j + 1] @ Hk
                g[j, k] = (-1j * dt * np.trace(lam @ comm)).real
            for _ in range(n_sub):
                lam = rk.rk4_step(fa, lam, h)
        else:
            gj, lam = rk.gradient_exact(model, u[j:j + 1], [rhos[j], rhos[j + 1]], lam, dt, n_sub)
            g[j] = gj[0]
        lam = lam - beta * dt * A
    return g


def multi_state_cost_and_grad(models, u, rho0s, sigma, dt, n_sub=1, mode="grape1"):
    """Eq. (22): Phi = sum_i Tr(sigma rho_i(T)); models may differ per state
    (qubit-conditioned resonator Hamiltonians) or be the same."""
    phi, g = 0.0, None
    for m, r0 in zip(models, rho0s):
        p, gi, _ = rk.cost_and_grad(m, u, r0, sigma, dt, n_sub, mode)
        phi += p
        g = gi if g is None else g + gi
    return phi, g
