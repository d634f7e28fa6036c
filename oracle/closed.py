"""Closed forms of the damped (driven) resonator used to pin the oracle
(test infrastructure).

Model (Sec. IV.A, Eqs. (19), (20), (23)): H = Delta a^dag a + eps a^dag +
eps^* a with eps = u_x + i u_y (the two-quadrature drive of Eq. (23)),
collapse kappa D[a].

* Free decay (u = 0): the amplitude-damping solution
      rho_mn(t) = e^{-i Delta (m-n) t} e^{-kappa (m+n) t / 2}
                  sum_k sqrt(C(m+k, k) C(n+k, k)) (1 - e^{-kappa t})^k rho_{m+k, n+k}(0),
  exact in any Fock truncation because the truncated space is invariant.
* Moments: v = (<a^dag a>, <a>, <a^dag>, 1) obeys dv/dt = M v with
      d<a>/dt  = -z <a> - i eps,  z = kappa/2 + i Delta,
      d<n>/dt  = -kappa <n> + i (eps^* <a> - eps <a^dag>).
  RK4 applied to rho moves the moments by the same polynomial,
  v' = P(h M) v, P(x) = 1 + x + x^2/2 + x^3/6 + x^4/24, as long as the
  truncation is not felt (d >= 30 for the states used in the tests).
* Steady state under constant eps (Eq. (20) with the drive on resonance
  with the rotating frame): alpha_ss = -i eps / (kappa/2 + i Delta),
  n_ss = |eps|^2 / (Delta^2 + kappa^2/4).
* Continuous-time gradient of Phi = <a^dag a>(T): the state is a displaced
  copy of the undriven one, so n(T) = n_free(T) + |A_T|^2 - |A_free(T)|^2 and
      dn(T)/du_x(j) = 2 Re( conj(A_T) (-i/z) (1 - e^{-z dt}) e^{-z (T - t_{j+1})} ),
      dn(T)/du_y(j) = 2 Re( conj(A_T) ( 1/z) (1 - e^{-z dt}) e^{-z (T - t_{j+1})} ).
  The first-order (Eq. (13)) analogue replaces (1 - e^{-z dt}) / z by dt.
"""
from __future__ import annotations

import math

import numpy as np


def rk4_poly(x):
    """Stability polynomial of classical RK4."""
    return 1.0 + x + x * x / 2.0 + x ** 3 / 6.0 + x ** 4 / 24.0


def rk4_poly_matrix(M):
    ident = np.eye(M.shape[0], dtype=np.complex128)
    M2 = M @ M
    M3 = M2 @ M
    M4 = M3 @ M
    return ident + M + M2 / 2.0 + M3 / 6.0 + M4 / 24.0


def amplitude_damping(rho0, delta, kappa, t):
    """Exact rho(t) of the undriven damped resonator from rho0."""
    rho0 = np.asarray(rho0)
    N = rho0.shape[0]
    out = np.zeros_like(rho0, dtype=np.complex128)
    p = 1.0 - math.exp(-kappa * t)
    for m in range(N):
        for n in range(N):
            s = 0.0 + 0.0j
            for k in range(0, N - max(m, n)):
                s += math.sqrt(math.comb(m + k, k) * math.comb(n + k, k)) * p ** k * rho0[m + k, n + k]
            out[m, n] = np.exp(-1j * delta * (m - n) * t) * math.exp(-kappa * (m + n) * t / 2.0) * s
    return out


def moment_matrix(ux, uy, delta, kappa):
    eps = ux + 1j * uy
    z = kappa / 2.0 + 1j * delta
    M = np.zeros((4, 4), dtype=np.complex128)
    M[0, 0] = -kappa
    M[0, 1] = 1j * np.conj(eps)
    M[0, 2] = -1j * eps
    M[1, 1] = -z
    M[1, 3] = -1j * eps
    M[2, 2] = -np.conj(z)
    M[2, 3] = 1j * np.conj(eps)
    return M


def moment_recursion(u, dt, n_sub, delta, kappa, n0, A0):
    """RK4-discrete moments; returns (n_T, A_T, trajectory of n)."""
    u = np.asarray(u, dtype=np.float64)
    h = dt / n_sub
    v = np.array([n0, A0, np.conj(A0), 1.0], dtype=np.complex128)
    traj = [v[0].real]
    for j in range(u.shape[0]):
        P = rk4_poly_matrix(h * moment_matrix(u[j, 0], u[j, 1], delta, kappa))
        for _ in range(n_sub):
            v = P @ v
        traj.append(v[0].real)
    return v[0].real, v[1], np.array(traj)


def moment_fd_gradient(u, dt, n_sub, delta, kappa, n0, A0, step=1e-6):
    """Central finite differences of the RK4-discrete <n>(T) recursion."""
    u = np.array(u, dtype=np.float64)
    g = np.zeros_like(u)
    for j in range(u.shape[0]):
        for k in range(u.shape[1]):
            up = u.copy()
            up[j, k] += step
            dn = u.copy()
            dn[j, k] -= step
            g[j, k] = (moment_recursion(up, dt, n_sub, delta, kappa, n0, A0)[0]
                       - moment_recursion(dn, dt, n_sub, delta, kappa, n0, A0)[0]) / (2 * step)
    return g


def steady_state(ux, uy, delta, kappa):
    eps = ux + 1j * uy
    alpha = -1j * eps / (kappa / 2.0 + 1j * delta)
    n_ss = abs(eps) ** 2 / (delta ** 2 + kappa ** 2 / 4.0)
    return alpha, n_ss


def continuous_gradient_photon_number(u, dt, delta, kappa, A_T, first_order=False):
    """dn(T)/du[j, k] of the driven damped resonator (see module docstring)."""
    u = np.asarray(u, dtype=np.float64)
    n_t = u.shape[0]
    T = n_t * dt
    z = kappa / 2.0 + 1j * delta
    g = np.zeros((n_t, 2))
    w = dt if first_order else (1.0 - np.exp(-z * dt)) / z
    for j in range(n_t):
        prop = np.exp(-z * (T - (j + 1) * dt))
        g[j, 0] = 2.0 * (np.conj(A_T) * (-1j) * w * prop).real
        g[j, 1] = 2.0 * (np.conj(A_T) * w * prop).real
    return g
