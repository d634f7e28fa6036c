"""Adaptive-step integration of the slices (test infrastructure; plain
float64, written from the published method).

The paper integrates every slice with a standard adaptive Runge-Kutta
routine (Sec. III.A).  Here that is the embedded pair of Dormand and Prince
(J. Comput. Appl. Math. 6 (1980) 19): seven stages, a fifth-order solution
that is propagated and a fourth-order companion whose difference estimates
the local error, with the usual step-size control (Hairer, Norsett and
Wanner, Solving Ordinary Differential Equations I, Sec. II.4).

Within slice j the generator is constant (Eq. (1) with u[j]), so the stage
times c_i play no role.  From t_rem = dt:
    h_use = min(h, t_rem)
    k_1 = f(y),  k_i = f(y + h_use sum_{l<i} A[i][l] k_l)        i = 2..7
    y5  = y + h_use sum_i B[i] k_i
    e   = h_use sum_i E[i] k_i                                    (E = B - Bhat)
    sc  = atol + rtol max(|y|, |y5|), per real component (real and
          imaginary parts of every matrix element are separate components)
    err = sqrt(mean((e / sc)^2))
    accept when err <= 1: y = y5, t_rem = t_rem - h_use (exactly 0 when the
    step was clipped to t_rem); the next proposal is
        h = h_use min(fmax, max(0.2, 0.9 err^(-1/5)))
    with fmax = 1 right after a rejected attempt, else 5 (err = 0 gives fmax);
    on rejection  h = h_use max(0.2, 0.9 err^(-1/5)).
The proposal h and the "last attempt rejected" flag carry over from slice
to slice; the first slice starts with h = dt.  The backward sweep
integrates L^dag from lambda_N = sigma (Eq. (11)) with its own controller,
and the first-order gradient of Eq. (13) pairs rho_{j+1} with
lambda_{j+1}, as for fixed steps.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np

from . import rk

# Dormand-Prince 5(4) coefficients (exact rationals).
A = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
C = [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)]
B = [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0)]
BHAT = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200), F(187, 2100), F(1, 40)]
E = [b - bh for b, bh in zip(B, BHAT)]

FAC, FACMIN, FACMAX = 0.9, 0.2, 5.0
MAX_ATTEMPTS = 100000


def dopri_stages(f, y, h):
    """The seven stage derivatives of one attempt of size h."""
    ks = [f(y)]
    for i in range(1, 7):
        yi = y.copy()
        for l, a in enumerate(A[i]):
            if a != 0:
                yi = yi + (h * float(a)) * ks[l]
        ks.append(f(yi))
    return ks


def dopri_fixed(f, y, h, n):
    """n steps of the fifth-order solution with a fixed step h (no control)."""
    for _ in range(n):
        ks = dopri_stages(f, y, h)
        y = y + h * sum(float(b) * k for b, k in zip(B, ks))
    return y


class Controller:
    """Step-size state carried across the slices of one sweep."""

    def __init__(self, h0, rtol, atol):
        self.h = float(h0)
        self.rtol, self.atol = float(rtol), float(atol)
        self.rejected_last = False
        self.accepted = 0
        self.rejected = 0

    def error(self, y, y5, e):
        sc = self.atol + self.rtol * np.maximum(np.abs(np.concatenate([y.real.ravel(), y.imag.ravel()])),
                                                np.abs(np.concatenate([y5.real.ravel(), y5.imag.ravel()])))
        ev = np.concatenate([e.real.ravel(), e.imag.ravel()]) / sc
        return float(np.sqrt(np.mean(ev * ev)))

    def factor(self, err, fmax):
        if err == 0.0:
            return fmax
        return min(fmax, max(FACMIN, FAC * err ** (-0.2)))

    def slice(self, f, y, dt):
        """Integrate one slice of length dt from y; returns the end state."""
        t_rem = float(dt)
        attempts = 0
        while t_rem > 0.0:
            attempts += 1
            if attempts > MAX_ATTEMPTS:
                raise RuntimeError("step size control did not finish the slice")
            clipped = self.h >= t_rem
            h_use = t_rem if clipped else self.h
            ks = dopri_stages(f, y, h_use)
            y5 = y + h_use * sum(float(b) * k for b, k in zip(B, ks))
            e = h_use * sum(float(c) * k for c, k in zip(E, ks))
            err = self.error(y, y5, e)
            if err <= 1.0:
                y = y5
                t_rem = 0.0 if clipped else t_rem - h_use
                self.h = h_use * self.factor(err, 1.0 if self.rejected_last else FACMAX)
                self.rejected_last = False
                self.accepted += 1
            else:
                self.h = h_use * max(FACMIN, FAC * err ** (-0.2))
                self.rejected_last = True
                self.rejected += 1
        return y


def forward(model, u, rho0, dt, rtol, atol):
    """Adaptive forward sweep; returns ([rho_0 .. rho_N], controller)."""
    u = np.asarray(u, dtype=np.float64)
    ctl = Controller(dt, rtol, atol)
    rho = np.array(rho0, dtype=np.complex128)
    rhos = [rho]
    for j in range(u.shape[0]):
        H = model.hamiltonian(u[j])
        rho = ctl.slice(lambda Y, H=H: rk.lindblad(model, H, Y), rho, dt)
        rhos.append(rho)
    return rhos, ctl


def backward(model, u, sigma, dt, rtol, atol):
    """Adaptive backward sweep of Eq. (11) with L^dag; ([lambda_0 .. lambda_N], controller)."""
    u = np.asarray(u, dtype=np.float64)
    n_t = u.shape[0]
    ctl = Controller(dt, rtol, atol)
    lam = np.array(rk._dense(sigma), dtype=np.complex128)
    lams = [None] * (n_t + 1)
    lams[n_t] = lam
    for j in range(n_t - 1, -1, -1):
        H = model.hamiltonian(u[j])
        lam = ctl.slice(lambda X, H=H: rk.lindblad_adjoint(model, H, X), lam, dt)
        lams[j] = lam
    return lams, ctl


def cost_and_grad(model, u, rho0, sigma, dt, rtol, atol):
    """Phi and the first-order gradient (Eq. (13)) with adaptive sweeps.
    Returns (phi, g, rhos, (forward controller, backward controller))."""
    rhos, cf = forward(model, u, rho0, dt, rtol, atol)
    lams, cb = backward(model, u, sigma, dt, rtol, atol)
    phi = rk.cost(sigma, rhos[-1])
    g = rk.gradient_grape1(model, u, rhos, lams, dt)
    return phi, g, rhos, (cf, cb)
