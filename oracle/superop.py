"""The standard Liouville-space open GRAPE that the paper replaces
(test infrastructure).

Sec. II.B: rho is written as a d^2 vector, the master equation as a
d^2 x d^2 matrix, and each slice propagator is the matrix exponential
L_j = exp(dt L_j) (Eqs. (5)-(7)).  Used here only as an independent check of
the Runge-Kutta path at small d (d <= 30).

Vectorisation is row-major: vec(Y)[i d + j] = Y[i, j], so that
vec(A Y B) = (A kron B^T) vec(Y).

The matrix exponential is this package's own: scaling and squaring with the
diagonal [q/q] Pade approximant, as in Golub and Van Loan, "Matrix
Computations", the algorithm for the Pade approximation of exp (scale so
that the infinity norm is at most 1/2, evaluate N/D with the recurrence for
the Pade coefficients, square back).  With q = 8 the a-priori relative
error bound 2^(3-2q) (q!)^2 / ((2q)! (2q+1)!) is below 1e-20.

Exact (continuous-time) gradients use Van Loan's block-triangular identity
    expm([[A, E], [0, A]]) = [[expm(A), Dexpm(A)[E]], [0, expm(A)]].
"""
from __future__ import annotations

import math

import numpy as np


def _dense(X):
    return np.asarray(X.todense()) if hasattr(X, "todense") else np.asarray(X)


def expm(A, q: int = 8):
    """exp(A) by scaling and squaring with the [q/q] Pade approximant."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    norm = np.max(np.sum(np.abs(A), axis=1)) if n else 0.0
    j = max(0, 1 + int(math.floor(math.log2(norm)))) if norm > 0 else 0
    As = A / (2.0 ** j)
    ident = np.eye(n, dtype=np.complex128)
    Nmat = ident.copy()
    Dmat = ident.copy()
    X = ident.copy()
    c = 1.0
    for k in range(1, q + 1):
        c = c * (q - k + 1) / ((2 * q - k + 1) * k)
        X = As @ X
        Nmat = Nmat + c * X
        Dmat = Dmat + ((-1) ** k) * c * X
    F = np.linalg.solve(Dmat, Nmat)
    for _ in range(j):
        F = F @ F
    return F


def superop_left_right(A, B):
    """Matrix of Y -> A Y B in the row-major vectorisation."""
    return np.kron(_dense(A), _dense(B).T)


def liouvillian(H, c_ops, gammas):
    """Eqs. (3)-(4) as a d^2 x d^2 matrix:
    -i (H x I - I x H^T) + sum_j gamma_j (a_j x conj(a_j)
        - (a_j^dag a_j x I + I x (a_j^dag a_j)^T) / 2)."""
    H = _dense(H)
    d = H.shape[0]
    ident = np.eye(d, dtype=np.complex128)
    L = -1j * (superop_left_right(H, ident) - superop_left_right(ident, H))
    for c, g in zip(c_ops, gammas):
        c = _dense(c)
        cdc = c.conj().T @ c
        L = L + g * (superop_left_right(c, c.conj().T)
                     - 0.5 * (superop_left_right(cdc, ident) + superop_left_right(ident, cdc)))
    return L


def commutator_superop(Hk):
    """Matrix of Y -> -i [H_k, Y]: the derivative of L with respect to u_k."""
    Hk = _dense(Hk)
    ident = np.eye(Hk.shape[0], dtype=np.complex128)
    return -1j * (superop_left_right(Hk, ident) - superop_left_right(ident, Hk))


def vec(Y):
    return np.asarray(Y, dtype=np.complex128).reshape(-1)


def unvec(v, d):
    return v.reshape(d, d)


def slice_propagators(model, u, dt):
    """E_j = exp(dt L_j) for every slice (Eq. (7))."""
    u = np.asarray(u, dtype=np.float64)
    return [expm(dt * liouvillian(model.hamiltonian(u[j]), model.c_ops, model.gammas))
            for j in range(u.shape[0])]


def forward(model, u, rho0, dt, props=None):
    """rho_j = E_j ... E_1 rho(0) (Eq. (10)); returns [rho_0 .. rho_N]."""
    d = model.d
    props = slice_propagators(model, u, dt) if props is None else props
    r = vec(rho0)
    out = [unvec(r.copy(), d)]
    for E in props:
        r = E @ r
        out.append(unvec(r.copy(), d))
    return out


def backward(model, u, sigma, dt, props=None):
    """lambda_j = E_{j+1}^dag ... E_N^dag sigma (Eq. (11)); [lambda_0 .. lambda_N]."""
    d = model.d
    props = slice_propagators(model, u, dt) if props is None else props
    n = len(props)
    lam = vec(_dense(sigma))
    out = [None] * (n + 1)
    out[n] = unvec(lam.copy(), d)
    for j in range(n - 1, -1, -1):
        lam = props[j].conj().T @ lam
        out[j] = unvec(lam.copy(), d)
    return out


def gradient_frechet(model, u, rhos, lams, dt):
    """Exact gradient of Phi = Tr(sigma E_N ... E_1 rho0) with respect to u[j, k]:
    dPhi/du[j,k] = <vec lambda_{j+1}, Dexpm(dt L_j)[dt C_k] vec rho_j>, with the
    Frechet derivative taken from Van Loan's block exponential."""
    u = np.asarray(u, dtype=np.float64)
    n_t, K = u.shape
    g = np.zeros((n_t, K))
    Cs = [commutator_superop(H) for H in model.Hk]
    for j in range(n_t):
        A = dt * liouvillian(model.hamiltonian(u[j]), model.c_ops, model.gammas)
        n = A.shape[0]
        for k in range(K):
            M = np.zeros((2 * n, 2 * n), dtype=np.complex128)
            M[:n, :n] = A
            M[n:, n:] = A
            M[:n, n:] = dt * Cs[k]
            F = expm(M)[:n, n:]
            g[j, k] = np.vdot(vec(lams[j + 1]), F @ vec(rhos[j])).real
    return g
