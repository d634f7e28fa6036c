"""Synthetic cQED-shaped workloads (operators, states, targets, controls).

The paper's numerical examples are physical models with printed parameters:
a damped driven resonator (Sec. IV.A, Eqs. (18)-(21)), the dispersive
transmon-resonator system with Kerr non-linearity and two-quadrature drive
(Sec. IV.B, Eq. (23)), and the Jaynes-Cummings scaling test of Fig. 2.  No
dataset is involved.  The generators below produce seeded stand-ins with the
same structure: ladder operators on a truncated Fock space, a transmon of
n_q levels tensored with the resonator (basis index q*N + n), I/Q drives,
cavity damping, coherent initial states.  A dense random family (GUE/Ginibre
operators, Wishart initial state) covers the general, unstructured case.

Conventions fixed here (readings of points the paper leaves open):
  * A truncated coherent state uses c_n = exp(-|a|^2/2) a^n / sqrt(n!) for
    n < N and is renormalised.
  * The multi-level transmon replaces the two-level dispersive term
    chi*sigma_z*a^dag a of Eq. (18) by chi * a^dag a * b^dag b, works in the
    frame rotating with both modes, and adds (alpha_q/2) b^dag b^dag b b.
    The Kerr term is K (a^dag a)^2 as in Eq. (21).
  * The resonator drive is u_x (a + a^dag) + u_y i (a^dag - a) (Eq. (23)),
    the qubit drive the same with b.
  * "Leakage" is the projector on transmon levels >= 2.
All arrays are complex128 / float64 numpy arrays, row-major.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One open-GRAPE evaluation problem: H(t) = H0 + sum_k u_k(t) H_k with
    Lindblad channels gamma_m D[c_m] (Eqs. (1), (3), (4)), initial state
    rho0, target/observable sigma (Eq. (8)), N_t slices of length dt."""

    name: str
    H0: np.ndarray            # (d, d) complex128, Hermitian
    Hk: np.ndarray            # (K, d, d) complex128, Hermitian
    c_ops: np.ndarray         # (J, d, d) complex128
    gammas: np.ndarray        # (J,) float64, >= 0
    rho0: np.ndarray          # (d, d) or (B, d, d) complex128
    sigma: np.ndarray         # (d, d) complex128, Hermitian
    dt: float
    u: np.ndarray             # (N_t, K) or (B, N_t, K) float64
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return self.H0.shape[0]

    @property
    def K(self) -> int:
        return self.Hk.shape[0]

    @property
    def J(self) -> int:
        return self.c_ops.shape[0]

    @property
    def n_t(self) -> int:
        return self.u.shape[-2]


# ----------------------------------------------------------------------------
# Building blocks
# ----------------------------------------------------------------------------

def destroy(n: int) -> np.ndarray:
    """Truncated annihilation operator: a|m> = sqrt(m)|m-1>."""
    a = np.zeros((n, n), dtype=np.complex128)
    for m in range(1, n):
        a[m - 1, m] = math.sqrt(m)
    return a


def coherent_ket(n: int, alpha: complex) -> np.ndarray:
    """Truncated, renormalised coherent state |alpha> on n Fock levels."""
    c = np.zeros(n, dtype=np.complex128)
    logfact = 0.0
    for m in range(n):
        if m > 0:
            logfact += math.log(m)
        if alpha == 0:
            c[m] = 1.0 if m == 0 else 0.0
            continue
        mag = math.exp(-abs(alpha) ** 2 / 2 + m * math.log(abs(alpha)) - 0.5 * logfact)
        c[m] = mag * np.exp(1j * m * np.angle(alpha))
    return c / np.linalg.norm(c)


def _dm(ket: np.ndarray) -> np.ndarray:
    return np.outer(ket, ket.conj())


def _basis(n: int, k: int) -> np.ndarray:
    v = np.zeros(n, dtype=np.complex128)
    v[k] = 1.0
    return v


def controls_uniform(seed: int, n_t: int, K: int, scale=1.0, batch: int | None = None) -> np.ndarray:
    """u ~ U[-1, 1] * scale (scale may be a per-channel vector)."""
    rng = np.random.default_rng(seed)
    shape = (n_t, K) if batch is None else (batch, n_t, K)
    return rng.uniform(-1.0, 1.0, size=shape) * np.asarray(scale, dtype=np.float64)


def controls_smooth_noise(seed: int, n_t: int, rms, sigma_t: float = 25.0) -> np.ndarray:
    """Smooth Gaussian-filtered noise controls.

    iid N(0, 1) samples per channel, convolved along time with a Gaussian of
    standard deviation sigma_t slices (support +-4 sigma_t, reflect padding),
    then rescaled so each channel has the requested RMS.
    """
    rms = np.asarray(rms, dtype=np.float64)
    K = rms.shape[0]
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n_t, K))
    half = int(math.ceil(4 * sigma_t))
    t = np.arange(-half, half + 1, dtype=np.float64)
    kern = np.exp(-0.5 * (t / sigma_t) ** 2)
    kern /= kern.sum()
    out = np.empty_like(white)
    for k in range(K):
        padded = np.pad(white[:, k], half, mode="reflect") if n_t > half else np.pad(
            white[:, k], half, mode="wrap")
        out[:, k] = np.convolve(padded, kern, mode="valid")[:n_t]
        cur = math.sqrt(np.mean(out[:, k] ** 2))
        out[:, k] *= rms[k] / cur if cur > 0 else 0.0
    return out


# ----------------------------------------------------------------------------
# Model families
# ----------------------------------------------------------------------------

def resonator_problem(N: int, delta: float, kappa: float, alpha: complex,
                      u: np.ndarray, dt: float, name: str = "resonator") -> Workload:
    """Damped driven resonator (Eqs. (19), (20), (23)): H = delta a^dag a +
    u_x (a + a^dag) + u_y i (a^dag - a), collapse kappa D[a], rho0 = |alpha><alpha|,
    sigma = a^dag a."""
    a = destroy(N)
    ad = a.conj().T
    n_op = ad @ a
    H0 = delta * n_op
    Hk = np.stack([a + ad, 1j * (ad - a)])
    c_ops = a[None, :, :].copy()
    gammas = np.array([kappa], dtype=np.float64)
    rho0 = _dm(coherent_ket(N, alpha))
    return Workload(name, H0, Hk, c_ops, gammas, rho0, n_op.copy(), dt, u,
                    meta=dict(N=N, delta=delta, kappa=kappa, alpha=alpha))


def transmon_resonator_problem(n_q: int, N: int, *, chi: float = -2.0, kerr: float = -0.01,
                               anharm: float = -100.0, kappa: float = 1.0,
                               gamma1: float = 0.01, gamma_phi: float = 0.005,
                               alpha: complex = 3.0, qubit_drive: bool = False,
                               u: np.ndarray | None = None, dt: float = 0.01,
                               name: str = "transmon_resonator") -> Workload:
    """Transmon (n_q levels, operator b) x resonator (N levels, operator a),
    basis index q*N + n.  H0 = chi a^dag a b^dag b + K (a^dag a)^2 +
    (anharm/2) b^dag b^dag b b (diagonal in this basis).  Controls: resonator
    I/Q and, if qubit_drive, transmon I/Q.  Collapses sqrt(kappa) a,
    sqrt(gamma1) b, sqrt(gamma_phi) b^dag b.  rho0 = |1><1| x |alpha><alpha|,
    sigma = a^dag a + P_(q>=2)."""
    Iq = np.eye(n_q, dtype=np.complex128)
    In = np.eye(N, dtype=np.complex128)
    a = np.kron(Iq, destroy(N))
    b = np.kron(destroy(n_q), In)
    ad, bd = a.conj().T, b.conj().T
    na, nb = ad @ a, bd @ b
    H0 = chi * na @ nb + kerr * na @ na + 0.5 * anharm * (bd @ bd @ b @ b)
    ctrl = [a + ad, 1j * (ad - a)]
    if qubit_drive:
        ctrl += [b + bd, 1j * (bd - b)]
    Hk = np.stack(ctrl)
    c_ops = np.stack([a, b, nb])
    gammas = np.array([kappa, gamma1, gamma_phi], dtype=np.float64)
    qstate = _basis(n_q, 1) if n_q > 1 else _basis(n_q, 0)
    rho0 = np.kron(_dm(qstate), _dm(coherent_ket(N, alpha)))
    pf = np.zeros((n_q, n_q), dtype=np.complex128)
    for q in range(2, n_q):
        pf[q, q] = 1.0
    sigma = na + np.kron(pf, In)
    if u is None:
        u = np.zeros((1, len(ctrl)))
    return Workload(name, H0, Hk, c_ops, gammas, rho0, sigma, dt, u,
                    meta=dict(n_q=n_q, N=N, chi=chi, kerr=kerr, anharm=anharm, kappa=kappa,
                              gamma1=gamma1, gamma_phi=gamma_phi, alpha=alpha))


def _ginibre(rng, d):
    return (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)


def _spectral_norm(M):
    return float(np.linalg.norm(M, 2))


def dense_random_problem(d: int = 512, K: int = 4, J: int = 4, n_t: int = 1000, dt: float = 0.005,
                         seeds=(3, 4, 5, 6, 7, 8), rank: int = 8, name: str = "dense_random") -> Workload:
    """General dense problem: H0 Hermitian with spectral radius 10, K random
    Hermitian controls of spectral norm 1, J Ginibre collapse operators of
    spectral norm 1 with rates U[0.01, 0.1], rho0 = W W^dag / Tr (W d x rank
    complex Gaussian), sigma Hermitian of spectral norm 1, u ~ U[-1, 1]."""
    s_h0, s_hk, s_c, s_rho, s_sig, s_u = seeds
    rng = np.random.default_rng(s_h0)
    X = _ginibre(rng, d)
    A = 0.5 * (X + X.conj().T)
    H0 = 10.0 * A / np.max(np.abs(np.linalg.eigvalsh(A)))
    rng = np.random.default_rng(s_hk)
    Hk = []
    for _ in range(K):
        X = _ginibre(rng, d)
        A = 0.5 * (X + X.conj().T)
        Hk.append(A / _spectral_norm(A))
    Hk = np.stack(Hk)
    rng = np.random.default_rng(s_c)
    cs = []
    for _ in range(J):
        X = _ginibre(rng, d)
        cs.append(X / _spectral_norm(X))
    c_ops = np.stack(cs)
    gammas = rng.uniform(0.01, 0.1, size=J)
    rng = np.random.default_rng(s_rho)
    W = (rng.standard_normal((d, rank)) + 1j * rng.standard_normal((d, rank))) / math.sqrt(2.0)
    rho0 = W @ W.conj().T
    rho0 /= np.trace(rho0).real
    rng = np.random.default_rng(s_sig)
    X = _ginibre(rng, d)
    A = 0.5 * (X + X.conj().T)
    sigma = A / _spectral_norm(A)
    u = controls_uniform(s_u, n_t, K)
    return Workload(name, H0, Hk, c_ops, gammas, rho0, sigma, dt, u, meta=dict(seeds=seeds))


def _banded(rng, d, offsets, hermitian):
    """Random matrix whose nonzeros lie on the given diagonals (offset o:
    entries (i, i + o)); Hermitian ones get each diagonal pair conjugate."""
    M = np.zeros((d, d), dtype=np.complex128)
    for o in sorted(set(offsets)):
        if hermitian and o < 0:
            continue
        n = d - abs(o)
        if n <= 0:
            continue
        v = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
        i = np.arange(n) if o >= 0 else np.arange(-o, d)
        if hermitian and o == 0:
            v = v.real.astype(np.complex128)
        M[i, i + o] = v
        if hermitian and o > 0:
            M[i + o, i] = v.conj()
    return M


def banded_random_problem(d: int, h_offsets, hk_offsets, c_offsets, K: int = 2, n_t: int = 12,
                          dt: float = 0.01, seeds=(21, 22, 23, 24, 25, 26), name: str = "banded_random") -> Workload:
    """Operators with prescribed diagonals and random entries, for the stage
    kernels' tap layouts: H0 Hermitian on the offsets +-h_offsets (spectral
    norm 5), K Hermitian controls on +-hk_offsets (norm 1), one collapse
    operator per entry of c_offsets, each on its own list of diagonals (norm
    1, rate U[0.05, 0.2]), rho0 of rank 4, sigma Hermitian of norm 1,
    u ~ U[-1, 1]."""
    s_h0, s_hk, s_c, s_rho, s_sig, s_u = seeds
    sym = lambda offs: sorted({o for x in offs for o in (x, -x)})
    rng = np.random.default_rng(s_h0)
    H0 = _banded(rng, d, sym(h_offsets), True)
    H0 *= 5.0 / _spectral_norm(H0)
    rng = np.random.default_rng(s_hk)
    Hk = np.stack([_banded(rng, d, sym(hk_offsets), True) for _ in range(K)])
    Hk /= np.array([_spectral_norm(h) for h in Hk])[:, None, None]
    rng = np.random.default_rng(s_c)
    cs = [_banded(rng, d, offs, False) for offs in c_offsets]
    c_ops = np.stack([c / _spectral_norm(c) for c in cs])
    gammas = rng.uniform(0.05, 0.2, size=len(cs))
    rng = np.random.default_rng(s_rho)
    W = (rng.standard_normal((d, 4)) + 1j * rng.standard_normal((d, 4))) / math.sqrt(2.0)
    rho0 = W @ W.conj().T
    rho0 /= np.trace(rho0).real
    rng = np.random.default_rng(s_sig)
    X = _ginibre(rng, d)
    A = 0.5 * (X + X.conj().T)
    sigma = A / _spectral_norm(A)
    u = controls_uniform(s_u, n_t, K)
    return Workload(name, H0, Hk, c_ops, gammas, rho0, sigma, dt, u, meta=dict(seeds=seeds))


# ----------------------------------------------------------------------------
# The five named configurations
# ----------------------------------------------------------------------------

def config_c1() -> Workload:
    """d = 10 damped driven resonator, Delta = 0.5 kappa, alpha = 2, N_t = 200,
    dt = 0.05/kappa, u ~ U[-1, 1] (seed 0), sigma = a^dag a."""
    u = controls_uniform(0, 200, 2)
    return resonator_problem(10, 0.5, 1.0, 2.0, u, 0.05, name="C1_resonator_d10")


def config_c2() -> Workload:
    """3-level transmon x resonator N = 30 (d = 90), resonator I/Q drive,
    N_t = 2000, dt = 0.01/kappa, u ~ U[-1, 1] (seed 1)."""
    u = controls_uniform(1, 2000, 2)
    return transmon_resonator_problem(3, 30, u=u, dt=0.01, name="C2_cqed_d90")


C3_RMS = (1.0, 1.0, 0.2, 0.2)


def config_c3(batch: int = 1, n_t: int = 10000, dt: float = 0.002, N: int = 80, n_q: int = 3,
              seed0: int = 2) -> Workload:
    """3-level transmon x resonator N = 80 (d = 240), 4 controls (resonator
    I/Q, qubit I/Q) as smooth Gaussian-filtered noise, N_t = 10000,
    dt = 0.002/kappa.  Problem b of a batch uses seed seed0 + b."""
    us = np.stack([controls_smooth_noise(seed0 + b, n_t, C3_RMS) for b in range(batch)])
    w = transmon_resonator_problem(n_q, N, qubit_drive=True, u=us if batch > 1 else us[0], dt=dt,
                                   name=f"C3_cqed_d{n_q * N}")
    w.meta["batch"] = batch
    return w


def config_c4(n_t: int = 1000, d: int = 512) -> Workload:
    """Dense random d = 512, K = 4, J = 4, N_t = 1000, dt = 0.005."""
    return dense_random_problem(d=d, n_t=n_t, name=f"C4_dense_d{d}")


SERVING_SHAPES = ((2, 10), (2, 20), (3, 30), (2, 80), (3, 80))
SERVING_SCALE = (1.0, 1.0, 0.2, 0.2)


def serving_requests(n_requests: int = 4096, seed: int = 10, arrival_seed: int = 9,
                     rate: float = 1.0, n_t_range=(500, 5000), dt: float = 0.002):
    """Serving stream: each request draws (n_q, N) uniformly from
    SERVING_SHAPES (d in {20, 40, 90, 160, 240}), N_t ~ U{500..5000}, controls
    u ~ U[-1, 1] * (1, 1, 0.2, 0.2), and arrives by a Poisson process of the
    given rate (requests per unit time).  Returns a list of dicts with keys
    shape, n_t, u, arrival (the controls are generated lazily per request
    seed so that a small sample is cheap)."""
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(arrival_seed)
    gaps = arr.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_requests):
        shape = SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))]
        n_t = int(rng.integers(n_t_range[0], n_t_range[1] + 1))
        useed = int(rng.integers(2**31 - 1))
        reqs.append(dict(id=i, shape=shape, n_t=n_t, u_seed=useed, arrival=float(arrivals[i]), dt=dt))
    return reqs


def serving_model(shape) -> Workload:
    """The operator set for one serving shape (n_q, N): qubit and resonator
    I/Q drives, alpha = sqrt(N/8)."""
    n_q, N = shape
    return transmon_resonator_problem(n_q, N, qubit_drive=True, alpha=math.sqrt(N / 8.0),
                                      dt=0.002, name=f"serve_{n_q}x{N}")


def serving_controls(req) -> np.ndarray:
    return controls_uniform(req["u_seed"], req["n_t"], 4, scale=SERVING_SCALE)
