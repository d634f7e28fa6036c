"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
the float64 oracle on the same seeded inputs, and the error metrics."""
from __future__ import annotations

import sys

import numpy as np

from oracle import rk

# Tolerances (normwise relative, against the float64 oracle).
TOL = {
    "f64": dict(rho=1e-12, phi=1e-12, grad=1e-10),
    "f32": dict(rho=1e-5, phi=1e-5, grad=1e-5),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grad_err(g, ref):
    """Error of a gradient [..., N_t, K] against the oracle's: the largest of
    the normwise relative error over all entries and that of every control
    channel k (relative to the channel's own norm, floored at 1e-3 of the
    whole gradient's norm for channels that are identically zero), so that a
    channel with a small share of the norm (the qubit drives at d = 240) is
    held to the same tolerance."""
    g = np.asarray(g)
    ref = np.asarray(ref)
    total = max(np.linalg.norm(ref), 1e-300)
    worst = float(np.linalg.norm(g - ref) / total)
    for k in range(ref.shape[-1]):
        den = max(np.linalg.norm(ref[..., k]), 1e-3 * total)
        worst = max(worst, float(np.linalg.norm(g[..., k] - ref[..., k]) / den))
    return worst


def phi_err(phi, ref, sigma_norm=1.0):
    return abs(phi - ref) / max(abs(ref), 1e-3 * sigma_norm)


def oracle_eval(w, u, mode="grape1", n_sub=1, sparse=False, rho0=None):
    m = rk.Model.from_workload(w, sparse=sparse)
    r0 = w.rho0 if rho0 is None else rho0
    phi, g, rhos = rk.cost_and_grad(m, u, r0, w.sigma, w.dt, n_sub=n_sub, mode=mode)
    return phi, g, rhos[-1]


def gpu_eval(w, u, *, prec="f64", path="auto", gmode="grape1", n_sub=1, ckpt_stride=0, rho0=None,
             validate=True, problem=None):
    """Returns (phi[B], grad[B, N_t, K], rho_T[B, d, d], problem) as numpy."""
    import torch

    from paper_1609_03170_amd import Problem

    dev = torch.device("cuda", 0)
    p = problem or Problem.from_workload(w, prec=prec, path=path, gmode=gmode, n_sub=n_sub,
                                         ckpt_stride=ckpt_stride, validate=validate)
    uu = np.asarray(u, dtype=np.float64)
    if uu.ndim == 2:
        uu = uu[None]
    r0 = w.rho0 if rho0 is None else rho0
    r0 = np.asarray(r0)
    if r0.ndim == 2:
        r0 = np.broadcast_to(r0, (uu.shape[0],) + r0.shape)
    ut = torch.tensor(uu, device=dev)
    rt = torch.tensor(np.ascontiguousarray(r0), device=dev)
    st = torch.tensor(w.sigma, device=dev)
    rhoT = p.forward(ut, rt, w.dt, want_rho_T=True)
    phi = p.cost(st)
    p.adjoint(st)
    g = p.gradient()
    torch.cuda.synchronize()
    return phi.cpu().numpy(), g.cpu().numpy(), rhoT.cpu().numpy(), p
