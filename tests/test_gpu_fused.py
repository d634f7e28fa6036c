"""The fused RK4 step (four nested stages per launch on tiles of the
multi-level x oscillator structure, d = nq N) against the float64 oracle,
over the tile geometries it meets: one level (nq = 1, a bare resonator,
one tile and a ragged 1-D tiling), two to four levels, windows clipped at
both ends of the n range, several tiles per axis with ragged blocks;
substeps (n_sub = 2, 3), checkpoints with a resident tail, the exact
gradient (its forward sweep fused, its stage recomputation not), and a
batch whose problems differ; then fused against the four stage kernels on
the same inputs, bitwise repeatability, and the structures it must refuse."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, grad_err, oracle_eval, phi_err, relerr, say

pytestmark = pytest.mark.gpu


def _problem(w, prec, gmode="grape1", n_sub=1, ckpt_stride=0, fused=True):
    from paper_1609_03170_amd import Problem

    p = Problem.from_workload(w, prec=prec, path="banded", gmode=gmode, n_sub=n_sub, ckpt_stride=ckpt_stride)
    p.set_fused(fused)
    return p


def _cqed(n_q, N, n_t, batch=1, seed=5, dt=0.002):
    us = np.stack([wl.controls_uniform(seed + b, n_t, 4) * np.array([1.0, 1.0, 0.2, 0.2]) for b in range(batch)])
    return wl.transmon_resonator_problem(n_q, N, qubit_drive=True, u=us if batch > 1 else us[0], dt=dt,
                                         alpha=np.sqrt(N / 8.0), name=f"cqed_{n_q}x{N}")


GEOMETRIES = {
    "resonator_d10": lambda: wl.resonator_problem(10, 0.5, 1.0, 2.0, wl.controls_uniform(3, 17, 2), 0.05),
    "resonator_d130_3tiles": lambda: wl.resonator_problem(130, 0.5, 1.0, 3.0, wl.controls_uniform(4, 9, 2), 0.002),
    "cqed_2x10": lambda: _cqed(2, 10, 15),
    "cqed_3x20_2tiles": lambda: _cqed(3, 20, 13),
    "cqed_3x37_ragged": lambda: _cqed(3, 37, 11),
    "cqed_4x12": lambda: _cqed(4, 12, 9),
}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom", list(GEOMETRIES))
def test_fused_geometries_against_oracle(geom, prec):
    w = GEOMETRIES[geom]()
    p = _problem(w, prec)
    say(f"[case] fused {geom} d={w.d} prec={prec}")
    assert p.fused, "the workload has the multi-level x oscillator structure"
    phi, g, rhoT, p = gpu_eval(w, w.u, problem=p)
    p.close()
    phi_r, g_r, rho_r = oracle_eval(w, w.u, sparse=w.d > 60)
    tol = TOL[prec]
    e_phi, e_g, e_rho = phi_err(phi[0], phi_r), grad_err(g[0], g_r), relerr(rhoT[0], rho_r)
    say(f"   phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
    assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]
    assert np.array_equal(rhoT[0], rhoT[0].conj().T)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n_sub", [2, 3])
def test_fused_substeps_checkpoints_resident(prec, n_sub):
    w = _cqed(3, 20, 23, batch=3)
    say(f"[case] fused cqed_3x20 B=3 n_sub={n_sub} stride=4 resident=7 prec={prec}")
    p = _problem(w, prec, n_sub=n_sub, ckpt_stride=4)
    p.set_resident(7)
    phi, g, rhoT, p = gpu_eval(w, w.u, problem=p, n_sub=n_sub)
    p.close()
    tol = TOL[prec]
    for b in range(3):
        phi_r, g_r, rho_r = oracle_eval(w, w.u[b], n_sub=n_sub)
        e_phi, e_g, e_rho = phi_err(phi[b], phi_r), grad_err(g[b], g_r), relerr(rhoT[b], rho_r)
        say(f"   problem {b}: phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
        assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_forward_exact_gradient(prec):
    w = _cqed(3, 20, 12)
    say(f"[case] fused cqed_3x20 exact gradient prec={prec}")
    p = _problem(w, prec, gmode="exact")
    phi, g, rhoT, p = gpu_eval(w, w.u, problem=p)
    p.close()
    phi_r, g_r, rho_r = oracle_eval(w, w.u, mode="exact")
    tol = TOL[prec]
    e_phi, e_g = phi_err(phi[0], phi_r), grad_err(g[0], g_r)
    say(f"   phi {e_phi:.2e} grad {e_g:.2e}")
    assert e_phi < tol["phi"] and e_g < tol["grad"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_against_stage_kernels_and_repeatable(prec):
    w = _cqed(3, 37, 40, batch=5)
    say(f"[case] fused vs four stage kernels cqed_3x37 B=5 prec={prec}")
    pf = _problem(w, prec)
    phi_f, g_f, rho_f, pf = gpu_eval(w, w.u, problem=pf)
    phi_f2, g_f2, rho_f2, pf = gpu_eval(w, w.u, problem=pf)
    pf.close()
    assert np.array_equal(phi_f, phi_f2) and np.array_equal(g_f, g_f2) and np.array_equal(rho_f, rho_f2)
    ps = _problem(w, prec, fused=False)
    assert not ps.fused
    phi_s, g_s, rho_s, ps = gpu_eval(w, w.u, problem=ps)
    ps.close()
    tol = TOL[prec]
    for b in range(5):
        e = (phi_err(phi_f[b], phi_s[b]), grad_err(g_f[b], g_s[b]), relerr(rho_f[b], rho_s[b]))
        say(f"   problem {b}: fused vs stages phi {e[0]:.2e} grad {e[1]:.2e} rho {e[2]:.2e}")
        assert e[0] < tol["phi"] and e[1] < tol["grad"] and e[2] < tol["rho"]


def test_fused_refused_outside_the_structure():
    """Operators outside the structure run the four stage kernels: a +1
    coupling across the blocks of N, and a diagonal at +-2."""
    w = _cqed(3, 10, 4)
    H0 = w.H0.copy()
    H0[9, 10] = H0[10, 9] = 0.3  # couples n = N - 1 of level 0 to n = 0 of level 1
    w2 = wl.Workload("cross", H0, w.Hk, w.c_ops, w.gammas, w.rho0, w.sigma, w.dt, w.u)
    w3 = wl.banded_random_problem(30, [0, 2], [1], [[1]], K=2, n_t=4, dt=0.01)
    for ww in (w2, w3):
        p = _problem(ww, "f64")
        assert not p.fused
        phi, g, rhoT, p = gpu_eval(ww, ww.u, problem=p)
        p.close()
        phi_r, g_r, _ = oracle_eval(ww, ww.u)
        assert phi_err(phi[0], phi_r) < 1e-12 and grad_err(g[0], g_r) < 1e-10
