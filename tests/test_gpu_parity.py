"""Parity of the HIP path (through the C ABI) with the float64 oracle on the
same seeded inputs, element by element / normwise, at sizes the oracle
finishes in seconds; several tiles and ragged tails are covered."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, oracle_eval, phi_err, grad_err, relerr, say

pytestmark = pytest.mark.gpu


def _check(w, u, prec, path, gmode, n_sub=1, sparse=False, tag="", B_rho0=None, **kw):
    say(f"[case] {tag} d={w.d} K={w.K} J={w.J} N_t={np.asarray(u).shape[-2]} prec={prec} path={path} "
        f"gmode={gmode} n_sub={n_sub} {kw}")
    phi, g, rhoT, p = gpu_eval(w, u, prec=prec, path=path, gmode=gmode, n_sub=n_sub, **kw)
    assert path == "auto" or p.path == path
    uu = np.asarray(u)
    if uu.ndim == 2:
        uu = uu[None]
    tol = TOL[prec]
    for b in range(uu.shape[0]):
        phi_r, g_r, rho_r = oracle_eval(w, uu[b], mode=gmode, n_sub=n_sub, sparse=sparse)
        e_rho, e_phi, e_g = relerr(rhoT[b], rho_r), phi_err(phi[b], phi_r), grad_err(g[b], g_r)
        say(f"   b={b} rho {e_rho:.2e} phi {e_phi:.2e} grad {e_g:.2e}")
        assert e_rho < tol["rho"]
        assert e_phi < tol["phi"]
        assert e_g < tol["grad"]
        # exact Hermiticity of the returned state
        assert np.array_equal(rhoT[b], rhoT[b].conj().T)
    p.close()
    return phi, g


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("path", ["banded", "dense"])
@pytest.mark.parametrize("gmode", ["grape1", "exact"])
def test_c1_resonator_d10(prec, path, gmode):
    w = wl.config_c1()
    _check(w, w.u, prec, path, gmode, tag="C1")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("path", ["banded", "dense"])
def test_c2_cqed_d90_reduced(prec, path):
    w = wl.config_c2()
    _check(w, w.u[:150], prec, path, "grape1", tag="C2[:150]")


def test_c2_exact_banded_f64():
    w = wl.config_c2()
    _check(w, w.u[:40], "f64", "banded", "exact", tag="C2[:40]")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("gmode", ["grape1", "exact"])
def test_c3_cqed_d240_batch(prec, gmode):
    w = wl.config_c3(batch=2, n_t=24)
    _check(w, w.u, prec, "banded", gmode, sparse=True, tag="C3-shape B=2")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("gmode", ["grape1", "exact"])
def test_dense_random_ragged_d70(prec, gmode):
    w = wl.dense_random_problem(d=70, K=3, J=2, n_t=12, dt=0.005, seeds=(31, 32, 33, 34, 35, 36))
    u = wl.controls_uniform(37, 12, 3, batch=2)
    _check(w, u, prec, "dense", gmode, tag="dense d=70 B=2")


@pytest.mark.parametrize("prec,bound_phi,bound_g", [("bf16x3", 1e-4, 2e-3), ("f16x3", 1e-5, 1e-4)])
@pytest.mark.parametrize("gmode", ["grape1", "exact"])
def test_dense_split_precision_ragged_d70(prec, bound_phi, bound_g, gmode):
    """16-bit split GEMMs: the error is reported per result; the bounds only
    catch a broken split (a dropped term costs orders of magnitude more)."""
    w = wl.dense_random_problem(d=70, K=3, J=2, n_t=12, dt=0.005, seeds=(31, 32, 33, 34, 35, 36))
    u = wl.controls_uniform(37, 12, 3, batch=2)
    say(f"[case] dense d=70 B=2 prec={prec} gmode={gmode}")
    phi, g, rhoT, p = gpu_eval(w, u, prec=prec, path="dense", gmode=gmode)
    p.close()
    for b in range(2):
        phi_r, g_r, rho_r = oracle_eval(w, u[b], mode=gmode)
        e_phi, e_g, e_rho = phi_err(phi[b], phi_r), grad_err(g[b], g_r), relerr(rhoT[b], rho_r)
        say(f"   b={b} rho {e_rho:.2e} phi {e_phi:.2e} grad {e_g:.2e}")
        assert e_phi < bound_phi and e_g < bound_g
        assert np.array_equal(rhoT[b], rhoT[b].conj().T)


def test_n_sub_two_exact():
    w = wl.config_c1()
    _check(w, w.u[:60], "f64", "banded", "exact", n_sub=2, tag="C1 n_sub=2")
    _check(w, w.u[:60], "f64", "dense", "grape1", n_sub=3, tag="C1 n_sub=3")


@pytest.mark.parametrize("path", ["banded", "dense"])
def test_checkpoint_stride_does_not_change_results(path):
    w = wl.config_c1()
    outs = []
    for s in (1, 7, 200, 0):
        say(f"[case] C1 ckpt_stride={s} path={path}")
        phi, g, rhoT, p = gpu_eval(w, w.u, prec="f32", path=path, gmode="exact", ckpt_stride=s)
        p.close()
        outs.append((phi, g))
    for phi, g in outs[1:]:
        assert np.array_equal(phi, outs[0][0])
        assert np.array_equal(g, outs[0][1])


def test_determinism_bitwise():
    w = wl.config_c3(batch=3, n_t=10)
    say("[case] C3-shape determinism B=3")
    a = gpu_eval(w, w.u, prec="f32", path="banded", gmode="grape1")
    b = gpu_eval(w, w.u, prec="f32", path="banded", gmode="grape1", problem=a[3])
    a[3].close()
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_batch_member_equals_alone():
    w = wl.config_c3(batch=3, n_t=8)
    say("[case] C3-shape batch vs alone")
    phi, g, rhoT, p = gpu_eval(w, w.u, prec="f32", path="banded", gmode="exact")
    p.close()
    phi1, g1, rhoT1, p1 = gpu_eval(w, w.u[1], prec="f32", path="banded", gmode="exact")
    p1.close()
    assert np.array_equal(phi[1], phi1[0])
    assert np.array_equal(g[1], g1[0])


def test_single_slice_and_identity_target():
    w = wl.config_c1()
    say("[case] C1 N_t=1")
    _check(w, w.u[:1], "f64", "banded", "exact", tag="C1 N_t=1")
    w2 = wl.config_c1()
    w2.sigma = np.eye(w2.d, dtype=np.complex128)
    say("[case] C1 sigma=I")
    phi, g, rhoT, p = gpu_eval(w2, w2.u[:50], prec="f64", path="banded", gmode="exact")
    p.close()
    assert abs(phi[0] - 1.0) < 1e-13
    assert np.max(np.abs(g)) < 1e-12


def test_tiny_dimension_d1_and_d2():
    # d = 1: the only state is 1, Phi = sigma, gradient 0.  d = 2: a qubit.
    for d in (1, 2):
        rng = np.random.default_rng(40 + d)
        X = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        H0 = 0.5 * (X + X.conj().T)
        Hk = np.stack([np.diag(np.arange(d, dtype=complex)) + 0.1])
        c = np.zeros((1, d, d), complex)
        c[0, 0, d - 1] = 1.0
        rho0 = np.zeros((d, d), complex)
        rho0[d - 1, d - 1] = 1
        sigma = np.diag(np.arange(1, d + 1, dtype=complex))
        w = wl.Workload("tiny", H0, Hk, c, np.array([0.3]), rho0, sigma, 0.05,
                        wl.controls_uniform(50 + d, 17, 1))
        for path in ("banded", "dense"):
            _check(w, w.u, "f64", path, "exact", tag=f"tiny d={d}")


def _diagonals(mats, offsets):
    d = mats.shape[-1]
    out = np.zeros(mats.shape[:-2] + (len(offsets), d), np.complex128)
    for t, o in enumerate(offsets):
        for i in range(max(0, -o), min(d, d - o)):
            out[..., t, i] = mats[..., i, i + o]
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_create_banded_equals_dense_create(prec):
    """og_create_banded with the diagonals of the C3-shaped operators gives
    bitwise the results of og_create with the dense matrices."""
    from paper_1609_03170_amd import Problem

    w = wl.config_c3(batch=2, n_t=12)
    mats = np.concatenate([w.H0[None], w.Hk, w.c_ops])
    offsets = sorted({int(j - i) for m in mats for i, j in zip(*np.nonzero(m))})
    say(f"[case] create_banded C3-shape prec={prec} offsets={offsets}")
    pb = Problem.from_banded(offsets, _diagonals(w.H0, offsets), _diagonals(w.Hk, offsets),
                             _diagonals(w.c_ops, offsets), w.gammas, prec=prec, gmode="exact")
    assert pb.path == "banded"
    a = gpu_eval(w, w.u, prec=prec, gmode="exact", problem=pb)
    pb.close()
    b = gpu_eval(w, w.u, prec=prec, path="auto", gmode="exact")
    b[3].close()
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
