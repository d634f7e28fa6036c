"""Parity at the full configuration sizes against stored oracle values
(tests/golden/*.npz, written by tests/golden/make_golden.py, which calls only
the oracle), plus properties that hold at any size for the batch members the
oracle was not run on."""
import os

import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, phi_err, grad_err, relerr, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return dict(np.load(path))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("path", ["banded", "dense"])
def test_c2_full_d90_nt2000(prec, path):
    g = _golden("c2_cqed_d90.npz")
    w = wl.config_c2()
    for gmode in ("grape1", "exact"):
        say(f"[case] C2 full prec={prec} path={path} gmode={gmode}")
        phi, grad, rhoT, p = gpu_eval(w, w.u, prec=prec, path=path, gmode=gmode)
        p.close()
        tol = TOL[prec]
        e_phi = phi_err(phi[0], float(g["phi"]))
        e_g = grad_err(grad[0], g["g_" + gmode])
        e_rho = relerr(rhoT[0], g["rhoT"])
        say(f"   phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
        assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_c3_full_d240_nt10000_bench_configuration(prec):
    """The benchmark's launch configuration: banded path, B = 128 problems
    (seeds 2..129), N_t = 10000.  Problem 0 against the stored oracle values;
    every problem against trace, Hermiticity and positivity; problem 0 alone
    equals problem 0 in the batch."""
    import gc

    import torch

    g = _golden("c3_cqed_d240.npz")
    B = 128
    w = wl.config_c3(batch=B)
    gc.collect()
    torch.cuda.empty_cache()  # no cached segment of an earlier test is split below
    say(f"[case] C3 full B={B} prec={prec} grape1")
    phi, grad, rhoT, p = gpu_eval(w, w.u, prec=prec, path="banded", gmode="grape1")
    p.close()
    tol = TOL[prec]
    e_phi = phi_err(phi[0], float(g["phi"]))
    e_g = grad_err(grad[0], g["g_grape1"])
    e_diag = relerr(np.diag(rhoT[0]).real, g["rhoT_diag"])
    e_rows = relerr(rhoT[0][[0, 80, 81, 161, 239]], g["rhoT_rows"])
    say(f"   problem 0: phi {e_phi:.2e} grad {e_g:.2e} diag {e_diag:.2e} rows {e_rows:.2e}")
    assert e_phi < tol["phi"] and e_g < tol["grad"]
    assert e_diag < tol["rho"] and e_rows < tol["rho"]
    tr_tol = 1e-12 if prec == "f64" else 1e-5
    for b in range(B):
        r = rhoT[b]
        assert np.array_equal(r, r.conj().T)
        assert abs(np.trace(r).real - 1.0) < tr_tol
        assert np.min(np.linalg.eigvalsh(r)) > -1e-4
        assert np.all(np.isfinite(grad[b]))
    say("[case] C3 full problem 0 alone")
    phi1, grad1, _, p1 = gpu_eval(w, w.u[0], prec=prec, path="banded", gmode="grape1")
    p1.close()
    assert np.array_equal(phi1[0], phi[0]) and np.array_equal(grad1[0], grad[0])
    # the benchmark's memory split: as many final states resident as fit in
    # the free device memory (less the benchmark's headroom), the slices
    # before them recomputed from checkpoints every ceil(sqrt(N_t - resident))
    # slices (a ragged last segment); bitwise the results without resident
    # states, problem 0 against the stored oracle values
    from paper_1609_03170_amd import Problem

    dev = torch.device("cuda", 0)
    pr = Problem.from_workload(w, prec=prec, path="banded", gmode="grape1")
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info(dev)
    budget = free - max(4 << 30, int(0.03 * total)) - (4 << 30)  # and room for this test's own tensors
    n_res = pr.resident_for_budget(B, w.n_t, budget)
    stride = int(np.ceil(np.sqrt(w.n_t - n_res)))
    say(f"[case] C3 full B={B} prec={prec} resident={n_res} stride={stride} "
        f"(last segment {(w.n_t - n_res) % stride or stride} slices; free {free / 2**30:.1f} GiB)")
    assert n_res > 0, "no resident slice fits in the free device memory"
    pr.set_resident(n_res)
    phi2, grad2, rhoT2, pr = gpu_eval(w, w.u, problem=pr)
    pr.close()
    torch.cuda.empty_cache()
    assert np.array_equal(phi2, phi) and np.array_equal(grad2, grad) and np.array_equal(rhoT2, rhoT)
    e_g2 = grad_err(grad2[0], g["g_grape1"])
    say(f"   problem 0 with resident states: grad {e_g2:.2e}")
    assert e_g2 < tol["grad"]
    del pr
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_c4_full_dense_d512_nt1000(prec):
    """Dense random d = 512, N_t = 1000 on the matrix-core path; float64 and
    float32 to their tolerances, the 16-bit splits reported (bounded loosely)."""
    g = _golden("c4_dense_d512_nt1000.npz")
    w = wl.config_c4()
    say(f"[case] C4 full d=512 N_t=1000 prec={prec}")
    phi, grad, rhoT, p = gpu_eval(w, w.u, prec=prec, path="dense", gmode="grape1")
    p.close()
    e_phi = phi_err(phi[0], float(g["phi"]))
    e_g = grad_err(grad[0], g["g_grape1"])
    e_rows = relerr(rhoT[0][[0, 255, 511]], g["rhoT_rows"])
    say(f"   phi {e_phi:.2e} grad {e_g:.2e} rows {e_rows:.2e}")
    tol = TOL.get(prec, dict(phi=1e-3, grad=1e-2, rho=1e-3))
    assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rows < tol["rho"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_c3_full_exact_gradient(prec):
    g = _golden("c3_cqed_d240.npz")
    w = wl.config_c3(batch=1)
    say(f"[case] C3 full B=1 prec={prec} exact")
    phi, grad, rhoT, p = gpu_eval(w, w.u, prec=prec, path="banded", gmode="exact")
    p.close()
    e_phi = phi_err(phi[0], float(g["phi"]))
    e_g = grad_err(grad[0], g["g_exact"])
    say(f"   phi {e_phi:.2e} grad {e_g:.2e}")
    assert e_phi < TOL[prec]["phi"] and e_g < TOL[prec]["grad"]
