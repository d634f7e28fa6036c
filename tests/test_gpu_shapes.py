"""The launch shapes of the batched stage kernel, chosen by the number of
blocks of a launch (problems x upper tiles): one tile per block with one
row per thread (float32) or two (float64) for small grids, two rows per
thread in float32 for mid-size grids, four rows per thread for full grids.
A batch of transmon(3) x resonator(20) problems (d = 60, ragged: 3 upper
tiles each, the ladder tap order of the headline configuration) with
distinct controls is sized to land in each shape; sampled problems of the
batch are compared with the float64 oracle."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, oracle_eval, phi_err, grad_err, relerr, say

pytestmark = pytest.mark.gpu

# (precision, batch): 6, 600 and 3000 blocks in float32; 6 and 1200 in
# float64
SHAPES = [("f32", 2), ("f32", 200), ("f32", 1000), ("f64", 2), ("f64", 400)]


@pytest.mark.parametrize("prec,B", SHAPES)
def test_launch_shapes(prec, B):
    w = wl.config_c3(batch=B, n_t=6, N=20)
    u = w.u
    say(f"[case] d=60 prec={prec} B={B} blocks={3 * B}")
    from paper_1609_03170_amd import Problem

    p = Problem.from_workload(w, prec=prec, path="banded", gmode="grape1")
    p.set_fused(False)  # the four-launch stage kernels, whose launch shapes are under test
    phi, g, rhoT, p = gpu_eval(w, u, problem=p)
    assert p.path == "banded" and not p.fused
    p.close()
    tol = TOL[prec]
    for b in sorted({0, B // 2, B - 1}):
        phi_r, g_r, rho_r = oracle_eval(w, u[b])
        e_phi, e_g, e_rho = phi_err(phi[b], phi_r), grad_err(g[b], g_r), relerr(rhoT[b], rho_r)
        say(f"   problem {b}: phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
        assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]
    assert np.isfinite(phi).all() and np.isfinite(g).all()
