"""Stage-kernel tap layouts on operators outside the ladder structure of the
cQED configurations, against the float64 oracle: the general (8, 4)
instantiation (diagonals 0, +-2, +-3 and four dissipator taps from one
two-diagonal collapse operator), the library maximum (16, 16) (nine
diagonals), and the ladder order with zero-coefficient taps inserted
(diagonals 0, +-5 and a single (2, 2) dissipator tap, to which the host adds
the +-1 diagonals and the (0, 0), (1, 1) taps).  Ragged d = 70: three tile
rows, the last one partial."""
import pytest

import workloads as wl
from _gpu_util import TOL, gpu_eval, oracle_eval, phi_err, grad_err, relerr, say

pytestmark = pytest.mark.gpu

CASES = {
    "general_8_4": ([0, 2, 3], [2], [[1, 2]]),
    "max_16_16": ([0, 1, 2, 3, 4], [1], [[1], [2]]),
    "ladder_inserted": ([0, 5], [5], [[2]]),
}


@pytest.mark.parametrize("gmode", ["grape1", "exact"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_tap_layouts(case, prec, gmode):
    hoffs, hkoffs, coffs = CASES[case]
    w = wl.banded_random_problem(70, hoffs, hkoffs, coffs, K=2, n_t=12, dt=0.01)
    say(f"[case] {case} d=70 prec={prec} gmode={gmode}")
    phi, g, rhoT, p = gpu_eval(w, w.u, prec=prec, path="banded", gmode=gmode)
    assert p.path == "banded"
    p.close()
    phi_r, g_r, rho_r = oracle_eval(w, w.u, mode=gmode)
    tol = TOL[prec]
    e_phi, e_g, e_rho = phi_err(phi[0], phi_r), grad_err(g[0], g_r), relerr(rhoT[0], rho_r)
    say(f"   phi {e_phi:.2e} grad {e_g:.2e} rho {e_rho:.2e}")
    assert e_phi < tol["phi"] and e_g < tol["grad"] and e_rho < tol["rho"]
