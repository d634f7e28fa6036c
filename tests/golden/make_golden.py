"""Write the stored expected values used by the full-size GPU parity tests.

Every number here comes from the float64 oracle (oracle/) on the seeded
workloads (workloads/); nothing is read from the GPU library.  Run from the
repository root:  python tests/golden/make_golden.py [c2] [c3] [c4] [d4096]
(all of them when no argument is given).  The C3 case needs about 10 GB of
memory and tens of minutes on 8 cores.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import rk  # noqa: E402


def _run(w, u, sparse, exact=True):
    m = rk.Model.from_workload(w, sparse=sparse)
    t0 = time.time()
    rhos = rk.forward(m, u, w.rho0, w.dt)
    phi = rk.cost(w.sigma, rhos[-1])
    lams = rk.backward(m, u, w.sigma, w.dt)
    g1 = rk.gradient_grape1(m, u, rhos, lams, w.dt)
    del lams
    ge = None
    if exact:
        ge, _ = rk.gradient_exact(m, u, rhos, w.sigma, w.dt)
    rhoT = rhos[-1]
    print(f"{w.name}: Phi = {phi:.15g}  ({time.time() - t0:.0f} s)", flush=True)
    return phi, g1, ge, rhoT


def c2():
    w = wl.config_c2()
    phi, g1, ge, rhoT = _run(w, w.u, sparse=False)
    np.savez_compressed(os.path.join(HERE, "c2_cqed_d90.npz"), phi=phi, g_grape1=g1, g_exact=ge, rhoT=rhoT)


def c3():
    w = wl.config_c3(batch=1)
    phi, g1, ge, rhoT = _run(w, w.u, sparse=True)
    np.savez_compressed(os.path.join(HERE, "c3_cqed_d240.npz"), phi=phi, g_grape1=g1, g_exact=ge,
                        rhoT_diag=np.diag(rhoT).real.copy(), rhoT_rows=rhoT[[0, 80, 81, 161, 239]].copy())


def c4(n_t=1000):
    w = wl.config_c4()
    u = w.u[:n_t]
    phi, g1, ge, rhoT = _run(w, u, sparse=False, exact=False)
    np.savez_compressed(os.path.join(HERE, f"c4_dense_d512_nt{n_t}.npz"), phi=phi, g_grape1=g1,
                        rhoT_rows=rhoT[[0, 255, 511]].copy(), rhoT_diag=np.diag(rhoT).real.copy())


D4096_ROWS = [0, 1, 63, 64, 65, 2047, 4095]


def d4096():
    """The largest dimension the library accepts: a damped driven resonator
    truncated at N = 4096 (coherent amplitude 8), two slices of 2e-4."""
    w = wl.resonator_problem(4096, 0.5, 1.0, 8.0, wl.controls_uniform(61, 2, 2), 2e-4, name="resonator4096")
    phi, g1, _, rhoT = _run(w, w.u, sparse=True, exact=False)
    np.savez_compressed(os.path.join(HERE, "resonator_d4096_nt2.npz"), phi=phi, g_grape1=g1,
                        rhoT_rows=rhoT[D4096_ROWS].copy(), rows=np.array(D4096_ROWS))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3", "c4", "d4096"]
    for name in which:
        {"c2": c2, "c3": c3, "c4": c4, "d4096": d4096}[name]()
