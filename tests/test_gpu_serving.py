"""Continuous batching: requests of mixed shapes and lengths admitted while
others run; every result equals the same request evaluated alone (through
the server and through the batch entry points) and the float64 oracle."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import grad_err, relerr, say
from oracle import rk

pytestmark = pytest.mark.gpu

SHAPES = wl.SERVING_SHAPES  # (n_q, N): d = 20, 40, 90, 160, 240


def _trace(n, seed=3, n_t_range=(40, 130)):
    reqs = wl.serving_requests(n, seed=seed, arrival_seed=seed + 1, rate=400.0, n_t_range=n_t_range)
    for r in reqs:
        r["shape"] = SHAPES[r["id"] % len(SHAPES)]
    return reqs


def _loop(budget=1 << 30, max_slices=5):
    from paper_1609_03170_amd.serve import ServingLoop

    models = {s: wl.serving_model(s) for s in SHAPES}
    return ServingLoop(models, prec="f32", budget_bytes=budget, max_slices=max_slices), models


def test_mix_matches_alone_and_oracle():
    import torch

    from paper_1609_03170_amd import Problem

    reqs = _trace(10)  # two requests of every shape
    loop, models = _loop()
    say(f"[case] serving mix of {len(reqs)} requests, shapes {SHAPES}")
    out = loop.run(reqs, wl.serving_controls, keep=True)
    assert len(out.latencies) == len(reqs)
    for r in reqs:
        phi_mix, g_mix = (t.cpu().numpy() for t in out.results[r["id"]])
        # alone through the server
        alone = loop.run([dict(r, arrival=0.0)], wl.serving_controls, keep=True)
        phi_a, g_a = (t.cpu().numpy() for t in alone.results[r["id"]])
        assert np.array_equal(phi_mix, phi_a) and np.array_equal(g_mix, g_a)
        # alone through the batch entry points (same kernels, strided addressing)
        w = models[r["shape"]]
        p = Problem.from_workload(w, prec="f32", path="banded", gmode="grape1")
        dev = torch.device("cuda", 0)
        u = wl.serving_controls(r)
        phi_b, g_b = p.cost_and_grad(torch.tensor(u, device=dev), torch.tensor(w.rho0, device=dev),
                                     torch.tensor(w.sigma, device=dev), w.dt)
        torch.cuda.synchronize()
        p.close()
        assert abs(phi_b.cpu().numpy()[0] - phi_mix[0]) <= 1e-12 * max(1.0, abs(phi_mix[0]))
        assert relerr(g_mix, g_b.cpu().numpy()[0]) < 1e-12
        # float64 oracle
        m = rk.Model.from_workload(w, sparse=True)
        phi_r, g_r, _ = rk.cost_and_grad(m, u, w.rho0, w.sigma, w.dt)
        e_phi = abs(phi_mix[0] - phi_r) / max(abs(phi_r), 1e-3)
        e_g = grad_err(g_mix, g_r)
        say(f"   id={r['id']} shape={r['shape']} N_t={r['n_t']}: phi {e_phi:.2e} grad {e_g:.2e}")
        assert e_phi < 1e-5 and e_g < 1e-5
    loop.close()


@pytest.mark.parametrize("resident", [7, 1 << 30])
def test_resident_serving_bitwise(resident):
    """Requests that keep the packed halves of their last `resident` forward
    states (a tail and recomputed segments before it, or every state) give
    the bits of requests that keep none."""
    reqs = _trace(10, seed=5, n_t_range=(20, 60))
    base, _ = _loop()
    ref = base.run(reqs, wl.serving_controls, keep=True)
    base.close()
    loop, _ = _loop()
    for p in loop.problems.values():
        p.set_resident(resident)
    say(f"[case] serving {len(reqs)} requests with resident={resident}")
    out = loop.run(reqs, wl.serving_controls, keep=True)
    assert len(out.latencies) == len(reqs)
    for r in reqs:
        a = [t.cpu().numpy() for t in out.results[r["id"]]]
        b = [t.cpu().numpy() for t in ref.results[r["id"]]]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), r
    loop.close()


def test_budget_admission_bounds_memory():
    reqs = _trace(8, seed=11)
    loop, models = _loop(budget=1)  # room for a single request at a time
    say("[case] serving with a one-request budget")
    out = loop.run(reqs, wl.serving_controls)
    one = max(loop.servers[r["shape"]].request_bytes(r["n_t"]) for r in reqs)
    assert len(out.latencies) == len(reqs)
    assert out.peak_bytes <= one
    loop.close()


def test_server_full_and_errors():
    import torch

    from paper_1609_03170_amd import OgError, Problem
    from paper_1609_03170_amd.api import Server

    w = wl.serving_model((2, 10))
    p = Problem.from_workload(w, prec="f32", path="banded")
    srv = Server(p, max_active=1)
    dev = torch.device("cuda", 0)
    u = torch.tensor(wl.controls_uniform(5, 20, 4), device=dev)
    r0 = torch.tensor(w.rho0, device=dev)
    sg = torch.tensor(w.sigma, device=dev)
    assert srv.submit(1, u, r0, sg, w.dt)
    assert not srv.submit(2, u, r0, sg, w.dt)  # full
    with pytest.raises(OgError):
        srv.step(0)
    while srv.active:
        srv.step(7)
    torch.cuda.synchronize()
    assert list(srv.completed().keys()) == [1]
    with pytest.raises(OgError) as e:
        srv.submit(3, u, r0, sg, 10.0)
    assert e.value.name == "OG_ERR_UNSTABLE_DT"
    srv.close()
    p.close()
    wd = wl.dense_random_problem(d=16, K=1, J=1, n_t=2, seeds=(1, 2, 3, 4, 5, 6))
    pd = Problem.from_workload(wd, prec="f32", path="dense")
    with pytest.raises(OgError) as e:
        Server(pd)
    assert e.value.name == "OG_ERR_SHAPE"
    pd.close()
