"""Served form on the GPU: the inter-step advance against the oracle, a
served request against the oracle step by step, results alone vs in a mix
of concurrent requests, and admission by the HBM budget."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_05504_amd as sidm
    sidm.lib()


def _announce(msg):
    print(f"[case] {msg}", flush=True)


def test_advance_matches_oracle():
    import torch
    from paper_2607_05504_amd import Context, runner
    w = W.hernquist_halo(20000, ic_seed=301, philox_seed=5)
    _announce("advance_hernquist n=20000")
    rng = np.random.Generator(np.random.PCG64(9))
    dt_sidm = rng.uniform(0.003, 0.5, w.n)
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, w.n)
    dts = torch.from_numpy(dt_sidm).cuda()
    dt_next = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    dt_step = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.advance_hernquist(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, dts, w.n, 0.25, 1.0, 1.0,
                          dt_next=dt_next, dt_step=dt_step)
    ctx.sync()
    ref = oracle.advance_hernquist(w.x, w.y, w.z, w.vx, w.vy, w.vz, dt_sidm, 0.25, 1.0, 1.0)
    assert float(dt_step.item()) == ref[6]
    assert np.all(dt_next.cpu().numpy() == ref[6])
    for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        np.testing.assert_allclose(getattr(ds, f).cpu().numpy(), ref[k], rtol=1e-14, atol=1e-300)
    ctx.close()


@pytest.mark.parametrize("case", ["no active particle", "every bound infinite"])
def test_advance_without_a_finite_bound_takes_dt_cap(case):
    """No per-pair bound (no active particle, or every bound +inf): the step
    is dt_cap itself, as the oracle's step rule gives."""
    import torch
    from paper_2607_05504_amd import Context, runner
    w = W.hernquist_halo(5000, ic_seed=303, philox_seed=6)
    _announce(f"advance_hernquist {case}")
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, w.n)
    n_act = 0 if case == "no active particle" else w.n
    dts = torch.full((w.n,), float("inf"), dtype=torch.float64, device="cuda")
    dt_step = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.advance_hernquist(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, dts, n_act, 0.25, 1.0, 1.0,
                          dt_step=dt_step)
    ctx.sync()
    ref = oracle.advance_hernquist(w.x, w.y, w.z, w.vx, w.vy, w.vz,
                                   np.full(n_act, np.inf), 0.25, 1.0, 1.0)
    assert ref[6] == 0.25
    assert float(dt_step.item()) == 0.25
    for k, f in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        np.testing.assert_allclose(getattr(ds, f).cpu().numpy(), ref[k], rtol=1e-14, atol=1e-300)
    ctx.close()


def test_drift_matches_oracle():
    import torch
    from paper_2607_05504_amd import Context, runner
    w = W.uniform_box(20000, ic_seed=302)
    _announce("drift n=20000 periodic")
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, w.n)
    ctx.drift(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, 0.37)
    ctx.sync()
    ref = oracle.drift(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.37, True, 1.0)
    for k, f in enumerate(("x", "y", "z")):
        np.testing.assert_array_equal(getattr(ds, f).cpu().numpy(), ref[k])
    ctx.close()


def _reqs(ns, steps, gap=0.0, s0_scale=(1.0, 3.0, 0.3, 10.0, 0.1, 2.0)):
    base = W.hernquist_s0()
    return [W.Request(rid=r, arrival=r * gap, n=n, s0=base * s0_scale[r % len(s0_scale)],
                      ic_seed=500 + r, philox_seed=70 + r, steps=steps) for r, n in enumerate(ns)]


def test_served_request_matches_oracle_steps():
    """Two served steps of one halo (the first step's length from the bounds
    of the initial state; scatter step, pair timestep, advance with the step
    length from the bounds) against the oracle doing the same."""
    from paper_2607_05504_amd.serve import Server, ServeConfig
    req = _reqs([3000], steps=2)[0]
    _announce("served request n=3000 steps=2 vs oracle")
    srv = Server(ServeConfig(n_slots=1, keep_results=True))
    rep = srv.run([req], W.request_workload)
    srv.close()
    g = rep["results"][0]
    w = W.request_workload(req)
    # the first step's length: from the per-pair bounds of the initial state
    ngb0, h0 = oracle.find_ngb(w)
    w.dt = np.full(w.n, oracle.step_length(oracle.pair_timestep(w, ngb0, h0), 0.25))
    for t in range(2):
        w.step = t
        r = oracle.full_step(w)
        w.vx, w.vy, w.vz, w.state = r["vx"], r["vy"], r["vz"], r["state"]
        x, y, z, vx, vy, vz, d = oracle.advance_hernquist(w.x, w.y, w.z, w.vx, w.vy, w.vz,
                                                          r["dt_sidm"], 0.25, 1.0, 1.0)
        w.x, w.y, w.z, w.vx, w.vy, w.vz = x, y, z, vx, vy, vz
        w.dt = np.full(w.n, d)
    w.step = 0
    vs = max(np.abs(w.vx).max(), np.abs(w.vy).max(), np.abs(w.vz).max())
    for f in ("vx", "vy", "vz"):
        assert np.abs(g[f] - getattr(w, f)).max() <= 1e-11 * vs
    for f in ("x", "y", "z"):
        assert np.abs(g[f] - getattr(w, f)).max() <= 1e-11 * np.abs(getattr(w, f)).max()
    assert np.array_equal(g["state"], w.state)


def test_alone_equals_mix():
    """Each request's final state is bit-identical whether it is served alone
    or concurrently with others on several streams (the kernels use no
    floating-point atomics and each request has its own context)."""
    from paper_2607_05504_amd.serve import Server, ServeConfig
    reqs = _reqs([12000, 30000, 9000, 45000, 20000, 15000], steps=3, gap=0.002)
    _announce("alone vs mix, 6 requests")
    alone = {}
    srv = Server(ServeConfig(n_slots=1, keep_results=True))
    for r in reqs:
        alone[r.rid] = srv.run([r], W.request_workload)["results"][r.rid]
    srv.close()
    srv = Server(ServeConfig(n_slots=4, keep_results=True))
    seen = []
    mix = srv.run(reqs, W.request_workload, on_admit=lambda req, k: seen.append(k))
    srv.close()
    assert len(set(seen)) > 1, "the mix ran on one slot only"
    for r in reqs:
        a, m = alone[r.rid], mix["results"][r.rid]
        for f in ("x", "y", "z", "vx", "vy", "vz", "state"):
            assert np.array_equal(a[f], m[f]), f"request {r.rid}: {f} differs"
        assert a["stats"]["n_events"] == m["stats"]["n_events"]


def test_admission_respects_budget():
    """With a budget that holds about two requests, requests wait for memory;
    all complete, and a request larger than the budget is refused."""
    from paper_2607_05504_amd import footprint, runner
    from paper_2607_05504_amd.serve import Server, ServeConfig, capacity_class, state_bytes
    reqs = _reqs([20000] * 5, steps=2)
    w0 = W.request_workload(reqs[0])
    one = footprint(runner.config_for(w0), capacity_class(w0.n), capacity_class(w0.n)) + \
        state_bytes(w0.n, w0.n_ngb)
    _announce(f"budget admission, one request = {one} bytes")
    srv = Server(ServeConfig(n_slots=4, hbm_budget=int(2.5 * one), keep_results=False))
    rep = srv.run(reqs, W.request_workload)
    assert rep["n_requests"] == 5
    assert rep["max_admission_wait_s"] > 0.0
    with pytest.raises(ValueError):
        srv.run(_reqs([200000], steps=1), W.request_workload)
    srv.close()
