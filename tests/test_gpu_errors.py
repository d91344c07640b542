"""Error paths and degenerate inputs through the C ABI on the GPU.

Every bad input here is one the library itself turns into an error: the host
checks reject sizes and call order before anything is enqueued, and the
kernels test every index against its range before using it (a duplicate or
out-of-range active entry, an out-of-range neighbour index) and latch a bit
that sidm_sync reports.  After a reported error the context stays usable."""
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


def _setup(n=2000, n_active=None):
    from paper_2607_05504_amd import Context, runner
    w = W.uniform_box(n, ic_seed=55, scatters_per_particle=0.2)
    if n_active is not None:
        w = w.subset_active(n_active)
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, max(1, w.n_active))
    out = runner.alloc_out(ds, w.n_ngb, with_info=True)
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    return w, ds, ctx, out


def _sync_error(ctx):
    from paper_2607_05504_amd import SidmError
    with pytest.raises(SidmError) as e:
        ctx.sync()
    return str(e.value)


def test_duplicate_active_is_reported_and_context_recovers():
    _announce("duplicate active entry")
    w, ds, ctx, out = _setup()
    act = ds.active.clone()
    act[10] = act[11]
    ctx.find_ngb(act, out.ngb, out.h)
    assert "duplicate" in _sync_error(ctx)
    ctx.find_ngb(ds.active, out.ngb, out.h)
    ctx.sync()
    ngb, h = oracle.find_ngb(w)
    assert np.array_equal(out.ngb.cpu().numpy(), ngb)
    assert np.array_equal(out.h.cpu().numpy(), h)
    ctx.close()


def test_active_index_out_of_range_is_reported():
    _announce("active index out of range")
    w, ds, ctx, out = _setup()
    act = ds.active.clone()
    act[5] = w.n + 7
    act[6] = -3
    ctx.find_ngb(act, out.ngb, out.h)
    assert "index" in _sync_error(ctx)
    ctx.close()


@pytest.mark.parametrize("force_rows", ["0", "1"])
def test_bad_neighbour_index_is_reported(monkeypatch, force_rows):
    """Out-of-range entries of a caller's ngb are latched whether the rows
    are checked by their own kernel or (partner records forced on) by the
    evaluation."""
    monkeypatch.setenv("SIDM_TEST_FORCE_ROWS", force_rows)
    _announce(f"neighbour index out of range in scatter_step and pair_timestep, force_rows={force_rows}")
    w, ds, ctx, out = _setup()
    ctx.find_ngb(ds.active, out.ngb, out.h)
    ctx.sync()
    bad = out.ngb.clone()
    bad[3, 4] = -1
    bad[7, 0] = w.n
    ctx.scatter_step(ds.active, bad, out.h, ds.dt, w.seed, w.step)
    assert "index" in _sync_error(ctx)
    ctx.pair_timestep(ds.active, bad, out.h, out.dt_sidm)
    assert "index" in _sync_error(ctx)
    ctx.close()


def test_host_errors_return_before_anything_runs():
    import torch
    from paper_2607_05504_amd import (SIDM_E_CAPACITY, SIDM_E_INVAL, SIDM_E_STATE, Context,
                                      SidmError, make_config, runner)
    _announce("host-side errors")
    w = W.uniform_box(500, ic_seed=56)
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, 100)
    out = runner.alloc_out(ds, w.n_ngb)
    with pytest.raises(SidmError) as e:        # find_ngb before build_tree
        ctx.find_ngb(ds.active[:50], out.ngb[:50], out.h[:50])
    assert e.value.status == SIDM_E_STATE
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    with pytest.raises(SidmError) as e:        # more active particles than the capacity
        ctx.find_ngb(ds.active, out.ngb, out.h)
    assert e.value.status == SIDM_E_CAPACITY
    with pytest.raises(SidmError) as e:        # too few particles for n_ngb + 1 neighbours
        small = runner.upload(W.uniform_box(33, ic_seed=57), "cuda")
        ctx.build_tree(small.x, small.y, small.z, small.vx, small.vy, small.vz, small.ids,
                       state=small.state, m_scalar=small.mass)
    assert e.value.status == SIDM_E_INVAL
    with pytest.raises(SidmError) as e:        # the layout-fixing n_ngb cannot change
        ctx.reconfigure(make_config(n_ngb=16, periodic=True, box=1.0, sigma0=1.0))
    assert e.value.status == SIDM_E_INVAL
    ctx.sync()                                 # nothing was enqueued by the failed calls
    ctx.close()
    torch.cuda.synchronize()


def test_empty_active_set_changes_nothing():
    import torch
    _announce("empty active set")
    w, ds, ctx, out = _setup()
    v0 = ds.vx.clone()
    empty = ds.active[:0]
    ctx.find_ngb(empty, out.ngb[:0], out.h[:0])
    ctx.scatter_step(empty, out.ngb[:0], out.h[:0], ds.dt[:0], w.seed, w.step)
    ctx.pair_timestep(empty, out.ngb[:0], out.h[:0], out.dt_sidm[:0])
    st = ctx.sync()
    assert st["error"] == 0 and st["n_events"] == 0
    assert torch.equal(ds.vx, v0)
    ctx.close()


def test_active_mapping_reuse_rules():
    """active == NULL reuses the previous call's mapping of the active set:
    refused (nothing enqueued) right after a tree build or with another
    n_active; after find_ngb it gives the results of an explicit list."""
    import torch
    from paper_2607_05504_amd import SIDM_E_STATE, SidmError
    _announce("active-set mapping reuse")
    w, ds, ctx, out = _setup(n_active=1500)
    with pytest.raises(SidmError) as e:            # nothing mapped since the tree build
        ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step, reuse_active=True)
    assert e.value.status == SIDM_E_STATE
    ctx.find_ngb(ds.active, out.ngb, out.h)
    with pytest.raises(SidmError) as e:            # another n_active
        ctx.pair_timestep(ds.active[:100], out.ngb[:100], out.h[:100], out.dt_sidm[:100],
                          reuse_active=True)
    assert e.value.status == SIDM_E_STATE
    v0 = [t.clone() for t in (ds.vx, ds.vy, ds.vz)]
    ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step, reuse_active=True)
    ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)
    st = ctx.sync()
    got = [t.clone() for t in (ds.vx, ds.vy, ds.vz)] + [out.dt_sidm.clone()]
    # the same step with explicit lists on the step-start velocities
    for t, t0 in zip((ds.vx, ds.vy, ds.vz), v0):
        t.copy_(t0)
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    with pytest.raises(SidmError) as e:            # the new tree dropped the mapping
        ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)
    assert e.value.status == SIDM_E_STATE
    ctx.find_ngb(ds.active, out.ngb, out.h)
    ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step)
    ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm)
    st2 = ctx.sync()
    for a, b in zip(got, (ds.vx, ds.vy, ds.vz, out.dt_sidm)):
        assert torch.equal(a, b)
    assert st["n_events"] == st2["n_events"] > 0
    ctx.close()


def test_timing_mask_times_only_the_chosen_phases():
    """sidm_timing_enable takes a mask of phases: the ones in it report a
    mean launch time, the others 0; unknown bits are refused."""
    from paper_2607_05504_amd import (SIDM_E_INVAL, TIMING_ALL, TIMING_KNN, TIMING_TIMESTEP,
                                      SidmError)
    _announce("timing mask")
    w, ds, ctx, out = _setup(n_active=1500)
    with pytest.raises(SidmError) as e:
        ctx.timing_enable(TIMING_ALL + 1)
    assert e.value.status == SIDM_E_INVAL

    def step():
        ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state,
                       m_scalar=ds.mass)
        ctx.find_ngb(ds.active, out.ngb, out.h)
        ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step, reuse_active=True)
        ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)

    ctx.timing_enable(TIMING_KNN | TIMING_TIMESTEP)
    step()
    step()
    t = ctx.timing_read()
    assert t["samples"] == 2
    assert t["knn_ms"] > 0 and t["timestep_ms"] > 0
    assert t["tree_ms"] == 0 and t["map_ms"] == 0 and t["eval_ms"] == 0
    assert t["resolve_ms"] == 0 and t["overlap_ms"] == 0
    ctx.timing_enable(TIMING_ALL)
    step()
    t = ctx.timing_read()
    assert min(t[k] for k in ("tree_ms", "map_ms", "knn_ms", "eval_ms", "resolve_ms",
                              "timestep_ms")) > 0
    ctx.timing_enable(0)
    step()
    t = ctx.timing_read()
    assert t["samples"] == 0 and t["knn_ms"] == 0
    assert ctx.sync()["error"] == 0
    ctx.close()


def test_accepted_list_overflow_is_reported_and_the_context_recovers():
    """Every candidate accepted (sigma/m so large that P >> 1) on 40000 active
    particles: 1.28M accepted candidates against a list of 65536 entries.  The
    evaluation's flush drops what does not fit and latches the overflow,
    sidm_sync reports SIDM_E_OVERFLOW, and after a reconfiguration with a
    normal cross-section the next step runs clean."""
    from paper_2607_05504_amd import SIDM_E_OVERFLOW, Context, SidmError, runner
    w = W.uniform_box(40000, ic_seed=57, scatters_per_particle=0.1)
    _announce(f"accepted-list overflow n={w.n}")
    normal = w.sigma0
    w.sigma0 = normal * 1e7
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, w.n_active)
    out = runner.alloc_out(ds, w.n_ngb)
    runner.run_step(ctx, ds, out, w.seed, w.step)
    with pytest.raises(SidmError) as e:
        ctx.sync()
    assert e.value.status == SIDM_E_OVERFLOW
    w.sigma0 = normal
    ctx.reconfigure(runner.config_for(w))
    runner.run_step(ctx, ds, out, w.seed, w.step + 1)
    st = ctx.sync()
    assert st["error"] == 0 and st["n_events"] > 0
    ctx.close()
