"""The allocation-free entry point (sidm_advance_hernquist_noalloc) against
the context form (sidm_advance_hernquist) it is a variant of, through the C
ABI: two calls in a row, the second on fewer particles."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_05504_amd as sidm
    sidm.lib()


def _one(n, n_active, seed):
    import torch
    from paper_2607_05504_amd import Context, advance_hernquist_noalloc, runner
    w = W.hernquist_halo(n, ic_seed=seed, philox_seed=seed)
    print(f"[case] noalloc advance n={n} n_active={n_active}", flush=True)
    rng = np.random.Generator(np.random.PCG64(seed))
    dt = torch.from_numpy(rng.uniform(0.003, 0.5, n)).cuda()
    a = runner.upload(w, "cuda")
    b = runner.upload(w, "cuda")
    nxt_a = torch.zeros(n, dtype=torch.float64, device="cuda")
    nxt_b = torch.zeros(n, dtype=torch.float64, device="cuda")
    st_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    st_b = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ctx = Context(runner.config_for(w), n, max(n_active, 1))
    ctx.advance_hernquist(a.x, a.y, a.z, a.vx, a.vy, a.vz, dt, n_active, 0.25, 1.0, 1.0,
                          dt_next=nxt_a, dt_step=st_a)
    ctx.sync()
    ctx.close()
    advance_hernquist_noalloc(b.x, b.y, b.z, b.vx, b.vy, b.vz, dt, n_active, 0.25, 1.0, 1.0,
                              dt_next=nxt_b, dt_step=st_b)
    torch.cuda.synchronize()
    assert st_a.item() == st_b.item()
    assert torch.equal(nxt_a, nxt_b)
    for f in ("x", "y", "z", "vx", "vy", "vz"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f
    return st_b.item()


def test_noalloc_equals_context_form_on_two_calls():
    # the first call leaves its partial minima in the array; the second,
    # smaller one must not see them (a larger bound there would show)
    d1 = _one(300_000, 250_000, 401)
    d2 = _one(5_000, 3_000, 402)
    assert d1 > 0 and d2 > 0


def test_noalloc_without_active_particles_takes_dt_cap():
    assert _one(4_000, 0, 403) == 0.25


def test_noalloc_refuses_more_active_particles_than_its_scratch_holds():
    import torch
    from paper_2607_05504_amd import SIDM_E_CAPACITY, SidmError, advance_hernquist_noalloc
    n = 8_388_609
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    big = torch.zeros(n, dtype=torch.float64, device="cuda").expand(n).contiguous()
    with pytest.raises(SidmError) as e:
        advance_hernquist_noalloc(big, big, big, big, big, big, big, n, 0.25, 1.0, 1.0,
                                  dt_step=t)
    assert e.value.status == SIDM_E_CAPACITY
