"""GPU (HIP, through the C ABI) against the CPU oracle, element by element."""
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


from gpu_helpers import gpu_step, assert_parity  # noqa: E402
from paper_2607_05504_amd import FP64, MIXED  # noqa: E402


def _announce(msg):
    print(f"[case] {msg}", flush=True)


def test_uniform_box_32k_full():
    """Uniform periodic 32^3 box, all active, plain FP64 (the small workload)."""
    w = W.uniform_box(32768)
    _announce("uniform_box 32768")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)
    assert 120 < g["stats"]["n_events"] < 220


@pytest.mark.parametrize("n,n_active,periodic", [
    (34, 34, True), (35, 1, True), (100, 37, False), (1000, 1000, True),
    (2049, 1537, False), (5000, 4097, True), (5003, 65, False)])
def test_ragged_sizes(n, n_active, periodic):
    w = W.uniform_box(n, ic_seed=n + 7, scatters_per_particle=0.4)
    if not periodic:
        w.periodic, w.box = False, 0.0
    w = w.subset_active(n_active)
    _announce(f"ragged n={n} active={n_active} periodic={periodic}")
    ref = oracle.full_step(w, brute=n <= 4096)
    g = gpu_step(w)
    assert_parity(w, g, ref)


@pytest.mark.parametrize("side", [8, 16])
def test_lattice_exact_ties(side):
    w = W.uniform_box(side ** 3, lattice=True, ic_seed=3, scatters_per_particle=0.5)
    _announce(f"lattice {side}^3")
    ref = oracle.full_step(w, brute=True)
    g = gpu_step(w)
    assert_parity(w, g, ref)


def test_many_scatters_several_passes():
    """Three scatters per particle: most candidates take their turn after a
    kick of one of their particles; many that the step-start state rejects
    accept at their turn and the other way round."""
    w = W.uniform_box(6000, ic_seed=44, scatters_per_particle=3.0)
    _announce("high-probability box")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert ref["stats"]["n_passes"] >= 4
    acc0 = (ref["info"] & oracle.CAND_ACCEPT0) != 0
    hit = (ref["info"] & oracle.CAND_SCATTER) != 0
    assert (hit & ~acc0).sum() > 100 and (acc0 & ~hit).sum() > 100
    assert_parity(w, g, ref)


def test_rounds_in_one_workgroup(monkeypatch):
    """Many scatters per particle, every round after the first in the
    one-workgroup tail (no grid rounds): the same serial order."""
    monkeypatch.setenv("SIDM_TEST_DEVICE_ROUNDS", "0")
    w = W.uniform_box(3000, ic_seed=45, scatters_per_particle=2.0)
    _announce("rounds in one workgroup")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)
    acc0 = (ref["info"] & oracle.CAND_ACCEPT0) != 0
    hit = (ref["info"] & oracle.CAND_SCATTER) != 0
    assert (hit & ~acc0).any() and (acc0 & ~hit).any()


@pytest.mark.parametrize("grid_rounds", [6, 1])
def test_rounds_with_block_summaries(monkeypatch, grid_rounds):
    """Row block summaries and partner records forced on (the library keeps
    them for steps of 2^26 candidates and more): the first check's full scan
    writes the summaries; few particles per index bucket change after the
    first round, so the later checks scan only the row blocks that may touch
    them -- on the grid, or (one grid round) in the one-workgroup tail.  The
    same serial order."""
    monkeypatch.setenv("SIDM_TEST_FORCE_ROWS", "1")
    monkeypatch.setenv("SIDM_TEST_DEVICE_ROUNDS", str(grid_rounds))
    w = W.uniform_box(262144, ic_seed=46, scatters_per_particle=0.05)
    _announce(f"rounds with block summaries, {grid_rounds} on the grid")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert g["stats"]["n_rounds"] >= 2
    assert_parity(w, g, ref)


@pytest.mark.parametrize("k", [4, 16])
def test_block_summaries_other_row_lengths(monkeypatch, k):
    """Row block summaries and partner records forced on for rows of 4 and 16
    candidates (a block of 1024 candidates is 256 or 64 rows; a lane of the
    checks and of the evaluation takes four candidates of a row)."""
    monkeypatch.setenv("SIDM_TEST_FORCE_ROWS", "1")
    w = W.uniform_box(131072, ic_seed=47 + k, scatters_per_particle=0.1, n_ngb=k)
    _announce(f"block summaries, n_ngb={k}")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert g["stats"]["n_rounds"] >= 2
    assert_parity(w, g, ref)


@pytest.mark.parametrize("force_rows", ["0", "1"])
def test_caller_reordered_rows(monkeypatch, force_rows):
    """The step takes the caller's ngb, not the search's rows: with two entries
    of some rows swapped (the same candidates in another order), the rows
    the step uses are translated from ngb -- by their own kernel, or (partner
    records forced on) by the evaluation -- and the step is the same, its
    per-candidate information following the swap."""
    import torch
    from paper_2607_05504_amd import Context, runner
    monkeypatch.setenv("SIDM_TEST_FORCE_ROWS", force_rows)
    w = W.uniform_box(20000, ic_seed=48, scatters_per_particle=0.5)
    _announce(f"caller-reordered rows, force_rows={force_rows}")
    res = []
    for swap in (False, True):
        ds = runner.upload(w, "cuda")
        ctx = Context(runner.config_for(w), w.n, w.n_active)
        out = runner.alloc_out(ds, w.n_ngb, with_info=True)
        ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state,
                       m_scalar=ds.mass)
        ctx.find_ngb(ds.active, out.ngb, out.h)
        ngb = out.ngb
        if swap:
            ngb = out.ngb.clone()
            rows = torch.arange(0, w.n_active, 7, device=ngb.device)
            a, b = ngb[rows, 3].clone(), ngb[rows, 20].clone()
            ngb[rows, 3], ngb[rows, 20] = b, a
        ctx.scatter_step(ds.active, ngb, out.h, ds.dt, w.seed, w.step, cand_info=out.cand_info,
                         reuse_active=True)
        ctx.pair_timestep(ds.active, ngb, out.h, out.dt_sidm, reuse_active=True)
        stats = ctx.sync()
        info = out.cand_info.cpu().numpy().view(np.uint32).reshape(w.n_active, w.n_ngb).copy()
        if swap:
            r = np.arange(0, w.n_active, 7)
            info[r, 3], info[r, 20] = info[r, 20].copy(), info[r, 3].copy()
        res.append(dict(v=np.stack([ds.vx.cpu().numpy(), ds.vy.cpu().numpy(), ds.vz.cpu().numpy()]),
                        dt=out.dt_sidm.cpu().numpy(), info=info, events=stats["n_events"]))
        ctx.close()
    assert res[0]["events"] > 100
    assert res[0]["events"] == res[1]["events"]
    assert np.array_equal(res[0]["v"], res[1]["v"])
    assert np.array_equal(res[0]["dt"], res[1]["dt"])
    assert np.array_equal(res[0]["info"], res[1]["info"])


@pytest.mark.parametrize("k", [1, 8, 16, 31, 48, 63])
def test_neighbour_counts(k):
    """n_ngb from 1 to the largest accepted (63): the short-list and long-list
    forms of the search, and the step on rows of that length."""
    w = W.uniform_box(3000, ic_seed=90 + k, scatters_per_particle=0.5, n_ngb=k)
    w = w.subset_active(2111)
    _announce(f"n_ngb={k}")
    ref = oracle.full_step(w, brute=True)
    g = gpu_step(w)
    assert_parity(w, g, ref)


def test_hernquist_yukawa_small():
    w = W.hernquist_halo(20000, ic_seed=61)
    w = W.hernquist_bins(w, active_frac=0.3)
    _announce(f"hernquist 20000 active={w.n_active}")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)


def test_two_state_small():
    w = W.hernquist_halo(20000, ic_seed=62, two_state=True)
    w.sigma0 *= 20
    w = W.hernquist_bins(w, active_frac=0.5)
    _announce(f"two-state hernquist 20000 active={w.n_active}")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert ref["stats"]["n_events"] > 100
    assert_parity(w, g, ref)


def test_constant_eps_model():
    w = W.uniform_box(8000, ic_seed=63, scatters_per_particle=0.5)
    w.model, w.eps = W.MODEL_EPS, 0.8
    _announce("eps=0.8 box")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)


def test_hernquist_1e6_binned_full_size():
    """Isolated Hernquist halo, 1e6 particles, ~1/8 active in timestep bins."""
    w = W.hernquist_bins(W.hernquist_halo(1_000_000))
    _announce(f"hernquist 1e6 active={w.n_active}")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)


def test_determinism_and_permutation():
    w = W.uniform_box(20000, ic_seed=71, scatters_per_particle=0.8).subset_active(15000)
    _announce("determinism / permutation")
    a = gpu_step(w)
    b = gpu_step(w)
    for f in ("ngb", "h", "vx", "vy", "vz", "dt_sidm", "info"):
        assert np.array_equal(a[f], b[f]), f
    wp, perm = w.permuted(seed=5)
    c = gpu_step(wp)
    order = wp.meta["active_order"]
    assert np.array_equal(perm[c["ngb"]], a["ngb"][order])
    assert np.array_equal(c["h"], a["h"][order])
    for f in ("vx", "vy", "vz"):
        assert np.array_equal(c[f], a[f][perm]), f
    assert np.array_equal(c["info"], a["info"][order])


@pytest.mark.parametrize("case", ["halo_table", "box_table_mixed"])
def test_tabulated_cross_section(case):
    """sigma(w)/m given as a 64-node table (linear in ln w between
    log-spaced nodes): the same parity bar as the closed-form models, except
    that ln w comes from two libraries' log, so probabilities and the
    timestep agree to 1e-13 rather than bit for bit."""
    from paper_2607_05504_amd import MIXED, FP64
    if case == "halo_table":
        w = W.with_table(W.hernquist_bins(W.hernquist_halo(20000, ic_seed=206, philox_seed=16),
                                          active_frac=0.25))
        prec = FP64
    else:
        w = W.uniform_box(5000, ic_seed=207, scatters_per_particle=0.3)
        w.xsec, w.w0 = W.XSEC_YUKAWA, 1.0
        w = W.with_table(w)
        prec = MIXED
    _announce(f"tabulated cross-section {case} n={w.n} active={w.n_active}")
    ref = oracle.full_step(w)
    g = gpu_step(w, precision=prec)
    assert_parity(w, g, ref, mixed=(prec == MIXED), p_rtol=1e-13)
    assert g["stats"]["n_events"] > 0


@pytest.mark.parametrize("case,prec", [("box", FP64), ("halo", FP64), ("halo", MIXED)])
def test_refit_after_particles_moved(case, prec):
    """Tree reuse: after the particles have moved (drift in the periodic box,
    leapfrog steps in the halo) sidm_refit_tree keeps the old order, and the
    step still matches the oracle on the new positions exactly (the mixed
    form's leaf offsets are refitted too)."""
    import torch
    from paper_2607_05504_amd import Context, runner
    if case == "box":
        w = W.uniform_box(20000, ic_seed=208, scatters_per_particle=0.1)
    else:
        w = W.hernquist_bins(W.hernquist_halo(20000, ic_seed=209, philox_seed=18), active_frac=0.25)
    _announce(f"refit after motion: {case} n={w.n} precision={prec}")
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w, precision=prec), w.n, w.n_active)
    out = runner.alloc_out(ds, w.n_ngb, with_info=True)
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    dts = torch.full((w.n,), 0.01, dtype=torch.float64, device="cuda")
    for _ in range(3):
        if case == "box":
            ctx.drift(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, 0.05)
        else:
            ctx.advance_hernquist(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, dts, w.n, 0.25, 1.0, 1.0)
    ctx.refit_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    ctx.find_ngb(ds.active, out.ngb, out.h)
    ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step, cand_info=out.cand_info)
    ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm)
    stats = ctx.sync()
    moved = w.copy()
    moved.x, moved.y, moved.z = ds.x.cpu().numpy(), ds.y.cpu().numpy(), ds.z.cpu().numpy()
    torch.cuda.synchronize()
    # the oracle starts from the moved positions and the pre-step velocities
    pre = runner.upload(w, "cuda")
    for _ in range(3):
        if case == "box":
            ctx.drift(pre.x, pre.y, pre.z, pre.vx, pre.vy, pre.vz, 0.05)
        else:
            ctx.advance_hernquist(pre.x, pre.y, pre.z, pre.vx, pre.vy, pre.vz, dts, w.n, 0.25, 1.0, 1.0)
    ctx.sync()
    moved.vx, moved.vy, moved.vz = pre.vx.cpu().numpy(), pre.vy.cpu().numpy(), pre.vz.cpu().numpy()
    ref = oracle.full_step(moved)
    g = dict(ngb=out.ngb.cpu().numpy(), h=out.h.cpu().numpy(), vx=ds.vx.cpu().numpy(),
             vy=ds.vy.cpu().numpy(), vz=ds.vz.cpu().numpy(), state=ds.state.cpu().numpy(),
             dt_sidm=out.dt_sidm.cpu().numpy(),
             info=out.cand_info.cpu().numpy().view(np.uint32), stats=stats)
    assert_parity(moved, g, ref, mixed=(prec == MIXED))
    ctx.close()


def test_beam_model_small():
    """The fixed-target beam model (sec. 5.1): the same parity bar."""
    w = W.beam_lattice(n_side=10, n_beam=1500, rate_dt=0.3)
    _announce(f"beam lattice n={w.n}")
    ref = oracle.full_step(w)
    g = gpu_step(w)
    assert_parity(w, g, ref)
    assert g["stats"]["n_events"] > 0


@pytest.mark.parametrize("kind", ["elastic box", "two-state halo"])
def test_per_particle_masses(kind):
    """Unequal masses (a mass array instead of m_scalar): P uses m_j, the
    kick the two masses, the timestep m_i; every output against the oracle,
    and momentum sum m v (and the two-state energy with the gap) conserved."""
    import torch
    from paper_2607_05504_amd import Context, runner
    if kind == "elastic box":
        w = W.uniform_box(6000, ic_seed=211, philox_seed=21, scatters_per_particle=0.5)
    else:
        w = W.hernquist_halo(6000, ic_seed=212, philox_seed=22, two_state=True)
    rng = np.random.Generator(np.random.PCG64(13))
    w.masses = w.mass * rng.uniform(0.5, 1.5, w.n)
    _announce(f"per-particle masses: {kind} n={w.n}")
    ref = oracle.full_step(w)
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, w.n_active)
    out = runner.alloc_out(ds, w.n_ngb, with_info=True)
    m = torch.from_numpy(np.ascontiguousarray(w.masses)).cuda()
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, mass=m)
    ctx.find_ngb(ds.active, out.ngb, out.h)
    ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, w.seed, w.step, cand_info=out.cand_info,
                     reuse_active=True)
    ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)
    stats = ctx.sync()
    g = dict(ngb=out.ngb.cpu().numpy(), h=out.h.cpu().numpy(), vx=ds.vx.cpu().numpy(),
             vy=ds.vy.cpu().numpy(), vz=ds.vz.cpu().numpy(), state=ds.state.cpu().numpy(),
             dt_sidm=out.dt_sidm.cpu().numpy(), info=out.cand_info.cpu().numpy().view(np.uint32),
             stats=stats)
    ctx.close()
    assert_parity(w, g, ref)
    assert stats["n_events"] > 0
    mm = w.masses
    for f0, f1 in (("vx", "vx"), ("vy", "vy"), ("vz", "vz")):
        p0, p1 = float((mm * getattr(w, f0)).sum()), float((mm * g[f1]).sum())
        assert abs(p1 - p0) <= 1e-12 * float((mm * np.abs(getattr(w, f0))).sum())
    e = lambda vx, vy, vz, s: 0.5 * float((mm * (vx * vx + vy * vy + vz * vz)).sum()) + \
        w.delta * float((mm * s.astype(np.float64)).sum())
    e0 = e(w.vx, w.vy, w.vz, w.state)
    assert abs(e(g["vx"], g["vy"], g["vz"], g["state"]) - e0) <= 1e-12 * e0


def _morton_keys(x, y, z, periodic, box):
    """48-bit Morton keys as the tree defines them (16 bits an axis over the
    bounding box, or over [0, box) when periodic), computed here on the CPU."""
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0xffff)
        r = np.zeros_like(v)
        for b in range(16):
            r |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
        return r
    q = []
    for c in (x, y, z):
        lo, hi = (0.0, box) if periodic else (c.min(), c.max())
        ext = hi - lo
        scale = 65536.0 / ext if ext > 0 else 0.0
        f = (c - lo) * scale
        q.append(np.where(f > 0, np.where(f >= 65535.0, 65535.0, np.floor(f)), 0.0).astype(np.uint64))
    return (spread(q[0]) << np.uint64(2)) | (spread(q[1]) << np.uint64(1)) | spread(q[2])


@pytest.mark.parametrize("case", ["halo 3e5", "uniform 2e5 periodic", "ragged 5000+7",
                                  "halo 3e6"])
def test_tree_order_is_a_stable_morton_sort(case):
    """The radix sort: the tree's order is a permutation, ascending in the
    Morton key, equal keys in caller order -- over 3 sort tiles of 2048 keys
    (the last one ragged), about a hundred and about fifteen hundred."""
    import torch
    from paper_2607_05504_amd import Context, runner
    w = {"halo 3e5": lambda: W.hernquist_halo(300_000, ic_seed=61),
         "uniform 2e5 periodic": lambda: W.uniform_box(200_000, ic_seed=62),
         "ragged 5000+7": lambda: W.uniform_box(5007, ic_seed=63),
         "halo 3e6": lambda: W.hernquist_halo(3_000_000, ic_seed=64)}[case]()
    _announce(f"tree order {case} n={w.n}")
    ds = runner.upload(w, "cuda")
    ctx = Context(runner.config_for(w), w.n, 1)
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state,
                   m_scalar=ds.mass)
    order = torch.empty(w.n, dtype=torch.int32, device="cuda")
    ctx.tree_order(order)
    st = ctx.sync()
    ctx.close()
    assert st["error"] == 0
    o = order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(o), np.arange(w.n))
    k = _morton_keys(w.x, w.y, w.z, w.periodic, w.box)[o]
    assert np.all(k[1:] >= k[:-1])
    ties = k[1:] == k[:-1]
    assert np.all(o[1:][ties] > o[:-1][ties])
    ref = np.argsort(_morton_keys(w.x, w.y, w.z, w.periodic, w.box), kind="stable")
    assert np.array_equal(o, ref)


@pytest.mark.parametrize("case", ["halo two-state FP64", "halo two-state mixed",
                                  "periodic box FP64"])
def test_comoving_storage(case):
    """Comoving storage (sec. 4.2): lengths and relative speeds converted to
    physical units by factors that round (0.37, 1.9) inside W, sigma, P, the
    two-state energy balance and the timestep; the same parity bar."""
    import dataclasses
    if case.startswith("halo"):
        w = W.hernquist_bins(W.hernquist_halo(20000, ic_seed=210, philox_seed=19, two_state=True),
                             active_frac=0.25)
    else:
        w = W.uniform_box(8000, ic_seed=211, scatters_per_particle=0.2)
    w = dataclasses.replace(w, len_to_phys=0.37, vel_to_phys=1.9)
    prec = MIXED if "mixed" in case else FP64
    _announce(f"comoving storage {case} n={w.n} active={w.n_active}")
    ref = oracle.full_step(w)
    g = gpu_step(w, precision=prec)
    assert_parity(w, g, ref, mixed=(prec == MIXED))
    assert g["stats"]["n_events"] > 0
