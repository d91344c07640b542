"""Pins of the oracle's kernel-overlap estimator (the paper's Eq.
kernelOverlap and its appendix on the overlap kernel) against things other
than itself: the normalisation every overlap of two unit-mass kernels has,
exact rational integrals at zero separation, the point-partner limit, a
direct 3D quadrature, the symmetry g_ij = g_ji, an all-pairs numpy search, and
the density the estimator measures in a uniform box.

None of these tests needs a GPU.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W

NA, NR = oracle.OVERLAP_NA, oracle.OVERLAP_NR


def _w_spline(q):
    """Cubic spline of unit support, vectorised (the kernel's own closed forms
    are pinned in test_oracle_pins)."""
    q = np.asarray(q, dtype=np.float64)
    out = np.where(q <= 0.5, 1.0 - 6.0 * q**2 + 6.0 * q**3, 2.0 * (1.0 - q) ** 3)
    return np.where(q <= 1.0, out, 0.0) * (8.0 / math.pi)


@pytest.mark.parametrize("hi,hj", [(1.0, 1.0), (1.0, 0.3), (0.2, 1.7), (0.05, 1.0)])
def test_overlap_is_normalised(hi, hj):
    # int g(r) d^3r = (int W_i)(int W_j) = 1 for any pair of smoothing lengths
    def f(r):
        return 4.0 * math.pi * r * r * oracle.overlap_exact(hi, hj, r)
    pts = sorted({abs(hi - hj) / 2, hi / 2, hj / 2, abs(hi - hj), hi, hj} - {0.0})
    pts = [p for p in pts if p < hi + hj]
    v, _ = integrate.quad(f, 0.0, hi + hj, points=pts, limit=200, epsabs=1e-14, epsrel=1e-13)
    assert abs(v - 1.0) < 1e-11


def _poly_mul(a, b):
    r = [F(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            r[i + j] += x * y
    return r


def _integ(p, lo, hi):
    return sum(c * (F(hi) ** (k + 1) - F(lo) ** (k + 1)) / (k + 1) for k, c in enumerate(p))


def _spline_pieces(scale):
    """Exact polynomial pieces (in s) of pi/8 W(s, h) for h = 1/scale:
    pi/8 W = scale^3 w(scale s), w = 1 - 6q^2 + 6q^3 | 2(1 - q)^3."""
    s3 = F(scale) ** 3
    inner = [s3, F(0), -6 * s3 * F(scale) ** 2, 6 * s3 * F(scale) ** 3]
    one_m = [F(1), -F(scale)]
    outer = [2 * s3]
    for _ in range(3):
        outer = _poly_mul(outer, one_m)
    return inner, outer


def test_overlap_at_zero_separation_exact_rationals():
    # g(h, h, 0) = int W^2 d^3x = 256 I / (pi h^3), I = int_0^1 q^2 w(q)^2 dq = 491/40320
    for h in (1.0, 0.37, 2.5):
        assert oracle.overlap_exact(h, h, 0.0) == pytest.approx(
            256.0 * 491.0 / 40320.0 / (math.pi * h**3), rel=1e-14)
    # h_i = 1, h_j = 1/2: 4 pi (8/pi)^2 int s^2 w(s) (8 w(2s)) ds over [0, 1/2],
    # pieces split at 1/4 (w(2s) changes form) -- s < 1/2 keeps w(s) on its inner piece
    wi_in, _ = _spline_pieces(1)
    wj_in, wj_out = _spline_pieces(2)
    s2 = [F(0), F(0), F(1)]
    I = (_integ(_poly_mul(s2, _poly_mul(wi_in, wj_in)), 0, F(1, 4))
         + _integ(_poly_mul(s2, _poly_mul(wi_in, wj_out)), F(1, 4), F(1, 2)))
    expect = 4.0 * math.pi * (8.0 / math.pi) ** 2 * float(I)
    assert oracle.overlap_exact(1.0, 0.5, 0.0) == pytest.approx(expect, rel=1e-14)
    assert oracle.overlap_exact(0.5, 1.0, 0.0) == pytest.approx(expect, rel=1e-14)


def test_point_partner_limit_is_the_spline():
    # h_i -> 0: W_i becomes a point mass at x_i and g -> W(r, h_j), to O(h_i^2)
    for hj in (1.0, 0.4):
        for q in (0.0, 0.2, 0.5, 0.8, 0.99):
            g = oracle.overlap_exact(1e-5 * hj, hj, q * hj)
            assert abs(g - oracle.kernel(q * hj, hj)) <= 1e-8 * oracle.kernel(0.0, hj)


@pytest.mark.parametrize("hi,hj,r", [(1.0, 0.6, 0.8), (0.5, 0.5, 0.3), (1.0, 0.7, 0.05)])
def test_overlap_matches_direct_3d_quadrature(hi, hj, r):
    # midpoint rule over the lens where both kernels are non-zero (W is C2, so
    # the rule converges as the square of the cell size)
    n = 200
    lo = np.array([max(-hi, r - hj), -min(hi, hj), -min(hi, hj)])
    hi_ = np.array([min(hi, r + hj), min(hi, hj), min(hi, hj)])
    d = (hi_ - lo) / n
    ys = lo[1] + d[1] * (np.arange(n) + 0.5)
    zs = lo[2] + d[2] * (np.arange(n) + 0.5)
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    yz2 = Y * Y + Z * Z
    total = 0.0
    for ix in range(n):
        x = lo[0] + d[0] * (ix + 0.5)
        a = np.sqrt(x * x + yz2) / hi
        b = np.sqrt((x - r) ** 2 + yz2) / hj
        total += float((_w_spline(a) * _w_spline(b)).sum())
    g3 = total * d.prod() / (hi**3 * hj**3)
    assert g3 == pytest.approx(oracle.overlap_exact(hi, hj, r), rel=2e-4)


def test_overlap_symmetric_and_decreasing():
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(60):
        hi, hj = rng.uniform(0.05, 2.0, 2)
        rs = np.linspace(0.0, hi + hj, 41)
        g = np.array([oracle.overlap_exact(hi, hj, r) for r in rs])
        gt = np.array([oracle.overlap_exact(hj, hi, r) for r in rs])
        np.testing.assert_allclose(g, gt, rtol=1e-12, atol=1e-14 * g[0])
        # two radially decreasing kernels overlap most at zero separation and
        # less the further apart they are
        assert np.all(np.diff(g) <= 1e-13 * g[0])
        assert g[-1] == 0.0


def test_table_nodes_and_interpolation_accuracy():
    T = oracle.overlap_table()
    assert T.shape == (NA + 1, NR + 1)
    rho = np.arange(NR + 1) / NR
    np.testing.assert_array_equal(T[0], [oracle.kernel(q, 1.0) for q in rho])
    for a in (1, 7, 32, 63, 64):
        al = a / (2.0 * NA)
        for b in (0, 1, 100, 255, 256):
            assert T[a, b] == oracle.overlap_exact(al, 1.0 - al, rho[b])
    assert np.all(T[:, NR] == 0.0)
    # on the nodes the estimator returns the table over H^3 (H = h_i + h_j)
    for a, b, H in ((10, 40, 0.3), (64, 0, 2.0), (33, 255, 1.0)):
        al = a / (2.0 * NA)
        got = oracle.overlap_g(al * H, (1 - al) * H, rho[b] * H)
        assert got == pytest.approx(T[a, b] / H**3, rel=1e-13, abs=1e-300)
    # between the nodes: bilinear error below 3e-4 of the centre value
    rng = np.random.Generator(np.random.PCG64(4))
    worst = 0.0
    for _ in range(3000):
        hi, hj = rng.uniform(0.02, 1.0, 2)
        r = rng.uniform(0.0, hi + hj)
        e = abs(oracle.overlap_g(hi, hj, r) - oracle.overlap_exact(hi, hj, r))
        worst = max(worst, e / oracle.overlap_exact(hi, hj, 0.0))
    assert worst < 3e-4
    assert oracle.overlap_g(0.3, 0.2, 0.5) == 0.0          # r = h_i + h_j: no overlap


def _pairs_numpy(w, h_all, targets):
    """All-pairs overlap partners with the oracle's arithmetic, in numpy."""
    out = []
    for i in targets:
        d = [np.asarray(c, dtype=np.float64) - c[i] for c in (w.x, w.y, w.z)]
        if w.periodic:
            L = w.box
            d = [np.where(v >= 0.5 * L, v - L, np.where(v < -0.5 * L, v + L, v)) for v in d]
        r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        s = h_all[i] + h_all
        m = r2 < s * s
        m[i] = False
        out.append(np.nonzero(m)[0].astype(np.int32))
    return out


@pytest.mark.parametrize("periodic", [True, False])
def test_find_overlap_against_all_pairs(periodic):
    w = W.uniform_box(700, ic_seed=61) if periodic else W.hernquist_halo(700, ic_seed=62)
    h = oracle.smoothing_lengths(w)
    tg = np.arange(0, w.n, 3, dtype=np.int32)
    ngb, cnt = oracle.find_overlap(w, h, 700, targets=tg)
    ref = _pairs_numpy(w, h, tg)
    for a in range(tg.size):
        assert cnt[a] == ref[a].size
        assert np.array_equal(ngb[a, :cnt[a]], ref[a])
        assert np.all(ngb[a, cnt[a]:] == -1)
    # the relation is symmetric, and the N_ngb + 1 nearest always overlap
    rows = {int(i): set(ref[a].tolist()) for a, i in enumerate(tg)}
    for i, s in rows.items():
        for j in s:
            if j in rows:
                assert i in rows[j]
    assert cnt.min() >= w.n_ngb + 1
    # a short row keeps the first entries and reports the full count
    short, cs = oracle.find_overlap(w, h, 8, targets=tg[:5])
    assert np.array_equal(cs, cnt[:5])
    assert np.array_equal(short, ngb[:5, :8])


def test_overlap_density_estimate_in_uniform_box():
    # sum_j m_j g_ij over the partners estimates the density (int g = 1); in a
    # uniform box of unit density it averages 1 within the sampling error
    w = W.uniform_box(20000, ic_seed=63)
    h = oracle.smoothing_lengths(w)
    tg = np.arange(0, w.n, 10, dtype=np.int32)
    ngb, cnt = oracle.find_overlap(w, h, 512, targets=tg)
    dens = np.zeros(tg.size)
    for a, i in enumerate(tg):
        js = ngb[a, :cnt[a]]
        d = [np.asarray(c, dtype=np.float64)[js] - c[i] for c in (w.x, w.y, w.z)]
        d = [np.where(v >= 0.5, v - 1.0, np.where(v < -0.5, v + 1.0, v)) for v in d]
        r = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        dens[a] = w.mass * sum(oracle.overlap_g(h[i], h[j], rr) for j, rr in zip(js, r))
    err = dens.std() / math.sqrt(tg.size)
    assert abs(dens.mean() - 1.0) < max(5 * err, 0.02), (dens.mean(), err)


def _overlap_workload(n=3000, seed=71, s=0.3):
    w = W.uniform_box(n, ic_seed=seed, scatters_per_particle=s)
    h = oracle.smoothing_lengths(w)
    ngb, cnt = oracle.find_overlap(w, h, 512)
    return w, h, ngb, cnt


def test_overlap_criterion_bounds_pair_probability():
    # with dt_i equal to the overlap form of the bound, every P(i|j) <= C_SIDM
    w, h, ngb, cnt = _overlap_workload()
    w.dt = oracle.pair_timestep_overlap(w, h, ngb, cnt)
    *_, stats = oracle.scatter_overlap(w, h, ngb, cnt, want_info=False)
    assert stats["max_p"] <= w.c_sidm * (1 + 1e-12)
    assert stats["max_p"] > 0.3 * w.c_sidm
    assert stats["n_cand"] == int(cnt.sum())


def test_overlap_step_independent_of_row_order_and_conserving():
    # the order of a target's partners changes no result (the GPU lists come
    # in tree order), and the step conserves momentum and energy
    w, h, ngb, cnt = _overlap_workload(seed=72, s=1.0)
    vx, vy, vz, st, info, stats = oracle.scatter_overlap(w, h, ngb, cnt)
    assert stats["n_events"] > 50
    rng = np.random.Generator(np.random.PCG64(9))
    sh = ngb.copy()
    perm_rows = []
    for a in range(ngb.shape[0]):
        p = rng.permutation(cnt[a])
        sh[a, :cnt[a]] = ngb[a, p]
        perm_rows.append(p)
    vx2, vy2, vz2, _, info2, stats2 = oracle.scatter_overlap(w, h, sh, cnt)
    assert np.array_equal(vx, vx2) and np.array_equal(vy, vy2) and np.array_equal(vz, vz2)
    assert stats2["n_events"] == stats["n_events"]
    for a, p in enumerate(perm_rows):
        assert np.array_equal(info2[a, :cnt[a]], info[a, p])
    p0 = np.array([w.vx.sum(), w.vy.sum(), w.vz.sum()])
    p1 = np.array([vx.sum(), vy.sum(), vz.sum()])
    assert np.abs(p1 - p0).max() < 1e-12 * np.abs(w.vx).sum()
    e0 = (w.vx**2 + w.vy**2 + w.vz**2).sum()
    assert (vx**2 + vy**2 + vz**2).sum() == pytest.approx(e0, rel=1e-13)
