"""The seeded input generators (no arithmetic of the method): requests of
the served stream drawn from one large halo sample."""
import math

import numpy as np
from scipy import stats

import workloads as W


def test_pooled_request_is_a_rotated_subset_of_the_pool():
    pool = W.hernquist_halo(200_000, ic_seed=7)
    req = W.Request(rid=3, arrival=0.0, n=20_000, s0=2.0, ic_seed=100003, philox_seed=1003,
                    steps=4)
    w = W.request_workload_pooled(req, pool)
    assert w.n == req.n and w.mass == 1.0 / req.n and w.n_active == req.n
    assert w.sigma0 == req.s0 and w.seed == req.philox_seed
    # the same draw as the generator's: radii and speeds are the pool's
    rng = W._rng(req.ic_seed)
    idx = np.sort(rng.choice(pool.n, size=req.n, replace=False))
    r_pool = np.sqrt(pool.x[idx] ** 2 + pool.y[idx] ** 2 + pool.z[idx] ** 2)
    r_req = np.sqrt(w.x ** 2 + w.y ** 2 + w.z ** 2)
    np.testing.assert_allclose(r_req, r_pool, rtol=1e-12)
    v_pool = np.sqrt(pool.vx[idx] ** 2 + pool.vy[idx] ** 2 + pool.vz[idx] ** 2)
    v_req = np.sqrt(w.vx ** 2 + w.vy ** 2 + w.vz ** 2)
    np.testing.assert_allclose(v_req, v_pool, rtol=1e-12)
    # but turned: positions differ from the pool's
    assert np.max(np.abs(w.x - pool.x[idx])) > 1e-3
    # another request draws another subset
    other = W.request_workload_pooled(W.Request(4, 0.0, 20_000, 2.0, 100004, 1004, 4), pool)
    assert not np.array_equal(np.sort(np.sqrt(other.x ** 2 + other.y ** 2 + other.z ** 2)),
                              np.sort(r_req))


def test_pooled_request_follows_the_hernquist_profile():
    """A subset of an Eddington sample is an Eddington sample: the radii of a
    request follow the truncated Hernquist mass profile M(<r) = r^2/(1+r)^2
    (G = M = a = 1) divided by M(<r_max) (KS test)."""
    pool = W.hernquist_halo(300_000, ic_seed=8)
    w = W.request_workload_pooled(W.Request(0, 0.0, 50_000, 1.0, 123, 456, 1), pool)
    r = np.sqrt(w.x ** 2 + w.y ** 2 + w.z ** 2)
    r_max = 100.0
    m_max = r_max ** 2 / (1 + r_max) ** 2
    p = stats.kstest(r, lambda q: np.minimum(q ** 2 / (1 + q) ** 2 / m_max, 1.0)).pvalue
    assert p > 1e-3
    assert r.max() <= r_max * (1 + 1e-12)
    assert math.isclose(w.mass * w.n, 1.0)
