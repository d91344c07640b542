"""Seeded synthetic inputs for the SIDM scattering step.

This module only *generates inputs*: particle positions, velocities, masses,
IDs, internal states, the active set and each active particle's timestep, plus
the scalar parameters of the step (box, cross-section model, scatter model).
It contains none of the step's own arithmetic (no neighbour search, kernel,
probability, random draw, kick or timestep criterion).  Both the CPU oracle and
the GPU library are fed from here; neither is imported by this module.

Workloads (the paper ships no initial conditions, so every one is a stand-in):

* ``uniform_box``     -- periodic unit box, uniform positions, Maxwellian
  velocities; the thermalisation box of the paper's section 5.2 with a
  Maxwellian instead of a mono-speed start.
* ``hernquist_halo``  -- isolated Hernquist (1990) halo, G=M=a=1, sampled from
  its ergodic distribution function; stands in for the isolated-halo
  core-collapse runs of section 5.3 (whose IC generator is not available).
* ``hernquist_bins``  -- power-of-two timestep bins and the active subset for a
  halo, from the collision-time scaling the paper gives in section 4.4.
* ``clustered_box``   -- periodic box of NFW haloes plus a uniform background;
  stands in for the 256^3 cosmological boxes of section 6.2.
* ``serving_requests`` -- Poisson stream of independent halo requests.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Scatter models and cross-section models (mirrors of the library enums; the
# integer values are part of the C ABI and of the oracle's interface).
XSEC_CONST = 0
XSEC_YUKAWA = 1
XSEC_TABLE = 2
MODEL_ELASTIC = 0
MODEL_EPS = 1
MODEL_TWO_STATE = 2
MODEL_BEAM = 3


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    mass: float                 # equal-mass particles
    id: np.ndarray              # uint32
    state: np.ndarray           # uint8 (internal state bit, two-state model)
    active: np.ndarray          # int32 indices into the particle arrays
    dt: np.ndarray              # float64 [n_active]
    periodic: bool = False
    box: float = 0.0
    n_ngb: int = 32
    xsec: int = XSEC_CONST
    sigma0: float = 0.0         # sigma/m (const) or s0 (Yukawa)
    w0: float = 1.0
    model: int = MODEL_ELASTIC
    eps: float = 1.0
    delta: float = 0.0
    c_sidm: float = 0.1
    seed: int = 1
    step: int = 0
    meta: dict = dataclasses.field(default_factory=dict)
    len_to_phys: float = 1.0    # stored -> physical separations and smoothing lengths
    vel_to_phys: float = 1.0    # stored -> physical relative speeds
    table_w: Optional[np.ndarray] = None       # tabulated sigma(w)/m: node speeds
    table_sigma: Optional[np.ndarray] = None   # and values (xsec = XSEC_TABLE)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_active(self) -> int:
        return int(self.active.shape[0])

    def copy(self) -> "Workload":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, (np.ndarray, dict)) else v
        return Workload(**kw)

    def subset_active(self, n_active: int) -> "Workload":
        """Same particles, first ``n_active`` entries of the active list."""
        w = self.copy()
        w.active = w.active[:n_active].copy()
        w.dt = w.dt[:n_active].copy()
        return w

    def permuted(self, seed: int) -> tuple["Workload", np.ndarray]:
        """Storage-order permutation of the particles (IDs travel along).

        Returns the permuted workload and ``perm`` with new[k] = old[perm[k]].
        The active list is remapped and itself shuffled.
        """
        rng = np.random.Generator(np.random.PCG64(seed))
        perm = rng.permutation(self.n)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(self.n)
        w = self.copy()
        for f in ("x", "y", "z", "vx", "vy", "vz", "id", "state"):
            setattr(w, f, getattr(self, f)[perm].copy())
        order = rng.permutation(self.n_active)
        w.active = inv[self.active[order]].astype(np.int32)
        w.dt = self.dt[order].copy()
        w.meta = dict(self.meta, active_order=order)
        return w, perm


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Uniform periodic box
# ---------------------------------------------------------------------------

def uniform_box(n: int = 32768, ic_seed: int = 101, philox_seed: int = 1,
                sigma_1d: float = 1.0, scatters_per_particle: float = 0.01,
                dt: float = 1.0, n_ngb: int = 32, step: int = 0,
                lattice: bool = False, mono_speed: bool = False) -> Workload:
    """Uniform periodic unit box, total mass 1 (rho = 1), Maxwellian velocities.

    sigma/m is set so that the expected number of scatters a particle takes
    part in during one step is ``scatters_per_particle``: with the rate
    rho (sigma/m) <w> of the paper's section 5.2 and the Maxwellian mean
    relative speed <w> = 4 sigma_1D / sqrt(pi), including the (1 - 1/N)
    expectation of the one-sided kernel density estimate in a finite box.

    ``lattice=True`` places the particles on a simple cubic lattice instead
    (exact distance ties; n must be a cube).  ``mono_speed=True`` gives every
    particle speed ``sigma_1d`` in an isotropic direction (the thermalisation
    start of the paper's section 5.2, mean relative speed 4 v0 / 3).
    """
    rng = _rng(ic_seed)
    if lattice:
        side = round(n ** (1.0 / 3.0))
        assert side ** 3 == n, "lattice needs a cube number of particles"
        g = (np.arange(side, dtype=np.float64) + 0.5) / side
        gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
        x, y, z = gx.ravel().copy(), gy.ravel().copy(), gz.ravel().copy()
    else:
        x = rng.random(n)
        y = rng.random(n)
        z = rng.random(n)
    if mono_speed:
        ux, uy, uz = _isotropic(rng, n)
        vx, vy, vz = sigma_1d * ux, sigma_1d * uy, sigma_1d * uz
        mean_w = 4.0 * sigma_1d / 3.0
    else:
        vx = rng.normal(0.0, sigma_1d, n)
        vy = rng.normal(0.0, sigma_1d, n)
        vz = rng.normal(0.0, sigma_1d, n)
        mean_w = 4.0 * sigma_1d / math.sqrt(math.pi)
    sigma_m = scatters_per_particle / ((1.0 - 1.0 / n) * mean_w * dt)
    return Workload(
        name=f"uniform_box_n{n}", x=x, y=y, z=z, vx=vx, vy=vy, vz=vz,
        mass=1.0 / n, id=np.arange(n, dtype=np.uint32),
        state=np.zeros(n, dtype=np.uint8),
        active=np.arange(n, dtype=np.int32), dt=np.full(n, dt),
        periodic=True, box=1.0, n_ngb=n_ngb, xsec=XSEC_CONST, sigma0=sigma_m,
        seed=philox_seed, step=step,
        meta=dict(ic_seed=ic_seed, sigma_1d=sigma_1d, lattice=lattice,
                  mono_speed=mono_speed))


# ---------------------------------------------------------------------------
# Hernquist halo (G = M = a = 1)
# ---------------------------------------------------------------------------

def hernquist_density(r):
    """rho(r) = M a / (2 pi r (r + a)^3)  (Hernquist 1990, eq. 2)."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0 / (2.0 * np.pi * r * (1.0 + r) ** 3)


def hernquist_mass(r):
    """M(<r) = M r^2 / (r + a)^2."""
    r = np.asarray(r, dtype=np.float64)
    return r * r / ((1.0 + r) ** 2)


def hernquist_sigma_r(r):
    """Isotropic Jeans radial velocity dispersion (Hernquist 1990, eq. 10)."""
    r = np.asarray(r, dtype=np.float64)
    t1 = 12.0 * r * (1.0 + r) ** 3 * np.log((1.0 + r) / r)
    t2 = (r / (1.0 + r)) * (25.0 + 52.0 * r + 42.0 * r * r + 12.0 * r ** 3)
    return np.sqrt(np.maximum(t1 - t2, 0.0) / 12.0)


def hernquist_df(eps_rel):
    """Ergodic DF f(E) of the Hernquist model (Hernquist 1990, eq. 17),
    as a function of the relative energy eps_rel = -E a / (G M) in (0, 1)."""
    q = np.sqrt(np.clip(eps_rel, 0.0, 1.0 - 1e-15))
    q2 = q * q
    pre = 1.0 / (8.0 * math.sqrt(2.0) * math.pi ** 3) * (1.0 - q2) ** (-2.5)
    br = (3.0 * np.arcsin(q)
          + q * np.sqrt(1.0 - q2) * (1.0 - 2.0 * q2) * (8.0 * q2 * q2 - 8.0 * q2 - 3.0))
    return pre * br


def _hernquist_speeds(rng, psi):
    """Speeds v at relative potential psi from p(v) ~ v^2 f(psi - v^2/2)."""
    n = psi.shape[0]
    vesc = np.sqrt(2.0 * psi)
    # envelope: max of g(x) = x^2 f(psi (1 - x^2)) on a grid, padded
    xs = np.linspace(0.0, 1.0, 65)[1:-1]
    gmax = np.zeros(n)
    for xg in xs:
        gmax = np.maximum(gmax, xg * xg * hernquist_df(psi * (1.0 - xg * xg)))
    gmax *= 1.25
    out = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        xx = rng.random(todo.size)
        uu = rng.random(todo.size)
        g = xx * xx * hernquist_df(psi[todo] * (1.0 - xx * xx))
        ok = uu * gmax[todo] < g
        out[todo[ok]] = xx[ok] * vesc[todo[ok]]
        todo = todo[~ok]
    return out


def _isotropic(rng, n):
    cth = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return sth * np.cos(phi), sth * np.sin(phi), cth


def yukawa_mean(sigma_1d: float, w0: float, n_quad: int = 4000) -> float:
    """< w / (1 + (w/w0)^2)^2 > over Maxwellian relative speeds (1D dispersion
    sqrt(2) sigma_1d), by quadrature.  Used only to normalise s0."""
    s = math.sqrt(2.0) * sigma_1d
    w = np.linspace(0.0, 12.0 * s, n_quad + 1)
    pdf = np.sqrt(2.0 / np.pi) * w * w / s ** 3 * np.exp(-w * w / (2.0 * s * s))
    f = w / (1.0 + (w / w0) ** 2) ** 2 * pdf
    return float(np.trapezoid(f, w))


def hernquist_s0(w0: float = 0.5) -> float:
    """s0 giving ~1 scatter per particle per dynamical time at r = a:
    s0 = 1 / (t_dyn(a) rho(a) < w / (1+(w/w0)^2)^2 >), t_dyn(a) = sqrt(a^3 / G M(<a))."""
    t_dyn = math.sqrt(1.0 / float(hernquist_mass(1.0)))
    rho_a = float(hernquist_density(1.0))
    sig_a = float(hernquist_sigma_r(1.0))
    return 1.0 / (t_dyn * rho_a * yukawa_mean(sig_a, w0))


def hernquist_halo(n: int = 1_000_000, ic_seed: int = 102, philox_seed: int = 2,
                   r_max: float = 100.0, w0: float = 0.5,
                   s0: Optional[float] = None, n_ngb: int = 32,
                   two_state: bool = False, delta_frac: float = 0.05,
                   step: int = 0) -> Workload:
    """Hernquist halo particles (all active, dt = 1 until binned)."""
    rng = _rng(ic_seed)
    m_trunc = float(hernquist_mass(r_max))
    xq = rng.random(n) * m_trunc            # M(<r) uniform below the truncation
    sq = np.sqrt(xq)
    r = sq / (1.0 - sq)
    ux, uy, uz = _isotropic(rng, n)
    x, y, z = r * ux, r * uy, r * uz
    psi = 1.0 / (1.0 + r)
    v = _hernquist_speeds(rng, psi)
    wx, wy, wz = _isotropic(rng, n)
    state = np.zeros(n, dtype=np.uint8)
    model, delta = MODEL_ELASTIC, 0.0
    if two_state:
        state = (rng.random(n) < 0.5).astype(np.uint8)
        model = MODEL_TWO_STATE
        delta = delta_frac * float(hernquist_sigma_r(1.0)) ** 2
    if s0 is None:
        s0 = hernquist_s0(w0)
    return Workload(
        name=f"hernquist_n{n}" + ("_2state" if two_state else ""),
        x=x, y=y, z=z, vx=v * wx, vy=v * wy, vz=v * wz, mass=1.0 / n,
        id=np.arange(n, dtype=np.uint32), state=state,
        active=np.arange(n, dtype=np.int32), dt=np.ones(n),
        periodic=False, box=0.0, n_ngb=n_ngb, xsec=XSEC_YUKAWA, sigma0=s0,
        w0=w0, model=model, delta=delta, seed=philox_seed, step=step,
        meta=dict(ic_seed=ic_seed, r_max=r_max, r=r))


def hernquist_bins(w: Workload, active_frac: float = 0.125, dt_max: float = 2.0,
                   n_ngb: int = 32, c_sidm: float = 0.1, safety: float = 0.5) -> Workload:
    """Power-of-two timestep bins from the local collision time, and the
    active set of one synchronisation point with at most ``active_frac`` of the
    particles active.

    Each particle's target step is the paper's collision-time scaling of the
    per-pair criterion (section 4.4): dt ~ (3 N_ngb C / 16) / (rho sigma(v) v),
    evaluated with the analytic density and the Maxwellian mean relative speed
    4 sigma_1D / sqrt(pi) at the particle's radius, times ``safety``: the
    scaling uses the mean relative speed where the criterion uses the largest
    one, and the factor 1/2 keeps most steps below the per-pair bound.  Bin b holds steps
    dt_max / 2^b; the active set is every particle in bins >= b*, b* being the
    smallest bin for which at most ``active_frac`` of all particles are in bins
    >= b*.
    """
    r = np.sqrt(w.x ** 2 + w.y ** 2 + w.z ** 2)
    vbar = 4.0 * hernquist_sigma_r(r) / math.sqrt(math.pi)
    sig = w.sigma0 / (1.0 + (vbar / w.w0) ** 2) ** 2
    dt_t = safety * (3.0 * n_ngb * c_sidm / 16.0) / (hernquist_density(r) * sig * vbar)
    b = np.ceil(np.log2(dt_max / dt_t)).clip(0, 40).astype(np.int64)
    counts = np.bincount(b, minlength=41)
    tail = np.cumsum(counts[::-1])[::-1]          # particles in bins >= b
    ok = np.nonzero(tail <= active_frac * w.n)[0]
    b_star = int(ok[0])
    act = np.nonzero(b >= b_star)[0].astype(np.int32)
    out = w.copy()
    out.active = act
    out.dt = dt_max / (2.0 ** b[act].astype(np.float64))
    out.name = w.name + "_bins"
    out.meta = dict(w.meta, b_star=b_star, dt_max=dt_max,
                    active_fraction=act.size / w.n)
    return out


# ---------------------------------------------------------------------------
# Beam through a static lattice (the deflection test of the paper's sec. 5.1)
# ---------------------------------------------------------------------------

def beam_lattice(n_side: int = 20, n_beam: int = 8000, ic_seed: int = 105, philox_seed: int = 5,
                 speed: float = 1.0, rate_dt: float = 0.05, dt: float = 1.0,
                 n_ngb: int = 32) -> Workload:
    """Periodic unit box: n_side^3 targets at rest on a cubic lattice (state 0)
    and n_beam beam particles at uniform random positions moving along +x with
    the same speed (state 1); equal masses, total mass 1, all active.
    sigma/m is set so that a beam particle scatters with probability about
    rate_dt per step: Gamma dt = rho_target (sigma/m) v dt = rate_dt."""
    rng = _rng(ic_seed)
    n_t = n_side ** 3
    g = (np.arange(n_side, dtype=np.float64) + 0.5) / n_side
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    n = n_t + n_beam
    x = np.concatenate([gx.ravel(), rng.random(n_beam)])
    y = np.concatenate([gy.ravel(), rng.random(n_beam)])
    z = np.concatenate([gz.ravel(), rng.random(n_beam)])
    vx = np.concatenate([np.zeros(n_t), np.full(n_beam, speed)])
    vy = np.zeros(n)
    vz = np.zeros(n)
    state = np.concatenate([np.zeros(n_t, dtype=np.uint8), np.ones(n_beam, dtype=np.uint8)])
    m = 1.0 / n
    rho_t = n_t * m
    sigma_m = rate_dt / (rho_t * speed * dt)
    return Workload(
        name=f"beam_lattice_{n_side}_{n_beam}", x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, mass=m,
        id=np.arange(n, dtype=np.uint32), state=state, active=np.arange(n, dtype=np.int32),
        dt=np.full(n, dt), periodic=True, box=1.0, n_ngb=n_ngb, xsec=XSEC_CONST,
        sigma0=sigma_m, model=MODEL_BEAM, seed=philox_seed,
        meta=dict(ic_seed=ic_seed, n_target=n_t, n_beam=n_beam, rho_target=rho_t,
                  gamma_dt=rate_dt))


# ---------------------------------------------------------------------------
# Tabulated cross-section (a velocity-dependent model given as a table)
# ---------------------------------------------------------------------------

def yukawa_table(s0: float, w0: float, n_nodes: int = 64, w_min: float = 1e-3,
                 w_max: float = 1e2):
    """Nodes log-spaced in [w_min, w_max] with the values of
    s0 / (1 + (w/w0)^2)^2 at the nodes: a table standing in for the tabulated
    cross-sections of the paper's cosmological runs (whose table is not
    available)."""
    tw = np.logspace(math.log10(w_min), math.log10(w_max), n_nodes)
    ts = s0 / (1.0 + (tw / w0) ** 2) ** 2
    return tw, ts


def with_table(w: Workload, n_nodes: int = 64) -> Workload:
    """The same workload with its Yukawa-like cross-section given as a table."""
    out = w.copy()
    out.table_w, out.table_sigma = yukawa_table(w.sigma0, w.w0, n_nodes)
    out.xsec = XSEC_TABLE
    out.name = w.name + "_table"
    return out


# ---------------------------------------------------------------------------
# Clustered periodic box: NFW haloes plus a uniform background
# ---------------------------------------------------------------------------

def nfw_mu(x):
    """Enclosed-mass shape of the NFW profile: ln(1 + x) - x / (1 + x)."""
    x = np.asarray(x, dtype=np.float64)
    return np.log1p(x) - x / (1.0 + x)


def nfw_sigma_r_table(c: float = 10.0, n: int = 512):
    """Isotropic Jeans radial dispersion of an NFW halo of concentration c in
    units of sqrt(G M_200 / r_200), on a log grid of x = r / r_s in
    [1e-3, c]:  sigma^2(x) = c x (1+x)^2 / mu(c) * int_x^inf mu(t) / (t^3 (1+t)^2) dt
    (the profile continues beyond r_200 for the pressure integral)."""
    from scipy import integrate
    xs = np.logspace(-3, math.log10(c), n)

    def f(t):
        return float(nfw_mu(t)) / (t ** 3 * (1.0 + t) ** 2)
    tail = np.array([integrate.quad(f, x, np.inf, limit=200)[0] for x in xs])
    s2 = c * xs * (1.0 + xs) ** 2 / float(nfw_mu(c)) * tail
    return xs, np.sqrt(s2)


def clustered_box(n: int = 256 ** 3, n_halo: int = 2000, ic_seed: int = 103,
                  philox_seed: int = 3, halo_frac: float = 0.7, slope: float = 1.9,
                  decades: float = 3.0, conc: float = 10.0, events_per_particle: float = 0.005,
                  dt: float = 1.0, n_ngb: int = 32, step: int = 0) -> Workload:
    """Periodic unit box, total mass 1 (mean density 1): n_halo NFW haloes
    (concentration conc) with masses from dN/dM ~ M^-slope over `decades`
    decades, rescaled to carry halo_frac of the mass, and a uniform
    background for the rest.  r_200 from a mean density of 200; radii from the
    inverse of mu(x) / mu(c); isotropic Maxwellian velocities at the local
    isotropic-Jeans dispersion; background dispersion sqrt(G M_min / r_200,min)
    / sqrt(2).  All active, constant sigma/m set so that the expected number
    of scatters per particle is events_per_particle, from the rate
    rho (sigma/m) <w> dt with each particle's analytic local density
    (its halo's profile plus the background) and Maxwellian <w> = 4 sigma /
    sqrt(pi) at its dispersion."""
    rng = _rng(ic_seed)
    # halo masses: inverse CDF of a power law on [1, 10^decades], then rescaled
    u = rng.random(n_halo)
    a1 = 1.0 - slope
    lo, hi = 1.0, 10.0 ** decades
    m_rel = (lo ** a1 + u * (hi ** a1 - lo ** a1)) ** (1.0 / a1)
    m_h = m_rel * (halo_frac / m_rel.sum())
    mp = 1.0 / n
    counts = np.maximum(1, np.round(m_h / mp).astype(np.int64))
    n_halo_p = int(counts.sum())
    if n_halo_p > n:
        raise ValueError("haloes hold more particles than n")
    n_bg = n - n_halo_p
    r200 = (3.0 * m_h / (4.0 * math.pi * 200.0)) ** (1.0 / 3.0)
    centre = rng.random((n_halo, 3))
    # radii: inverse CDF of mu(x)/mu(c) by interpolation on a fine grid
    xg = np.concatenate([[0.0], np.logspace(-5, math.log10(conc), 4000)])
    cdf = nfw_mu(xg) / float(nfw_mu(conc))
    hid = np.repeat(np.arange(n_halo), counts)
    x_in = np.interp(rng.random(n_halo_p), cdf, xg)
    ux, uy, uz = _isotropic(rng, n_halo_p)
    rs = r200[hid] / conc
    rr = x_in * rs
    pos = np.empty((n, 3))
    pos[:n_halo_p, 0] = centre[hid, 0] + rr * ux
    pos[:n_halo_p, 1] = centre[hid, 1] + rr * uy
    pos[:n_halo_p, 2] = centre[hid, 2] + rr * uz
    pos[n_halo_p:] = rng.random((n_bg, 3))
    pos = np.mod(pos, 1.0)
    pos[pos >= 1.0] = 0.0
    # velocities
    xt, st = nfw_sigma_r_table(conc)
    v200 = np.sqrt(m_h / r200)
    sig = np.empty(n)
    sig[:n_halo_p] = np.interp(np.clip(x_in, xt[0], xt[-1]), xt, st) * v200[hid]
    i_min = int(np.argmin(m_h))
    sig[n_halo_p:] = math.sqrt(m_h[i_min] / r200[i_min]) / math.sqrt(2.0)
    v = rng.normal(0.0, 1.0, (n, 3)) * sig[:, None]
    # analytic local density for the cross-section normalisation
    rho = np.full(n, 1.0 - halo_frac)
    rho_s = m_h / (4.0 * math.pi * (r200 / conc) ** 3 * float(nfw_mu(conc)))
    xx = np.maximum(x_in, 1e-4)
    rho[:n_halo_p] += rho_s[hid] / (xx * (1.0 + xx) ** 2)
    mean_rate = float(np.mean(rho * 4.0 * sig / math.sqrt(math.pi))) * dt
    sigma_m = events_per_particle / mean_rate
    perm = rng.permutation(n)                      # storage order unrelated to structure
    pos, v = pos[perm], v[perm]
    return Workload(
        name=f"clustered_box_n{n}", x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
        vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy(), mass=mp,
        id=np.arange(n, dtype=np.uint32), state=np.zeros(n, dtype=np.uint8),
        active=np.arange(n, dtype=np.int32), dt=np.full(n, dt), periodic=True, box=1.0,
        n_ngb=n_ngb, xsec=XSEC_CONST, sigma0=sigma_m, seed=philox_seed, step=step,
        meta=dict(ic_seed=ic_seed, n_halo=n_halo, n_halo_particles=n_halo_p,
                  m_min=float(m_h.min()), m_max=float(m_h.max())))


# ---------------------------------------------------------------------------
# Serving stream: independent Hernquist haloes arriving at random times
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    n: int                  # particles
    s0: float               # cross-section normalisation (Yukawa-like, w0 = 0.5)
    ic_seed: int
    philox_seed: int
    steps: int


def serving_requests(n_requests: int = 1000, rate: float = 20.0, n_min: float = 1e4,
                     n_max: float = 2e6, s0_decades: float = 2.0, steps: int = 64,
                     seed: int = 7) -> list:
    """Poisson arrivals at ``rate`` per second (exponential gaps from ``seed``);
    request r: N log-uniform in [n_min, n_max], s0 = hernquist_s0() times a
    log-uniform factor spanning ``s0_decades`` decades centred on 1, IC seed
    100000 + r, Philox seed 1000 + r."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(math.log10(n_min), math.log10(n_max), n_requests)
    logs = rng.uniform(-0.5 * s0_decades, 0.5 * s0_decades, n_requests)
    base = hernquist_s0()
    return [Request(rid=r, arrival=float(t[r]), n=int(round(10.0 ** logn[r])),
                    s0=float(base * 10.0 ** logs[r]), ic_seed=100000 + r,
                    philox_seed=1000 + r, steps=steps) for r in range(n_requests)]


def request_workload(req: Request, dt_cap: float = 0.25) -> Workload:
    """The halo of one request: all particles active, every dt = dt_cap (the
    first step; later steps take theirs from the per-pair bounds)."""
    w = hernquist_halo(req.n, ic_seed=req.ic_seed, philox_seed=req.philox_seed, s0=req.s0)
    w.dt = np.full(w.n, dt_cap)
    w.name = f"request{req.rid}_n{req.n}"
    return w


def request_workload_pooled(req: Request, pool: Workload, dt_cap: float = 0.25) -> Workload:
    """The halo of one request drawn from ``pool``, one large Eddington sample
    of the same truncated Hernquist halo (``hernquist_halo``): a random subset
    of req.n of its particles (itself an Eddington sample of that halo, so the
    particle mass is 1/N) turned by a random rotation, with the request's s0
    and Philox seed; all particles active, every dt = dt_cap.  For streams
    whose requests are too many or too large to sample one by one."""
    if req.n > pool.n:
        raise ValueError(f"request of {req.n} particles from a pool of {pool.n}")
    rng = _rng(req.ic_seed)
    idx = np.sort(rng.choice(pool.n, size=req.n, replace=False))
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))                 # a uniformly random rotation (or reflection)
    pos = q @ np.stack([pool.x[idx], pool.y[idx], pool.z[idx]])
    vel = q @ np.stack([pool.vx[idx], pool.vy[idx], pool.vz[idx]])
    n = int(req.n)
    return Workload(
        name=f"request{req.rid}_n{n}_pooled",
        x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(),
        vx=vel[0].copy(), vy=vel[1].copy(), vz=vel[2].copy(), mass=1.0 / n,
        id=np.arange(n, dtype=np.uint32), state=np.zeros(n, dtype=np.uint8),
        active=np.arange(n, dtype=np.int32), dt=np.full(n, dt_cap),
        periodic=False, box=0.0, n_ngb=pool.n_ngb, xsec=XSEC_YUKAWA, sigma0=req.s0,
        w0=pool.w0, model=MODEL_ELASTIC, delta=0.0, seed=req.philox_seed, step=0,
        meta=dict(pool=pool.name, r=np.sqrt(pos[0] ** 2 + pos[1] ** 2 + pos[2] ** 2)))
