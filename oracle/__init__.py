"""Python side of the CPU oracle (test infrastructure only).

The oracle is a plain FP64 C implementation of the SIDM scattering step
(``sidm_oracle.c``), written from the paper and shared with nothing in the GPU
library.  Only the tests, the package smoke check and the benchmark's
CPU-baseline leg use it.  This module only marshals arguments, builds the C
file with gcc, and -- for inputs too large for an all-pairs ranking -- gathers
a *superset* of each target's candidate partners with scipy's k-d tree; the
exact ranking by (r^2, ID) over that superset is still the C oracle's.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sidm_oracle.c")
_LIB = os.path.join(_HERE, "libsidm_oracle.so")
# the same source built with -fopenmp: the CPU throughput baseline on all
# cores (identical results; the turns of a step stay serial)
_LIB_OMP = os.path.join(_HERE, "libsidm_oracle_omp.so")
_lib = None
_which = _LIB

XSEC_TABLE = 2
CAND_ACCEPT0 = 1
CAND_SCATTER = 2
CAND_FLAGGED = 4


def build(force: bool = True) -> str:
    """Compile the oracle: no FMA contraction, no fast-math; and its OpenMP
    build."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out):
            cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *extra,
                   "-fPIC", "-shared", "-o", out + ".tmp", _SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(out + ".tmp", out)
    return _LIB


def use_openmp(threads: int = 0) -> int:
    """Switch to the OpenMP build (threads > 0 sets its thread count, else
    all cores); returns the threads it will use."""
    global _lib, _which
    if _which != _LIB_OMP:
        _lib, _which = None, _LIB_OMP
    return int(lib().oref_threads(int(threads)))


_turn_mode = 0


def set_turn_mode(mode: int) -> int:
    """How the scatter step visits the serial order (same results): 0 every
    candidate in turn (the default), 1 only those whose turn can differ from
    the step-start evaluation (for steps of many millions of candidates)."""
    global _turn_mode
    _turn_mode = int(mode)
    return int(lib().oref_set_turn_mode(_turn_mode))


def use_serial() -> None:
    """Back to the single-threaded build (the default)."""
    global _lib, _which
    if _which != _LIB:
        _lib, _which = None, _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int64), ("n_accept0", ctypes.c_int64),
                ("n_events", ctypes.c_int64), ("n_flagged", ctypes.c_int64),
                ("n_p_ge_1", ctypes.c_int64), ("n_passes", ctypes.c_int32),
                ("max_p", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_which) or os.path.getmtime(_which) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_which)
        P = ctypes.c_void_p
        i64, i32, u32, u64, dbl = (ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.oref_threads.argtypes = [i32]
        L.oref_threads.restype = i32
        L.oref_set_turn_mode.argtypes = [i32]
        L.oref_set_turn_mode.restype = i32
        L.oref_set_turn_mode(_turn_mode)
        L.oref_philox4x32_10.argtypes = [P, P, P]
        L.oref_philox4x32_10.restype = None
        L.oref_uniform_decision.argtypes = [u64, u32, u32, u32]
        L.oref_uniform_decision.restype = dbl
        L.oref_r2.argtypes = [dbl] * 6 + [i32, dbl]
        L.oref_r2.restype = dbl
        L.oref_kernel.argtypes = [dbl, dbl]
        L.oref_kernel.restype = dbl
        L.oref_sigma.argtypes = [dbl, i32, dbl, dbl]
        L.oref_sigma.restype = dbl
        L.oref_find_ngb.argtypes = [i64, P, P, P, P, i32, dbl, i64, P, i32, P, P, P, P]
        L.oref_find_ngb.restype = i32
        L.oref_scatter_step.argtypes = ([i64, P, P, P, P, P, P, P, dbl, P, P, i32, dbl,
                                         i64, P, i32, P, P, P,
                                         i32, dbl, dbl, i32, dbl, dbl, u64, u32, dbl,
                                         P, ctypes.POINTER(_Stats)])
        L.oref_scatter_step.restype = i32
        L.oref_pair_timestep.argtypes = [i64, P, P, P, P, dbl, i64, P, i32, P, P,
                                         i32, dbl, dbl, dbl, P]
        L.oref_pair_timestep.restype = i32
        L.oref_kick_pair.argtypes = [i32, i32, P, dbl, P, P, P, P, P, i32, dbl, dbl, u64, u32]
        L.oref_kick_pair.restype = None
        L.oref_set_table.argtypes = [P, P, i32]
        L.oref_set_table.restype = i32
        L.oref_set_units.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oref_set_units.restype = i32
        L.oref_overlap_exact.argtypes = [dbl, dbl, dbl]
        L.oref_overlap_exact.restype = dbl
        L.oref_overlap_g.argtypes = [dbl, dbl, dbl]
        L.oref_overlap_g.restype = dbl
        L.oref_overlap_table.argtypes = [P]
        L.oref_overlap_table.restype = None
        L.oref_find_overlap.argtypes = [i64, P, P, P, i32, dbl, P, i64, P, i32, P, P]
        L.oref_find_overlap.restype = i64
        L.oref_scatter_overlap.argtypes = ([i64, P, P, P, P, P, P, P, dbl, P, P, i32, dbl,
                                            P, i64, P, i32, P, P, P,
                                            i32, dbl, dbl, i32, dbl, dbl, u64, u32, dbl,
                                            P, ctypes.POINTER(_Stats)])
        L.oref_scatter_overlap.restype = i32
        L.oref_pair_timestep_overlap.argtypes = [i64, P, P, P, P, dbl, P, i64, P, i32, P, P,
                                                 i32, dbl, dbl, dbl, P]
        L.oref_pair_timestep_overlap.restype = i32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
def philox4x32_10(counter, key) -> np.ndarray:
    c = _c(counter, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oref_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform_decision(seed: int, step: int, id_i: int, id_j: int) -> float:
    return lib().oref_uniform_decision(seed, step, id_i, id_j)


def kernel(r: float, h: float) -> float:
    return lib().oref_kernel(r, h)


def sigma(w: float, xsec: int, s0: float, w0: float) -> float:
    return lib().oref_sigma(w, xsec, s0, w0)


def set_table(table_w, table_sigma) -> None:
    """Load a tabulated cross-section (used when xsec is the table model)."""
    tw = np.ascontiguousarray(table_w, dtype=np.float64)
    ts = np.ascontiguousarray(table_sigma, dtype=np.float64)
    st = lib().oref_set_table(_p(tw), _p(ts), int(tw.shape[0]))
    if st != 0:
        raise ValueError("invalid cross-section table")


def _masses(w):
    """Per-particle masses of w (an optional ``masses`` array), else None:
    the scalar w.mass is used."""
    m = getattr(w, "masses", None)
    return None if m is None else np.ascontiguousarray(m, dtype=np.float64)


def set_units(len_to_phys: float = 1.0, vel_to_phys: float = 1.0) -> None:
    """Stored -> physical factors for separations and smoothing lengths, and
    for relative speeds (sec. 4.2: comoving storage, physical pair rate)."""
    if lib().oref_set_units(float(len_to_phys), float(vel_to_phys)) != 0:
        raise ValueError("unit factors must be > 0 and finite")


def _use_table(w) -> None:
    """The workload's tabulated cross-section (if any) and unit factors."""
    if getattr(w, "table_w", None) is not None and int(w.xsec) == XSEC_TABLE:
        set_table(w.table_w, w.table_sigma)
    set_units(getattr(w, "len_to_phys", 1.0), getattr(w, "vel_to_phys", 1.0))


def r2(pi, pj, periodic: bool, box: float) -> float:
    return lib().oref_r2(*map(float, pi), *map(float, pj), int(periodic), float(box))


# ---------------------------------------------------------------------------
def kd_tree(x, y, z, periodic, box):
    """scipy's k-d tree over all particles (the candidate gathering below)."""
    from scipy.spatial import cKDTree
    pts = np.stack([x, y, z], axis=1)
    if periodic:
        pts = np.where(pts >= box, pts - box, pts)
        return cKDTree(pts, boxsize=box), pts
    return cKDTree(pts), pts


def candidate_superset(x, y, z, periodic, box, targets, k, workers=-1, kd=None):
    """CSR superset of every target's partners with r <= r_(k+1), from scipy's
    k-d tree: the (k+2)-th closest point including the target itself bounds
    r_(k+1), and the radius is padded far beyond rounding differences.  A
    row is the k+8 closest points when the last of them lies beyond the padded
    radius (then every point within it is among them), else a ball query.
    kd: a tree from kd_tree() of the same particles, else one is built."""
    kd, pts = kd if kd is not None else kd_tree(x, y, z, periodic, box)
    q = pts[targets]
    kk = min(k + 8, len(pts))
    d, nb = kd.query(q, k=kk, workers=workers)
    rad = d[:, k + 1] * (1.0 + 1e-9) + 1e-300
    ok = d[:, kk - 1] > rad
    counts = np.full(len(q), kk, dtype=np.int64)
    rest = np.flatnonzero(~ok)
    lists = kd.query_ball_point(q[rest], rad[rest], workers=workers, return_sorted=False) \
        if rest.size else []
    for r, l in zip(rest, lists):
        counts[r] = len(l)
    ptr = np.zeros(len(q) + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    okr = np.flatnonzero(ok)
    # rows of kk entries: their slots in idx
    pos = (ptr[okr][:, None] + np.arange(kk)[None, :]).ravel()
    idx[pos] = nb[okr].ravel()
    for r, l in zip(rest, lists):
        idx[ptr[r]:ptr[r + 1]] = np.asarray(l, dtype=np.int32)
    return ptr, idx


def find_ngb(w, targets=None, brute: Optional[bool] = None, workers: int = -1, kd=None):
    """Neighbour lists and smoothing lengths of ``targets`` (default: w.active).

    Returns (ngb int32[n_t, k], h float64[n_t])."""
    L = lib()
    tg = _c(w.active if targets is None else targets, np.int32)
    k = w.n_ngb
    x, y, z = _c(w.x, np.float64), _c(w.y, np.float64), _c(w.z, np.float64)
    ids = _c(w.id, np.uint32)
    if brute is None:
        brute = w.n <= 4096
    ptr = idx = None
    if not brute:
        ptr, idx = candidate_superset(x, y, z, w.periodic, w.box, tg, k, workers, kd=kd)
    ngb = np.zeros((tg.size, k), dtype=np.int32)
    h = np.zeros(tg.size, dtype=np.float64)
    rc = L.oref_find_ngb(w.n, _p(x), _p(y), _p(z), _p(ids), int(w.periodic), float(w.box),
                         tg.size, _p(tg), k, _p(ptr), _p(idx), _p(ngb), _p(h))
    if rc != 0:
        raise ValueError(f"oref_find_ngb failed ({rc})")
    return ngb, h


def scatter_step(w, ngb, h, band: float = 1e-9, want_info: bool = True):
    """One scattering step on copies of w's velocities/states.

    Returns (vx, vy, vz, state, cand_info uint32[n_active, k] | None, stats dict)."""
    _use_table(w)
    L = lib()
    x, y, z = _c(w.x, np.float64), _c(w.y, np.float64), _c(w.z, np.float64)
    vx, vy, vz = (np.array(w.vx, dtype=np.float64), np.array(w.vy, dtype=np.float64),
                  np.array(w.vz, dtype=np.float64))
    st = np.array(w.state, dtype=np.uint8)
    ids = _c(w.id, np.uint32)
    act = _c(w.active, np.int32)
    ngb = _c(ngb, np.int32)
    h = _c(h, np.float64)
    dt = _c(w.dt, np.float64)
    info = np.zeros((act.size, w.n_ngb), dtype=np.uint32) if want_info else None
    stats = _Stats()
    rc = L.oref_scatter_step(w.n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(_masses(w)),
                             float(w.mass), _p(ids), _p(st), int(w.periodic), float(w.box),
                             act.size, _p(act), w.n_ngb, _p(ngb), _p(h), _p(dt),
                             int(w.xsec), float(w.sigma0), float(w.w0), int(w.model),
                             float(w.eps), float(w.delta), int(w.seed), int(w.step),
                             float(band), _p(info), ctypes.byref(stats))
    if rc != 0:
        raise ValueError(f"oref_scatter_step failed ({rc})")
    sd = {f: getattr(stats, f) for f, _ in _Stats._fields_}
    return vx, vy, vz, st, info, sd


def pair_timestep(w, ngb, h, vx=None, vy=None, vz=None):
    _use_table(w)
    L = lib()
    vx = _c(w.vx if vx is None else vx, np.float64)
    vy = _c(w.vy if vy is None else vy, np.float64)
    vz = _c(w.vz if vz is None else vz, np.float64)
    act = _c(w.active, np.int32)
    ngb = _c(ngb, np.int32)
    h = _c(h, np.float64)
    out = np.zeros(act.size, dtype=np.float64)
    rc = L.oref_pair_timestep(w.n, _p(vx), _p(vy), _p(vz), _p(_masses(w)), float(w.mass), act.size,
                              _p(act), w.n_ngb, _p(ngb), _p(h), int(w.xsec),
                              float(w.sigma0), float(w.w0), float(w.c_sidm), _p(out))
    if rc != 0:
        raise ValueError(f"oref_pair_timestep failed ({rc})")
    return out


def kick_pair(i, j, vx, vy, vz, state, ids, mass, model, eps, delta, seed, step):
    """Kick particles i and j in place (arrays are modified)."""
    set_units(1.0, 1.0)                  # a pair kick in physical units
    lib().oref_kick_pair(int(i), int(j), None, float(mass), _p(vx), _p(vy), _p(vz),
                         _p(state), _p(ids), int(model), float(eps), float(delta),
                         int(seed), int(step))


def full_step(w, brute: Optional[bool] = None, band: float = 1e-9, workers: int = -1, kd=None):
    """Neighbours, scatter step and per-pair timestep of workload w (kd: a
    prebuilt kd_tree of its particles)."""
    ngb, h = find_ngb(w, brute=brute, workers=workers, kd=kd)
    vx, vy, vz, st, info, stats = scatter_step(w, ngb, h, band=band)
    dt = pair_timestep(w, ngb, h, vx, vy, vz)
    return dict(ngb=ngb, h=h, vx=vx, vy=vy, vz=vz, state=st, info=info, stats=stats,
                dt_sidm=dt)


def step_length(dt_sidm, dt_cap: float) -> float:
    """Global step of the served form: the largest dt_cap / 2^b (b = 0..62)
    not above the smallest per-pair bound (sec. 4.4 bound; powers of two as in
    the hierarchical steps of sec. 3.2); dt_cap if there is no bound."""
    m = float(np.min(dt_sidm)) if len(dt_sidm) else np.inf
    d = float(dt_cap)
    b = 0
    while not d <= m and b < 62:
        d *= 0.5
        b += 1
    return d


def advance_hernquist(x, y, z, vx, vy, vz, dt_sidm, dt_cap: float, gm: float, a: float):
    """Served form, between two scattering steps: one kick-drift-kick leapfrog
    step of length step_length(dt_sidm, dt_cap) in the Hernquist (1990)
    potential Phi = -gm / (r + a), whose acceleration is
    -gm / (r (r + a)^2) times the position vector.  Returns new arrays and d."""
    d = step_length(dt_sidm, dt_cap)
    hd = 0.5 * d

    def force(px, py, pz):
        r = np.sqrt((px * px + py * py) + pz * pz)
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(r > 0.0, -gm / (r * ((r + a) * (r + a))), 0.0)
        return f

    x, y, z = (np.asarray(v, dtype=np.float64).copy() for v in (x, y, z))
    vx, vy, vz = (np.asarray(v, dtype=np.float64).copy() for v in (vx, vy, vz))
    f = force(x, y, z)
    vx = vx + hd * (f * x)
    vy = vy + hd * (f * y)
    vz = vz + hd * (f * z)
    x = x + d * vx
    y = y + d * vy
    z = z + d * vz
    f = force(x, y, z)
    vx = vx + hd * (f * x)
    vy = vy + hd * (f * y)
    vz = vz + hd * (f * z)
    return x, y, z, vx, vy, vz, d


def drift(x, y, z, vx, vy, vz, dt: float, periodic: bool, box: float):
    """Free drift between scattering steps (the thermalisation box of the
    paper's sec. 5.2 moves its particles ballistically): x + dt v, wrapped into
    [0, box) when periodic."""
    out = []
    for p, v in ((x, vx), (y, vy), (z, vz)):
        q = np.asarray(p, dtype=np.float64) + dt * np.asarray(v, dtype=np.float64)
        if periodic:
            q = q - box * np.floor(q / box)
            q = np.where(q >= box, q - box, np.where(q < 0.0, 0.0, q))
        out.append(q)
    return tuple(out)


# ---------------------------------------------------------------------------
# Kernel-overlap estimator (the paper's Eq. kernelOverlap and its appendix)
OVERLAP_NA = 64     # alpha nodes a / 128, a = 0..64, over [0, 1/2]
OVERLAP_NR = 256    # rho nodes b / 256, b = 0..256, over [0, 1]


def overlap_exact(hi: float, hj: float, r: float) -> float:
    """Overlap integral of two cubic splines, by quadrature exact for its
    piecewise-polynomial integrand (no table)."""
    return lib().oref_overlap_exact(float(hi), float(hj), float(r))


def overlap_g(hi: float, hj: float, r: float) -> float:
    """g_ij of the estimator: the tabulated dimensionless overlap, bilinear."""
    return lib().oref_overlap_g(float(hi), float(hj), float(r))


def overlap_table() -> np.ndarray:
    """The oracle's table ghat[alpha node, rho node]."""
    out = np.zeros((OVERLAP_NA + 1, OVERLAP_NR + 1), dtype=np.float64)
    lib().oref_overlap_table(_p(out))
    return out


def smoothing_lengths(w, workers: int = -1) -> np.ndarray:
    """h of every particle (active or not), in particle order."""
    _, h = find_ngb(w, targets=np.arange(w.n, dtype=np.int32), workers=workers)
    return h


def find_overlap(w, h_all, max_ngb: int, targets=None):
    """Overlap partners (r_ij < h_i + h_j) of ``targets`` (default w.active) by
    brute force, in increasing particle index.  Returns (ngb int32[n_t,
    max_ngb] padded with -1, count int32[n_t])."""
    tg = _c(w.active if targets is None else targets, np.int32)
    x, y, z = _c(w.x, np.float64), _c(w.y, np.float64), _c(w.z, np.float64)
    ha = _c(h_all, np.float64)
    ngb = np.full((tg.size, max_ngb), -1, dtype=np.int32)
    cnt = np.zeros(tg.size, dtype=np.int32)
    lib().oref_find_overlap(w.n, _p(x), _p(y), _p(z), int(w.periodic), float(w.box), _p(ha),
                            tg.size, _p(tg), int(max_ngb), _p(ngb), _p(cnt))
    return ngb, cnt


def scatter_overlap(w, h_all, ngb, count, band: float = 1e-9, want_info: bool = True):
    """One scattering step with the overlap estimator on copies of w's
    velocities/states.  Returns (vx, vy, vz, state, cand_info | None, stats)."""
    _use_table(w)
    x, y, z = _c(w.x, np.float64), _c(w.y, np.float64), _c(w.z, np.float64)
    vx, vy, vz = (np.array(w.vx, dtype=np.float64), np.array(w.vy, dtype=np.float64),
                  np.array(w.vz, dtype=np.float64))
    st = np.array(w.state, dtype=np.uint8)
    ids = _c(w.id, np.uint32)
    act = _c(w.active, np.int32)
    ngb = _c(ngb, np.int32)
    cnt = _c(count, np.int32)
    ha = _c(h_all, np.float64)
    dt = _c(w.dt, np.float64)
    m = ngb.shape[1]
    info = np.zeros((act.size, m), dtype=np.uint32) if want_info else None
    stats = _Stats()
    rc = lib().oref_scatter_overlap(w.n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), None,
                                    float(w.mass), _p(ids), _p(st), int(w.periodic),
                                    float(w.box), _p(ha), act.size, _p(act), m, _p(ngb),
                                    _p(cnt), _p(dt), int(w.xsec), float(w.sigma0),
                                    float(w.w0), int(w.model), float(w.eps), float(w.delta),
                                    int(w.seed), int(w.step), float(band), _p(info),
                                    ctypes.byref(stats))
    if rc != 0:
        raise ValueError(f"oref_scatter_overlap failed ({rc})")
    sd = {f: getattr(stats, f) for f, _ in _Stats._fields_}
    return vx, vy, vz, st, info, sd


def pair_timestep_overlap(w, h_all, ngb, count, vx=None, vy=None, vz=None):
    _use_table(w)
    vx = _c(w.vx if vx is None else vx, np.float64)
    vy = _c(w.vy if vy is None else vy, np.float64)
    vz = _c(w.vz if vz is None else vz, np.float64)
    act = _c(w.active, np.int32)
    ngb = _c(ngb, np.int32)
    cnt = _c(count, np.int32)
    ha = _c(h_all, np.float64)
    out = np.zeros(act.size, dtype=np.float64)
    rc = lib().oref_pair_timestep_overlap(w.n, _p(vx), _p(vy), _p(vz), None, float(w.mass),
                                          _p(ha), act.size, _p(act), ngb.shape[1], _p(ngb),
                                          _p(cnt), int(w.xsec), float(w.sigma0), float(w.w0),
                                          float(w.c_sidm), _p(out))
    if rc != 0:
        raise ValueError(f"oref_pair_timestep_overlap failed ({rc})")
    return out
