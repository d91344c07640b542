"""Thin Python binding of libsidm.so, the gfx950 SIDM scattering-step library.

Only argument marshalling lives here: every step of the method runs in the HIP
kernels behind the C ABI declared in ``include/sidm.h``.  PyTorch provides
device memory and the HIP stream.  There is no CPU fallback: if the library
is not built, importing :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsidm.so")

SIDM_OK = 0
SIDM_E_INVAL = -1
SIDM_E_NOMEM = -2
SIDM_E_DEVICE = -3
SIDM_E_CAPACITY = -4
SIDM_E_OVERFLOW = -5
SIDM_E_STATE = -6

KERNEL_CUBIC_SPLINE = 0
XSEC_CONST, XSEC_YUKAWA, XSEC_TABLE = 0, 1, 2
MODEL_ELASTIC, MODEL_EPS, MODEL_TWO_STATE, MODEL_BEAM = 0, 1, 2, 3
FP64, MIXED = 0, 1
EST_ONE_SIDED, EST_OVERLAP = 0, 1
OVERLAP_NA, OVERLAP_NR = 64, 256

CAND_ACCEPT0 = 1
CAND_SCATTER = 2
CAND_FLAGGED = 4


class SidmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n_ngb", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("xsec", ctypes.c_int32),
                ("model", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("box", ctypes.c_double), ("sigma0", ctypes.c_double), ("w0", ctypes.c_double),
                ("eps", ctypes.c_double), ("delta", ctypes.c_double),
                ("c_sidm", ctypes.c_double), ("flag_band", ctypes.c_double),
                ("band_r2", ctypes.c_double), ("band_p", ctypes.c_double),
                ("xsec_n", ctypes.c_int32), ("xsec_w", ctypes.c_void_p),
                ("xsec_sigma", ctypes.c_void_p), ("estimator", ctypes.c_int32),
                ("len_to_phys", ctypes.c_double), ("vel_to_phys", ctypes.c_double),
                ("max_accept", ctypes.c_int64)]


class Particles(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p), ("vz", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("m_scalar", ctypes.c_double),
                ("id", ctypes.c_void_p), ("state", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int64), ("n_accept0", ctypes.c_int64),
                ("n_events", ctypes.c_int64), ("n_flagged", ctypes.c_int64),
                ("n_p_ge_1", ctypes.c_int64), ("n_recheck", ctypes.c_int64),
                ("n_passes", ctypes.c_int32), ("error", ctypes.c_int32),
                ("max_p", ctypes.c_double), ("n_rounds", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tree_ms", ctypes.c_double), ("map_ms", ctypes.c_double),
                ("knn_ms", ctypes.c_double), ("eval_ms", ctypes.c_double),
                ("resolve_ms", ctypes.c_double), ("timestep_ms", ctypes.c_double),
                ("overlap_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# phase masks of Context.timing_enable (SIDM_TIMING_* in include/sidm.h)
TIMING_TREE, TIMING_MAP, TIMING_KNN, TIMING_EVAL = 1, 2, 4, 8
TIMING_RESOLVE, TIMING_TIMESTEP, TIMING_OVERLAP, TIMING_ALL = 16, 32, 64, 127

# Every symbol include/sidm.h declares (tests check the library exports them).
EXPORTS = ["sidm_footprint", "sidm_create", "sidm_destroy", "sidm_set_stream", "sidm_reconfigure",
           "sidm_last_error", "sidm_status_string", "sidm_build_tree", "sidm_find_ngb",
           "sidm_refit_tree", "sidm_tree_order", "sidm_scatter_step", "sidm_pair_timestep",
           "sidm_advance_hernquist", "sidm_advance_hernquist_noalloc", "sidm_drift",
           "sidm_find_overlap", "sidm_scatter_overlap", "sidm_pair_timestep_overlap",
           "sidm_overlap_table",
           "sidm_sync",
           "sidm_timing_enable", "sidm_timing_read"]

_lib = None


def lib():
    """Load libsidm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, u64, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        CP = ctypes.POINTER(Config)
        L.sidm_footprint.argtypes = [CP, i64, i64, ctypes.POINTER(ctypes.c_size_t)]
        L.sidm_create.argtypes = [CP, i64, i64, P, ctypes.POINTER(ctypes.c_void_p)]
        L.sidm_destroy.argtypes = [P]
        L.sidm_set_stream.argtypes = [P, P]
        L.sidm_reconfigure.argtypes = [P, CP]
        L.sidm_last_error.argtypes = [P]
        L.sidm_last_error.restype = ctypes.c_char_p
        L.sidm_status_string.argtypes = [ctypes.c_int]
        L.sidm_status_string.restype = ctypes.c_char_p
        L.sidm_build_tree.argtypes = [P, ctypes.POINTER(Particles)]
        L.sidm_refit_tree.argtypes = [P, ctypes.POINTER(Particles)]
        L.sidm_tree_order.argtypes = [P, P]
        L.sidm_find_ngb.argtypes = [P, P, i64, P, P]
        L.sidm_scatter_step.argtypes = [P, ctypes.POINTER(Particles), P, i64, P, P, P, u64, u32, P]
        L.sidm_pair_timestep.argtypes = [P, P, i64, P, P, P]
        d = ctypes.c_double
        L.sidm_advance_hernquist.argtypes = [P, P, P, P, P, P, P, i64, P, i64, d, d, d, P, P]
        L.sidm_advance_hernquist_noalloc.argtypes = [P, P, P, P, P, P, P, i64, P, i64, d, d, d,
                                                     P, P]
        L.sidm_drift.argtypes = [P, P, P, P, P, P, P, i64, d]
        L.sidm_find_overlap.argtypes = [P, P, P, P, i64, ctypes.c_int32, P, P]
        L.sidm_scatter_overlap.argtypes = [P, ctypes.POINTER(Particles), P, P, i64,
                                           ctypes.c_int32, P, P, P, u64, u32, P]
        L.sidm_pair_timestep_overlap.argtypes = [P, P, P, i64, ctypes.c_int32, P, P, P]
        L.sidm_overlap_table.argtypes = [P, P]
        L.sidm_sync.argtypes = [P, ctypes.POINTER(Stats)]
        L.sidm_timing_enable.argtypes = [P, ctypes.c_int]
        L.sidm_timing_read.argtypes = [P, ctypes.POINTER(Timing)]
        for name in EXPORTS:
            if name not in ("sidm_last_error", "sidm_status_string"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_config(n_ngb=32, periodic=False, box=0.0, xsec=XSEC_CONST, sigma0=0.0, w0=1.0,
                model=MODEL_ELASTIC, eps=1.0, delta=0.0, c_sidm=0.1, precision=FP64,
                flag_band=1e-9, band_r2=1e-5, band_p=1e-5, table_w=None,
                table_sigma=None, estimator=EST_ONE_SIDED, len_to_phys=1.0,
                vel_to_phys=1.0, max_accept=0) -> Config:
    """A sidm_config.  table_w / table_sigma (numpy arrays) give a tabulated
    cross-section (xsec = XSEC_TABLE); the Config keeps them alive.
    estimator = EST_OVERLAP reserves what the overlap-estimator calls need.
    len_to_phys / vel_to_phys: stored -> physical factors of lengths and
    relative speeds (comoving storage).  max_accept: candidates a step can
    list for its ordered replay (0: the library's default)."""
    tw = ts = None
    n_t = 0
    if table_w is not None:
        tw = np.ascontiguousarray(table_w, dtype=np.float64)
        ts = np.ascontiguousarray(table_sigma, dtype=np.float64)
        n_t = int(tw.shape[0])
    c = Config(int(n_ngb), KERNEL_CUBIC_SPLINE, int(bool(periodic)), int(xsec), int(model),
               int(precision), float(box), float(sigma0), float(w0), float(eps), float(delta),
               float(c_sidm), float(flag_band), float(band_r2), float(band_p), n_t,
               tw.ctypes.data if tw is not None else None,
               ts.ctypes.data if ts is not None else None, int(estimator),
               float(len_to_phys), float(vel_to_phys), int(max_accept))
    c._tables = (tw, ts)
    return c


def footprint(cfg: Config, cap_n: int, cap_active: int) -> int:
    out = ctypes.c_size_t(0)
    st = lib().sidm_footprint(ctypes.byref(cfg), int(cap_n), int(cap_active), ctypes.byref(out))
    if st != SIDM_OK:
        raise SidmError(st, "sidm_footprint")
    return int(out.value)


def advance_hernquist_noalloc(x, y, z, vx, vy, vz, dt_sidm, n_active: int, dt_cap: float,
                              gm: float, a: float, dt_next=None, dt_step=None, stream=None):
    """sidm_advance_hernquist_noalloc: the served form's step between two
    scattering steps without a context and without allocating (the
    reduction's scratch is the library's fixed device array).  Tensors are
    contiguous float64 on the current device; stream defaults to torch's."""
    import torch
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (vx, "vx"), (vy, "vy"), (vz, "vz"),
                  (dt_sidm, "dt_sidm"), (dt_next, "dt_next"), (dt_step, "dt_step")):
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError(f"{nm}: need a contiguous float64 device tensor")
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib().sidm_advance_hernquist_noalloc(
        ctypes.c_void_p(stream.cuda_stream), _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy),
        _ptr(vz), int(x.shape[0]), _ptr(dt_sidm), int(n_active), float(dt_cap), float(gm),
        float(a), _ptr(dt_next), _ptr(dt_step))
    if st != SIDM_OK:
        raise SidmError(st, "sidm_advance_hernquist_noalloc: " +
                        lib().sidm_status_string(st).decode())


def _act(active, reuse: bool):
    """The active list's pointer, or NULL to reuse the mapping of the previous
    call on the context (its length still gives n_active)."""
    return None if reuse else _ptr(active)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


class Context:
    """One sidm_ctx: scratch for up to ``cap_n`` particles / ``cap_active`` targets,
    bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, cfg: Config, cap_n: int, cap_active: int, stream=None):
        import torch
        self.cfg = cfg
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib().sidm_create(ctypes.byref(cfg), int(cap_n), int(cap_active),
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != SIDM_OK:
            raise SidmError(st, "sidm_create")
        self._h = h
        self._particles = None

    # -- helpers -----------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != SIDM_OK:
            msg = lib().sidm_last_error(self._h).decode()
            raise SidmError(st, f"{what}: {msg}")

    @staticmethod
    def _dev(t, dtype, name):
        if t is None:
            return None
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name}: need a contiguous {dtype} device tensor")
        return t

    def close(self):
        if getattr(self, "_h", None):
            lib().sidm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        self._check(lib().sidm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)),
                    "sidm_set_stream")

    def reconfigure(self, cfg: Config):
        self._check(lib().sidm_reconfigure(self._h, ctypes.byref(cfg)), "sidm_reconfigure")
        self.cfg = cfg

    # -- the four calls of the step ----------------------------------------------
    def build_tree(self, x, y, z, vx, vy, vz, ids, state=None, mass=None, m_scalar=0.0):
        self._tree_call("sidm_build_tree", x, y, z, vx, vy, vz, ids, state, mass, m_scalar)

    def refit_tree(self, x, y, z, vx, vy, vz, ids, state=None, mass=None, m_scalar=0.0):
        """Tree reuse: snapshot and boxes in the order of the last build_tree."""
        self._tree_call("sidm_refit_tree", x, y, z, vx, vy, vz, ids, state, mass, m_scalar)

    def _tree_call(self, fn, x, y, z, vx, vy, vz, ids, state, mass, m_scalar):
        torch = self._torch
        f64 = torch.float64
        arrs = dict(x=self._dev(x, f64, "x"), y=self._dev(y, f64, "y"), z=self._dev(z, f64, "z"),
                    vx=self._dev(vx, f64, "vx"), vy=self._dev(vy, f64, "vy"),
                    vz=self._dev(vz, f64, "vz"), id=self._dev(ids, torch.int32, "id"),
                    state=self._dev(state, torch.uint8, "state"),
                    mass=self._dev(mass, f64, "mass"))
        p = Particles(_ptr(arrs["x"]), _ptr(arrs["y"]), _ptr(arrs["z"]), _ptr(arrs["vx"]),
                      _ptr(arrs["vy"]), _ptr(arrs["vz"]), _ptr(arrs["mass"]), float(m_scalar),
                      _ptr(arrs["id"]), _ptr(arrs["state"]), int(x.shape[0]))
        self._particles = (p, arrs)      # keep tensors alive while the snapshot is in use
        self._check(getattr(lib(), fn)(self._h, ctypes.byref(p)), fn)
        if fn == "sidm_build_tree":
            self._n_sorted = int(x.shape[0])

    def find_ngb(self, active, ngb, h):
        torch = self._torch
        self._dev(active, torch.int32, "active")
        self._dev(ngb, torch.int32, "ngb")
        self._dev(h, torch.float64, "h")
        self._check(lib().sidm_find_ngb(self._h, _ptr(active), int(active.shape[0]), _ptr(ngb),
                                        _ptr(h)), "sidm_find_ngb")

    def scatter_step(self, active, ngb, h, dt, seed: int, step: int, cand_info=None,
                     reuse_active: bool = False):
        torch = self._torch
        if self._particles is None:
            raise SidmError(SIDM_E_STATE, "scatter_step before build_tree")
        self._dev(active, torch.int32, "active")
        self._dev(ngb, torch.int32, "ngb")
        self._dev(h, torch.float64, "h")
        self._dev(dt, torch.float64, "dt")
        self._dev(cand_info, torch.int32, "cand_info")
        p = self._particles[0]
        self._check(lib().sidm_scatter_step(self._h, ctypes.byref(p), _act(active, reuse_active),
                                            int(active.shape[0]), _ptr(ngb), _ptr(h), _ptr(dt),
                                            int(seed) & (2**64 - 1), int(step) & (2**32 - 1),
                                            _ptr(cand_info)), "sidm_scatter_step")

    def pair_timestep(self, active, ngb, h, dt_sidm, reuse_active: bool = False):
        torch = self._torch
        self._dev(active, torch.int32, "active")
        self._dev(ngb, torch.int32, "ngb")
        self._dev(h, torch.float64, "h")
        self._dev(dt_sidm, torch.float64, "dt_sidm")
        self._check(lib().sidm_pair_timestep(self._h, _act(active, reuse_active), int(active.shape[0]),
                                             _ptr(ngb), _ptr(h), _ptr(dt_sidm)),
                    "sidm_pair_timestep")

    # --- kernel-overlap estimator -------------------------------------------
    def find_overlap(self, h_all, active, ngb, count, h_active=None, reuse_active: bool = False):
        """Partners with r_ij < h_i + h_j: ngb int32[n_active, max_ngb] (rows in
        tree order), count int32[n_active] (full counts).  h_active (optional)
        is first written into h_all at the active particles."""
        torch = self._torch
        self._dev(h_all, torch.float64, "h_all")
        self._dev(h_active, torch.float64, "h_active")
        self._dev(active, torch.int32, "active")
        self._dev(ngb, torch.int32, "ngb")
        self._dev(count, torch.int32, "count")
        self._check(lib().sidm_find_overlap(self._h, _ptr(h_all), _act(active, reuse_active),
                                            _ptr(h_active),
                                            int(active.shape[0]), int(ngb.shape[1]), _ptr(ngb),
                                            _ptr(count)), "sidm_find_overlap")

    def scatter_overlap(self, h_all, active, ngb, count, dt, seed: int, step: int,
                        cand_info=None, reuse_active: bool = False):
        torch = self._torch
        if self._particles is None:
            raise SidmError(SIDM_E_STATE, "scatter_overlap before build_tree")
        for t, dtp, nm in ((h_all, torch.float64, "h_all"), (active, torch.int32, "active"),
                           (ngb, torch.int32, "ngb"), (count, torch.int32, "count"),
                           (dt, torch.float64, "dt"), (cand_info, torch.int32, "cand_info")):
            self._dev(t, dtp, nm)
        p = self._particles[0]
        self._check(lib().sidm_scatter_overlap(self._h, ctypes.byref(p), _ptr(h_all),
                                               _act(active, reuse_active), int(active.shape[0]),
                                               int(ngb.shape[1]), _ptr(ngb), _ptr(count),
                                               _ptr(dt), int(seed) & (2**64 - 1),
                                               int(step) & (2**32 - 1), _ptr(cand_info)),
                    "sidm_scatter_overlap")

    def pair_timestep_overlap(self, h_all, active, ngb, count, dt_sidm,
                              reuse_active: bool = False):
        torch = self._torch
        for t, dtp, nm in ((h_all, torch.float64, "h_all"), (active, torch.int32, "active"),
                           (ngb, torch.int32, "ngb"), (count, torch.int32, "count"),
                           (dt_sidm, torch.float64, "dt_sidm")):
            self._dev(t, dtp, nm)
        self._check(lib().sidm_pair_timestep_overlap(self._h, _ptr(h_all),
                                                     _act(active, reuse_active),
                                                     int(active.shape[0]), int(ngb.shape[1]),
                                                     _ptr(ngb), _ptr(count), _ptr(dt_sidm)),
                    "sidm_pair_timestep_overlap")

    def tree_order(self, order):
        """order[s] = caller index of the particle at sorted position s (the
        n particles of the last build_tree; a device int32 tensor of n)."""
        self._dev(order, self._torch.int32, "order")
        n = getattr(self, "_n_sorted", 0)
        if order.numel() < n:
            raise ValueError(f"order: need {n} entries, got {order.numel()}")
        self._check(lib().sidm_tree_order(self._h, _ptr(order)), "sidm_tree_order")

    def overlap_table(self) -> np.ndarray:
        out = np.zeros((OVERLAP_NA + 1, OVERLAP_NR + 1), dtype=np.float64)
        self._check(lib().sidm_overlap_table(self._h, out.ctypes.data), "sidm_overlap_table")
        return out

    def advance_hernquist(self, x, y, z, vx, vy, vz, dt_sidm, n_active: int, dt_cap: float,
                          gm: float, a: float, dt_next=None, dt_step=None):
        """Served form: global step length from the per-pair bounds, then one
        kick-drift-kick step in the potential -gm / (r + a)."""
        torch = self._torch
        f64 = torch.float64
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (vx, "vx"), (vy, "vy"), (vz, "vz"),
                      (dt_sidm, "dt_sidm"), (dt_next, "dt_next"), (dt_step, "dt_step")):
            self._dev(t, f64, nm)
        self._check(lib().sidm_advance_hernquist(
            self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), int(x.shape[0]),
            _ptr(dt_sidm), int(n_active), float(dt_cap), float(gm), float(a), _ptr(dt_next),
            _ptr(dt_step)), "sidm_advance_hernquist")

    def drift(self, x, y, z, vx, vy, vz, dt: float):
        """Free drift x += v dt (wrapped into the periodic box)."""
        f64 = self._torch.float64
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (vx, "vx"), (vy, "vy"), (vz, "vz")):
            self._dev(t, f64, nm)
        self._check(lib().sidm_drift(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy),
                                     _ptr(vz), int(x.shape[0]), float(dt)), "sidm_drift")

    def timing_enable(self, phases=True):
        """Time the phases in the mask (TIMING_*); True for all, False or 0 for none."""
        if phases is True:
            phases = TIMING_ALL
        elif phases is False:
            phases = 0
        self._check(lib().sidm_timing_enable(self._h, int(phases)), "sidm_timing_enable")

    def timing_read(self) -> dict:
        t = Timing()
        self._check(lib().sidm_timing_read(self._h, ctypes.byref(t)), "sidm_timing_read")
        return t.as_dict()

    def sync(self) -> dict:
        s = Stats()
        st = lib().sidm_sync(self._h, ctypes.byref(s))
        d = s.as_dict()
        self._check(st, "sidm_sync")
        return d
