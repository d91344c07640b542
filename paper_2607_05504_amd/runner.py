"""Device-resident state and one full SIDM step through the C ABI.

``DeviceState`` holds a set of particles as torch device tensors (the caller's
arrays of the ABI) and ``Step`` the per-step outputs; ``run_step`` issues
sidm_build_tree -> sidm_find_ngb -> sidm_scatter_step -> sidm_pair_timestep on
the context's stream.  Only marshalling: the arithmetic is in the kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import Context, make_config, FP64


@dataclasses.dataclass
class DeviceState:
    x: "torch.Tensor"
    y: "torch.Tensor"
    z: "torch.Tensor"
    vx: "torch.Tensor"
    vy: "torch.Tensor"
    vz: "torch.Tensor"
    ids: "torch.Tensor"
    state: "torch.Tensor"
    active: "torch.Tensor"
    dt: "torch.Tensor"
    mass: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_active(self) -> int:
        return int(self.active.shape[0])


@dataclasses.dataclass
class StepOut:
    ngb: "torch.Tensor"
    h: "torch.Tensor"
    dt_sidm: "torch.Tensor"
    cand_info: Optional["torch.Tensor"]


def upload(w, device="cuda") -> DeviceState:
    """Copy a workload's host arrays (numpy) to device tensors."""
    import torch

    def f64(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)

    return DeviceState(
        x=f64(w.x), y=f64(w.y), z=f64(w.z), vx=f64(w.vx), vy=f64(w.vy), vz=f64(w.vz),
        ids=torch.from_numpy(np.ascontiguousarray(w.id, dtype=np.uint32).view(np.int32)).to(device),
        state=torch.from_numpy(np.ascontiguousarray(w.state, dtype=np.uint8)).to(device),
        active=torch.from_numpy(np.ascontiguousarray(w.active, dtype=np.int32)).to(device),
        dt=f64(w.dt), mass=float(w.mass))


def config_for(w, precision=FP64, **kw):
    return make_config(n_ngb=w.n_ngb, periodic=w.periodic, box=w.box, xsec=w.xsec,
                       sigma0=w.sigma0, w0=w.w0, model=w.model, eps=w.eps, delta=w.delta,
                       c_sidm=w.c_sidm, precision=precision,
                       table_w=getattr(w, "table_w", None),
                       table_sigma=getattr(w, "table_sigma", None),
                       len_to_phys=getattr(w, "len_to_phys", 1.0),
                       vel_to_phys=getattr(w, "vel_to_phys", 1.0), **kw)


def alloc_out(ds: DeviceState, k: int, with_info: bool = False) -> StepOut:
    import torch
    dev = ds.x.device
    na = ds.n_active
    return StepOut(ngb=torch.empty((na, k), dtype=torch.int32, device=dev),
                   h=torch.empty(na, dtype=torch.float64, device=dev),
                   dt_sidm=torch.empty(na, dtype=torch.float64, device=dev),
                   cand_info=(torch.empty((na, k), dtype=torch.int32, device=dev)
                              if with_info else None))


def run_step(ctx: Context, ds: DeviceState, out: StepOut, seed: int, step: int,
             refit: bool = False):
    """One whole step (all four calls) on ctx's stream; no host synchronisation.
    refit: reuse the order of the last tree build (sidm_refit_tree)."""
    tree = ctx.refit_tree if refit else ctx.build_tree
    tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state, m_scalar=ds.mass)
    ctx.find_ngb(ds.active, out.ngb, out.h)
    # the later calls reuse find_ngb's mapping of the active set
    ctx.scatter_step(ds.active, out.ngb, out.h, ds.dt, seed, step, cand_info=out.cand_info,
                     reuse_active=True)
    ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)


@dataclasses.dataclass
class OverlapOut:
    everyone: "torch.Tensor"     # int32[n] 0..n-1 (all particles as targets)
    ngb_all: "torch.Tensor"      # int32[n, n_ngb] neighbour lists of every particle
    h_all: "torch.Tensor"        # float64[n] every particle's smoothing length
    ngb_k: "torch.Tensor"        # int32[n_active, n_ngb] neighbours of the active ones
    h_k: "torch.Tensor"          # float64[n_active] their new smoothing lengths
    ngb: "torch.Tensor"          # int32[n_active, max_ngb] overlap partners
    count: "torch.Tensor"        # int32[n_active]
    dt_sidm: "torch.Tensor"
    cand_info: Optional["torch.Tensor"]


def alloc_overlap(ds: DeviceState, k: int, max_ngb: int, with_info: bool = False) -> OverlapOut:
    import torch
    dev = ds.x.device
    n, na = ds.n, ds.n_active
    return OverlapOut(
        everyone=torch.arange(n, dtype=torch.int32, device=dev),
        ngb_all=torch.empty((n, k), dtype=torch.int32, device=dev),
        h_all=torch.empty(n, dtype=torch.float64, device=dev),
        ngb_k=torch.empty((na, k), dtype=torch.int32, device=dev),
        h_k=torch.empty(na, dtype=torch.float64, device=dev),
        ngb=torch.empty((na, max_ngb), dtype=torch.int32, device=dev),
        count=torch.empty(na, dtype=torch.int32, device=dev),
        dt_sidm=torch.empty(na, dtype=torch.float64, device=dev),
        cand_info=(torch.empty((na, max_ngb), dtype=torch.int32, device=dev)
                   if with_info else None))


def run_overlap_step(ctx: Context, ds: DeviceState, out: OverlapOut, seed: int, step: int,
                     smoothing: str = "all"):
    """One step with the kernel-overlap estimator: the tree, smoothing
    lengths, the overlap partners of the active particles, the scattering
    step and the per-pair timestep.  smoothing = "all": every particle's h
    from sidm_find_ngb over all of them (the context needs cap_active = n);
    "active": only the active particles' h, written into out.h_all by
    sidm_find_overlap (the others keep the values out.h_all holds)."""
    ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state,
                   m_scalar=ds.mass)
    if smoothing == "all":
        ctx.find_ngb(out.everyone, out.ngb_all, out.h_all)
        ctx.find_overlap(out.h_all, ds.active, out.ngb, out.count)
    else:
        ctx.find_ngb(ds.active, out.ngb_k, out.h_k)
        ctx.find_overlap(out.h_all, ds.active, out.ngb, out.count, h_active=out.h_k,
                         reuse_active=True)
    ctx.scatter_overlap(out.h_all, ds.active, out.ngb, out.count, ds.dt, seed, step,
                        cand_info=out.cand_info, reuse_active=True)
    ctx.pair_timestep_overlap(out.h_all, ds.active, out.ngb, out.count, out.dt_sidm,
                              reuse_active=True)
