"""Shared helpers of the GPU tests: run a workload through the C ABI and
compare with the CPU oracle."""
import numpy as np

import oracle
from paper_2607_05504_amd import Context, runner, FP64


def gpu_step(w, with_info=True, precision=FP64, ctx=None, seed=None, step=None, **cfg_kw):
    import torch
    ds = runner.upload(w, "cuda")
    own = ctx is None
    if own:
        ctx = Context(runner.config_for(w, precision=precision, **cfg_kw), w.n, max(1, w.n_active))
    out = runner.alloc_out(ds, w.n_ngb, with_info=with_info)
    runner.run_step(ctx, ds, out, w.seed if seed is None else seed,
                    w.step if step is None else step)
    stats = ctx.sync()
    res = dict(ngb=out.ngb.cpu().numpy(), h=out.h.cpu().numpy(),
               vx=ds.vx.cpu().numpy(), vy=ds.vy.cpu().numpy(), vz=ds.vz.cpu().numpy(),
               state=ds.state.cpu().numpy(), dt_sidm=out.dt_sidm.cpu().numpy(),
               info=(out.cand_info.cpu().numpy().view(np.uint32) if with_info else None),
               stats=stats)
    if own:
        ctx.close()
    torch.cuda.synchronize()
    return res


def assert_parity(w, g, ref, vel_rtol=1e-12, dt_rtol=1e-12, mixed=False, p_rtol=0.0):
    """The parity bar: neighbour sets and h bit-exact; decisions bit-exact
    except on flagged candidates; every particle's velocity and every dt to
    1e-12 relative (|v_gpu - v_ref| <= 1e-12 |v_ref| per particle).
    ``mixed``: the FP32 form, whose unrechecked probabilities are FP32 values,
    so the largest P is compared to 1e-5 and the P >= 1 count is not.
    ``p_rtol``: the largest P to that relative tolerance instead of bit for
    bit (a tabulated cross-section takes ln w from the device's log, the
    oracle from the C library's, which may differ in the last bit)."""
    assert np.array_equal(g["ngb"], ref["ngb"]), "neighbour lists differ"
    assert np.array_equal(g["h"], ref["h"]), "smoothing lengths differ"
    gi, ri = g["info"], ref["info"]
    flagged = ((gi | ri) & oracle.CAND_FLAGGED) != 0
    same = (gi == ri) | flagged
    assert same.all(), f"{(~same).sum()} candidate decisions differ"
    if flagged.any():
        # a flagged candidate that decided differently may change everything
        # downstream; none is expected with bit-identical probabilities
        assert ((gi ^ ri) & ~np.uint32(oracle.CAND_FLAGGED))[flagged].sum() == 0
    dv = np.sqrt((g["vx"] - ref["vx"]) ** 2 + (g["vy"] - ref["vy"]) ** 2 + (g["vz"] - ref["vz"]) ** 2)
    sp = np.sqrt(ref["vx"] ** 2 + ref["vy"] ** 2 + ref["vz"] ** 2)
    bad = dv > vel_rtol * sp
    assert not bad.any(), (f"{bad.sum()} velocities beyond {vel_rtol} relative, worst "
                           f"{(dv[bad] / np.maximum(sp[bad], 1e-300)).max()}")
    assert np.array_equal(g["state"], ref["state"]), "internal states differ"
    d_g, d_r = g["dt_sidm"], ref["dt_sidm"]
    fin = np.isfinite(d_r)
    assert np.array_equal(np.isfinite(d_g), fin)
    np.testing.assert_allclose(d_g[fin], d_r[fin], rtol=dt_rtol, atol=0)
    gs, rs = g["stats"], ref["stats"]
    assert gs["n_cand"] == rs["n_cand"]
    assert gs["n_accept0"] == rs["n_accept0"]
    assert gs["n_events"] == rs["n_events"]
    assert gs["n_passes"] == rs["n_passes"]
    if mixed:
        assert abs(gs["max_p"] - rs["max_p"]) <= 1e-5 * rs["max_p"]
    else:
        assert gs["n_p_ge_1"] == rs["n_p_ge_1"]
        assert abs(gs["max_p"] - rs["max_p"]) <= p_rtol * rs["max_p"]
    assert gs["error"] == 0
