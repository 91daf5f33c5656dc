"""Helpers shared by the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare under the near-tie rule."""
from __future__ import annotations

import numpy as np

from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

TOL = 2e-5   # max |GPU - oracle| per RGBA channel for FP32 arithmetic


def cam_of(v: synth.ViewSpec) -> rc.Camera:
    return rc.Camera(v.modelview, v.projection, v.width, v.height)


def gpu_render(vol, brick, views, tf_rgba, vmin, vmax, storage="f32", src="device", max_tiles=0,
               keep=False, options=None, op=None, dt_ref=1.0):
    import torch
    dims = vol.shape[::-1]
    bc = binding.BrickCaster(0)
    src_dtype = "f16" if vol.dtype == np.float16 else "f32"
    bc.plan(dims, brick, storage=storage, src_dtype=src_dtype, max_views=len(views),
            max_w=views[0].width, max_h=views[0].height, max_tiles=max_tiles)
    bc.bind()
    if src == "device":
        t = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
        bc.load(t)
        del t
    else:
        bc.load(np.ascontiguousarray(vol))
    for k, val in (options or {}).items():
        bc.set_option(k, val)
    if op is not None:
        bc.set_operator(*op)
    bc.set_transfer_function(tf_rgba, vmin, vmax, dt_ref)
    bc.set_views(views)
    out = bc.render()
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    if keep:
        return img, bc
    bc.close()
    return img


def compare(gpu_pixels, res: rc.RenderResult, label: str = ""):
    """Max |GPU - oracle| over every pixel under the near-tie rule (a near-tie
    ray may match any of its enumerated results).  Prints how many pixels were
    compared and how many were near-tie rays, and fails if any ray's branch
    enumeration overflowed: no pixel is exempt from the comparison.
    Returns (max error, n_tie, n_overflow)."""
    err = rc.max_abs_with_branches(gpu_pixels, res)
    n_tie, n_ovf = int(res.tie.sum()), int(res.overflow.sum())
    print(f"{label}: {len(err)} pixels compared, max err {err.max():.3g}, {n_tie} near-tie rays, "
          f"{n_ovf} overflowed", flush=True)
    assert n_ovf == 0, f"{label}: near-tie enumeration overflowed on {n_ovf} rays"
    return float(err.max()), n_tie, n_ovf


def compare_mip(gpu_pixels, res, label: str = ""):
    """compare() for maximum intensity projection (its branch lists never
    overflow: they are the reachable maxima, listed without combinations)."""
    from oracle import mip
    err = mip.max_abs_with_branches(gpu_pixels, res)
    print(f"{label}: {len(err)} pixels compared, max err {err.max():.3g}, {int(res.tie.sum())} near-tie rays",
          flush=True)
    return float(err.max())
