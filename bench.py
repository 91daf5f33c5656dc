#!/usr/bin/env python3
"""Frame-rate benchmark of the bricked ray caster on one MI355X.

Workload (default): a 1024^3 float32 spectral-cube stand-in (N(0,1) noise plus
500 Gaussian sources, 5% of voxels above 3), bricked into 4x4x4 bricks of
256^3 voxels with 1-voxel ghosts, rendered perspective at 1920x1080 with a
0.5-voxel step and early ray termination at opacity 0.99, over a 64-frame
orbit.  One step is one frame of the whole per-frame path: the FP64 set-up
(inverse view transform, visibility order, rendering rectangles, work list),
the per-brick ray casting into sub-images, and the sort-last compositing into
the output image.  The cube is resident in GPU memory before timing starts.

Prints one JSON line.  ``value`` is nominal samples (samples composited up to
early termination, empty-space-skipped ones included) per second over the
timed frames, in Gsamples/s.  The roofline object refers to the ray-casting
kernel; its algorithmic bytes per launch are the core voxels of every brick
whose rendering rectangle is non-empty (each voxel read once) plus the
sub-image tiles written (1 KiB per 64-pixel tile); on the paper's frame-size
and cube-shape workloads the voxel bytes are capped at one voxel per nominal
sample (those frames sample their bricks far less than once per voxel).  ``cpu_baseline`` is the FP64
oracle timed on a bounded random sample of the first frame's pixels, in
processes forked over the host cores before the GPU is touched.

On the default workload the line also carries ``forms``: the same orbit
rendered from FP16 and FP8-E4M3 bricks (each from its own context, loaded
from the same cube) and as learned frames (half-size coarse render plus the
trained upsampler, validated against plain tiles at 40 dB), each with its
milliseconds per frame, its speedup over plain FP32, its PSNR against the
plain FP32 frames and (storage forms) against the FP64 oracle on the FP32
cube, and whether it counts as chosen (PSNR >= 40 dB against plain on every
frame compared).

``--op mip`` runs the same path with maximum intensity projection (the
paper's operator: per-ray maximum, any-order merge, colour map after the
merge), with ``--step-policy voxel`` at one sample per voxel slice per ray.

    python bench.py [--gpus 1] [--steps 64] [--warmup 3] [--storage f32|f16|fp8]
                    [--op composite|mip] [--step-policy fixed|voxel]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import multiprocessing as mp
import os
import sys
import time

# the oracle's 4x4 products gain nothing from BLAS threads, and forked
# oracle workers must not inherit a BLAS thread pool
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1205_0282_amd import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
ORBIT = 64

# HBM bytes per launch of the ray-casting kernel, measured with rocprofv3
# counters: DRAM reads TCC_EA0_RDREQ_DRAM_32B x 32 plus DRAM writes
# TCC_EA0_WRREQ_WRITE_DRAM_32B x 32 (both count 32-byte units; on a plain
# 1 GiB device copy they read back 1.000 GiB each, so no scale is applied),
# mean over the render launches of
# `bench.py --warmup 0 --repeats 0 --cpu-seconds 0 --check-pixels 0 --forms 0
# [options]` (the 64-frame orbit, twice).  Valid only for the kernel sources
# whose SHA-256 is recorded; any other source reports null.
MEASURED_TRAFFIC = {
    "sources_sha256": "767e94236e551325df5546ab4f23daecb7fa462b135a0d3dbcbd0212cd0f23b7",
    "bytes": {   # "workload/storage/operator/step policy" -> bytes per launch
        "cube1024_persp1920x1080/f32/composite/fixed": 2379458324,
        "cube1024_persp1920x1080/f16/composite/fixed": 1530188545,
        "cube1024_persp1920x1080/fp8/composite/fixed": 1029400961,
        "cube1024_persp1920x1080/f32/mip/voxel": 2545890382,
        "cube3000x3000x1500_f16_4views/f16/composite/fixed": 55999454989,
    },
    # L2 (TCC) hit rate over the same launches: TCC_HIT / (TCC_HIT + TCC_MISS)
    "l2_hit_rate": {
        "cube1024_persp1920x1080/f32/composite/fixed": 0.7599,
        "cube1024_persp1920x1080/f16/composite/fixed": 0.8084,
        "cube1024_persp1920x1080/fp8/composite/fixed": 0.8265,
        "cube1024_persp1920x1080/f32/mip/voxel": 0.6784,
        "cube3000x3000x1500_f16_4views/f16/composite/fixed": 0.6583,
    },
}
KERNEL_SOURCES = ("bc_render.hip", "bc_types.h", "bc_kernels.h", "bc_df.h", "bc_e4m3.h")


def kernel_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1205_0282_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str, what: str = "bytes"):
    if MEASURED_TRAFFIC["sources_sha256"] != kernel_sha256():
        return None
    return MEASURED_TRAFFIC[what].get(key)

WORKLOADS = {
    # name: (recipe, brick edge, width, height, views per launch, source dtype)
    "cube1024_persp1920x1080": (synth.RECIPE_1024, 256, 1920, 1080, 1, "f32"),
    "cube128_ortho256": (synth.RECIPE_SMALL, 64, 256, 256, 1, "f32"),
    # 3000 x 3000 x 1500 FP16 cube (27 GB), 12 x 12 x 6 bricks of 256^3 with
    # uneven edge bricks, four orbit views 90 degrees apart per launch
    "cube3000x3000x1500_f16_4views": (synth.RECIPE_BATCH, 256, 1920, 1080, 4, "f16"),
    # the paper's frame sizes (1024^2 in its node-scaling figure, 2048^2 in
    # its frame-size figure) and the shapes of its test cubes (Table 1)
    "cube1024_persp1024x1024": (synth.RECIPE_1024, 256, 1024, 1024, 1, "f32"),
    "cube1024_persp2048x2048": (synth.RECIPE_1024, 256, 2048, 2048, 1, "f32"),
    "hipass1721x1721x1025_persp1024x1024": (synth.RECIPE_HIPASS, 256, 1024, 1024, 1, "f32"),
    "gass2502x2501x1093_persp1024x1024": (synth.RECIPE_GASS, 256, 1024, 1024, 1, "f32"),
    "nbody2600_f16_persp1024x1024": (synth.RECIPE_NBODY2600, 256, 1024, 1024, 1, "f16"),
}


# workloads outside the hot-path scope's measurement table (the paper's frame
# sizes and cube shapes): algorithmic voxel bytes capped at one voxel per sample
SAMPLE_CAPPED = {"cube1024_persp1024x1024", "cube1024_persp2048x2048", "hipass1721x1721x1025_persp1024x1024",
                 "gass2502x2501x1093_persp1024x1024", "nbody2600_f16_persp1024x1024"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=ORBIT)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--storage", choices=("f32", "f16", "fp8"), default="f32")
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="cube1024_persp1920x1080")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target wall time of the oracle sample (0 disables the CPU baseline)")
    p.add_argument("--cpu-workers", type=int, default=0,
                   help="0 = every core this process may use (affinity mask, capped by the cgroup CPU quota)")
    p.add_argument("--forms", type=int, choices=(0, 1), default=1,
                   help="1: also time FP16, FP8 and learned frames on the default workload (plain FP32 only)")
    p.add_argument("--op", choices=("composite", "mip"), default="composite",
                   help="ray operator: front-to-back compositing, or maximum intensity projection")
    p.add_argument("--step-policy", choices=("fixed", "voxel"), default="fixed",
                   help="fixed 0.5-voxel step, or one sample per voxel slice per ray (mip only)")
    p.add_argument("--learned", action="store_true",
                   help="time learned frames: coarse render + trained upsampler, validated against plain tiles")
    p.add_argument("--weights", default=os.path.join(ROOT, "paper_1205_0282_amd", "weights", "upsampler.npy"))
    p.add_argument("--psnr-threshold", type=float, default=40.0)
    p.add_argument("--graph", action="store_true", help="replay captured HIP graphs for the timed frames")
    p.add_argument("--tile-width", type=int, choices=(4, 8, 16), default=8,
                   help="screen tile of one wave: 4x16, 8x8 (default) or 16x4 pixels")
    p.add_argument("--xcd-queues", type=int, choices=(0, 1), default=1,
                   help="1: one work queue of whole bricks per XCD (default); 0: a single queue")
    p.add_argument("--autotune", action="store_true", help="pick the launch shape by timing candidates first")
    p.add_argument("--repeats", type=int, default=10,
                   help="frames per orbit angle for the median/p75 statistic (0 skips it)")
    p.add_argument("--frames", type=int, default=ORBIT,
                   help="distinct orbit frames cycled through (the first N of the 64-frame orbit)")
    p.add_argument("--check-pixels", type=int, default=1024,
                   help="sampled pixels of frame 0 compared with the FP64 oracle on the FP32 cube (0 disables)")
    return p.parse_args()


def host_cores() -> int:
    """Cores this process may run on: the affinity mask, capped by the cgroup
    CPU quota when one is set (a container's share of a larger host)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            quota, period = fh.read().split()[:2]
        if quota != "max":
            n = min(n, max(1, int(float(quota) / float(period))))
    except (OSError, ValueError):
        pass
    return max(1, n)


def views_for(recipe, width, height, kind):
    return [synth.orbit_view(recipe.dims, k, ORBIT, kind=kind, width=width, height=height, step=0.5, ert=0.99)
            for k in range(ORBIT)]


def view_sets(recipe, width, height, per_launch, n, kind):
    """Launch i renders orbit frames i, i + 64/v, ... (v views per launch)."""
    orbit = views_for(recipe, width, height, kind)
    stride = ORBIT // per_launch
    n_sets = max(1, min(stride, n))
    return [[orbit[i + j * stride] for j in range(per_launch)] for i in range(n_sets)]


# ------------------------------------------------------------------ CPU oracle
_CPU = {}


def _oracle_render(pix):
    """The bricked FP64 oracle of the benchmarked operator at some pixels."""
    from oracle import mip
    from oracle import raycast as rc
    c = _CPU
    if c["op"] == "mip":
        step = "voxel" if c["step_policy"] == "voxel" else 0.5
        return mip.render_mip_bricked(c["stored"], c["dims"], c["cam"], c["tf"], step, pixels=pix)
    return rc.render_bricked(c["stored"], c["dims"], c["cam"], c["tf"], 0.5, 0.99, pixels=pix)


def _cpu_chunk(pix):
    t0 = time.perf_counter()
    res = _oracle_render(pix)
    return int(res.samples.sum()), time.perf_counter() - t0


def _ref_chunk(pix):
    """Oracle pixels (main result and near-tie branches) for the precision check."""
    res = _oracle_render(pix)
    return res.image, {int(k): v for k, v in res.branches.items()}


def oracle_reference(vol, recipe, brick, view, rgba, vmin, vmax, n_px, workers, args):
    """FP64 oracle on the source cube (FP32, or an FP16 source as it is) at a seeded
    sample of hit pixels of one frame."""
    from oracle import raycast as rc
    dims = recipe.dims
    _CPU.update(stored=rc.store_bricks(vol, rc.brick_grid(dims, (brick,) * 3)), dims=dims,
                op=args.op, step_policy=args.step_policy,
                cam=rc.Camera(view.modelview, view.projection, view.width, view.height),
                tf=rc.TransferFunction(rgba, vmin, vmax))
    cam = _CPU["cam"]
    rng = np.random.default_rng(777)
    cand = np.stack([rng.integers(0, view.width, 8 * n_px), rng.integers(0, view.height, 8 * n_px)], axis=1)
    o, d = cam.rays(cand[:, 0], cand[:, 1])
    _, _, hit = rc.global_interval(o, d, dims)
    pix = cand[hit][:n_px]
    chunks = np.array_split(pix, workers * 2)
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_ref_chunk, chunks)
    img = np.concatenate([o[0] for o in out])
    branches, base = {}, 0
    for (im, br), ch in zip(out, chunks):
        for k, v in br.items():
            branches[base + k] = v
        base += len(ch)
    _CPU.clear()
    return pix, img, branches


def precision_report(gpu_px, ref_img, branches):
    """max |GPU - oracle| (near-tie rays: closest branch) and PSNR (peak 1)."""
    err = np.max(np.abs(gpu_px - ref_img), axis=1)
    for r, alts in branches.items():
        if alts:
            err[r] = min(err[r], min(float(np.max(np.abs(gpu_px[r] - a))) for a in alts))
    mse = float(np.mean((gpu_px - ref_img) ** 2))
    return {"pixels": int(len(ref_img)), "max_abs": float(err.max()),
            "psnr_db": (float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)), "near_tie_rays": len(branches)}


def cpu_baseline(vol, recipe, brick, view, rgba, vmin, vmax, seconds, workers, args):
    from oracle import raycast as rc
    dims = recipe.dims
    _CPU.update(stored=rc.store_bricks(vol, rc.brick_grid(dims, (brick,) * 3)), dims=dims,
                op=args.op, step_policy=args.step_policy,
                cam=rc.Camera(view.modelview, view.projection, view.width, view.height),
                tf=rc.TransferFunction(rgba, vmin, vmax))
    rng = np.random.default_rng(20240601)
    # calibration on a few pixels (not counted)
    cal = np.stack([rng.integers(0, view.width, 48), rng.integers(0, view.height, 48)], axis=1)
    _, tc = _cpu_chunk(cal)
    per_px = tc / len(cal)
    n_px = max(workers * 16, int(seconds * workers / max(per_px, 1e-6)))
    pix = np.stack([rng.integers(0, view.width, n_px), rng.integers(0, view.height, n_px)], axis=1)
    chunks = np.array_split(pix, workers * 4)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        out = pool.map(_cpu_chunk, chunks)
    wall = time.perf_counter() - t0
    samples = sum(o[0] for o in out)
    _CPU.clear()
    return {"value": samples / wall / 1e9, "unit": "Gsamples/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_px} uniformly drawn pixels of orbit frame 0 (seeded), FP64 bricked "
                      f"{'maximum-intensity' if args.op == 'mip' else 'compositing'} oracle with "
                      f"near-tie branches, {samples} samples in {wall:.1f} s over {workers} forked processes"}


# ------------------------------------------------------------------ learned frames
def setup_learned(bc, args, views, out, W, H):
    """Loads the trained upsampler, measures its quality on every orbit frame
    against the plain render (untimed) and switches the context to learned
    frames.  Returns the quality summary."""
    import torch
    import torch.nn.functional as F
    w = np.load(args.weights, allow_pickle=False).astype(np.float32)
    bc.cnn_setup(1, H // 2, W // 2)
    bc.cnn_set_weights(w)
    plain, psnr_net, psnr_bil, psnr_val, fell = [], [], [], [], 0
    for v in views:
        bc.set_learned(False)
        bc.set_views([v])
        ref = bc.render(out).clone()
        bc.set_learned(True, 2.0, args.psnr_threshold, 8)
        img = bc.render(out).clone()
        st = bc.stats()
        fell += int(st["fell_back"] == 1)
        psnr_val.append(st["psnr_db"])
        # the network alone and the bilinear baseline, from the same coarse render
        cv = dataclasses.replace(v, width=W // 2, height=H // 2, step=2.0)
        bc.set_learned(False)
        bc.set_views([cv])
        coarse = bc.render(torch.empty((1, H // 2, W // 2, 4), dtype=torch.float32, device=out.device)).clone()
        net = bc.cnn_forward(coarse)
        bil = F.interpolate(coarse.permute(0, 3, 1, 2), scale_factor=2, mode="bilinear",
                            align_corners=False).permute(0, 2, 3, 1)
        for lst, a in ((psnr_net, net), (psnr_bil, bil)):
            mse = float(((a - ref) ** 2).mean())
            lst.append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
        del img
    bc.set_learned(True, 2.0, args.psnr_threshold, 8)
    summary = {"weights": os.path.relpath(args.weights, ROOT), "coarse": [W // 2, H // 2], "coarse_step": 2.0,
               "psnr_threshold_db": args.psnr_threshold, "validate_stride": 8,
               "psnr_network_vs_plain_db": {"mean": float(np.mean(psnr_net)), "min": float(np.min(psnr_net))},
               "psnr_bilinear_vs_plain_db": {"mean": float(np.mean(psnr_bil)), "min": float(np.min(psnr_bil))},
               "psnr_validation_db_mean": float(np.mean(psnr_val)), "fell_back_frames": fell,
               "frames": len(views)}
    log(f"learned: {summary}")
    return summary


# ------------------------------------------------------------------ other forms
def timed_frames(bc, sets, out, steps, warmup):
    """Wall-clock ms per frame over `steps` frames after `warmup` (inputs
    resident), with the per-frame ms of the ray-casting kernel from HIP events
    around it in the timed frames (stage list: set-up and compositing read 0)."""
    import torch
    nf = len(sets)
    for i in range(warmup):
        bc.set_views(sets[i % nf])
        bc.render(out)
    torch.cuda.synchronize()
    bc.enable_timing(True, stages=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        bc.set_views(sets[i % nf])
        bc.render(out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, n = bc.timing()
    bc.enable_timing(False)
    return elapsed / steps * 1e3, [m / n for m in stage_ms]


def psnr_db(a, b) -> float:
    """PSNR (peak 1) of two device images over every pixel and channel."""
    mse = float(((a.double() - b.double()) ** 2).mean())
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def storage_leg(storage, args, recipe, brick, W, H, sets, vol, rgba, vmin, vmax, ref, plain_imgs, base_ms):
    """The orbit rendered from `storage` bricks in a context of its own: ms per
    frame, speedup over plain FP32, PSNR against the plain FP32 frames and
    against the FP64 oracle on the FP32 cube."""
    import torch
    from paper_1205_0282_amd import binding
    dev = torch.device("cuda", 0)
    bc = binding.BrickCaster(0)
    bc.plan(recipe.dims, (brick,) * 3, storage=storage, src_dtype="f32", max_views=1, max_w=W, max_h=H)
    bc.bind()
    src = torch.from_numpy(vol).to(dev)
    bc.load(src)
    torch.cuda.synchronize()
    del src
    bc.set_transfer_function(rgba, vmin, vmax)
    out = torch.empty((1, H, W, 4), dtype=torch.float32, device=dev)
    samples = []
    for vs in sets:
        bc.set_views(vs)
        bc.render(out)
        samples.append(bc.stats()["nominal_samples"])
    ms, stage = timed_frames(bc, sets, out, args.steps, args.warmup)
    nf = len(sets)
    gsps = sum(samples[i % nf] for i in range(args.steps)) / args.steps / (ms * 1e-3) / 1e9
    vs_plain = []
    for i, img in plain_imgs:
        bc.set_views(sets[i])
        vs_plain.append(psnr_db(bc.render(out), img))
    key = f"{args.workload}/{storage}/composite/fixed"
    leg = {"ms_per_frame": ms, "render_ms": stage[1], "gsamples_per_s": gsps, "speedup_vs_f32": base_ms / ms,
           "traffic": measured_traffic(key), "l2_hit_rate": measured_traffic(key, "l2_hit_rate"),
           "psnr_vs_plain_f32_db": {"min": min(vs_plain), "mean": float(np.mean(vs_plain)),
                                    "frames": len(vs_plain)}}
    if ref is not None:
        pix, ref_img, branches = ref
        bc.set_views(sets[0])
        img = bc.render(out)[0].cpu().numpy().astype(np.float64)
        leg["vs_fp64_oracle_on_f32_cube"] = precision_report(img[pix[:, 1], pix[:, 0]], ref_img, branches)
    leg["chosen"] = bool(leg["psnr_vs_plain_f32_db"]["min"] >= 40.0)
    bc.close()
    log(f"{storage}: {leg}")
    return leg


def learned_leg(bc, args, sets, views, out, W, H, base_ms):
    """Learned frames on the FP32 context: the trained upsampler's quality on
    every orbit frame (untimed), then the timed orbit at the 40 dB gate."""
    quality = setup_learned(bc, args, views, out, W, H)
    ms, _ = timed_frames(bc, sets, out, args.steps, args.warmup)
    bc.set_learned(False)
    net = quality["psnr_network_vs_plain_db"]
    leg = {"ms_per_frame": ms, "speedup_vs_f32": base_ms / ms,
           "psnr_vs_plain_f32_db": net, "bilinear_psnr_vs_plain_f32_db": quality["psnr_bilinear_vs_plain_db"],
           "gain_over_bilinear_db": net["mean"] - quality["psnr_bilinear_vs_plain_db"]["mean"],
           "fell_back_frames": quality["fell_back_frames"], "frames": quality["frames"],
           "psnr_threshold_db": args.psnr_threshold, "chosen": bool(net["min"] >= 40.0),
           "weights": quality["weights"]}
    log(f"learned: {leg}")
    return leg


# ------------------------------------------------------------------ GPU
def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; --gpus must be 1 (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)
    recipe, brick, W, H, per_launch, src_dtype = WORKLOADS[args.workload]
    if args.op == "composite" and args.step_policy != "fixed":
        sys.exit("bench.py: the per-voxel step policy needs --op mip")
    if args.op == "mip" and args.learned:
        sys.exit("bench.py: learned frames are composited frames; drop --learned for --op mip")
    if per_launch > 1 and (args.learned or args.check_pixels or args.cpu_seconds):
        log("batched workload: learned mode, oracle check and CPU baseline are not run")
        args.learned, args.check_pixels, args.cpu_seconds = False, 0, 0
    if src_dtype == "f16" and args.storage == "f32":
        args.storage = "f16"
    forms = (args.forms and args.workload == "cube1024_persp1920x1080" and args.storage == "f32"
             and args.op == "composite" and not args.learned and not args.graph)
    t = time.perf_counter()
    vol = synth.make_cube(recipe, workers=min(16, os.cpu_count() or 1),
                          out_dtype=np.float16 if src_dtype == "f16" else np.float32)
    if vol.dtype == np.float16:
        # numpy reduces FP16 element by element; torch's threaded reduction
        # gives the same (exact) extremes in seconds on a 27 GB cube
        import torch
        tv = torch.from_numpy(vol)
        vmin, vmax = float(tv.min()), float(tv.max())
        del tv
    else:
        vmin, vmax = float(vol.min()), float(vol.max())
    log(f"cube {recipe.dims} generated in {time.perf_counter() - t:.1f} s; range [{vmin:.3f}, {vmax:.3f}]")
    rgba = synth.ramp_tf(vmin, vmax)
    # the small parity workload is orthographic, every other one perspective
    sets = view_sets(recipe, W, H, per_launch, args.frames, "ortho" if "_ortho" in args.workload else "persp")
    views = [vs[0] for vs in sets]
    nf = len(sets)

    workers = args.cpu_workers or host_cores()
    ref = None
    if args.check_pixels > 0:
        t = time.perf_counter()
        ref = oracle_reference(vol, recipe, brick, views[0], rgba, vmin, vmax, args.check_pixels, workers, args)
        log(f"oracle reference: {len(ref[0])} pixels of frame 0 in {time.perf_counter() - t:.1f} s")
    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(vol, recipe, brick, views[0], rgba, vmin, vmax, args.cpu_seconds, workers, args)
        log(f"cpu baseline: {cpu['value'] * 1e3:.4f} Msamples/s on {cpu['cores']} processes")

    import torch
    from paper_1205_0282_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    bc = binding.BrickCaster(0)
    bc.plan(recipe.dims, (brick,) * 3, storage=args.storage, src_dtype=src_dtype, max_views=per_launch,
            max_w=W, max_h=H)
    bc.bind()
    bc.set_option(binding.BC_OPT_XCD_QUEUES, args.xcd_queues)
    bc.set_option(binding.BC_OPT_TILE_WIDTH, args.tile_width)
    bc.set_operator(args.op, args.step_policy)
    t = time.perf_counter()
    src = torch.from_numpy(vol).to(dev)
    bc.load(src)
    torch.cuda.synchronize()
    del src
    if not forms:
        del vol
    torch.cuda.empty_cache()
    log(f"bricks loaded in {time.perf_counter() - t:.1f} s")
    bc.set_transfer_function(rgba, vmin, vmax)
    out = torch.empty((per_launch, H, W, 4), dtype=torch.float32, device=dev)

    # per orbit frame: samples and algorithmic bytes of the ray-casting launch (untimed)
    lohi, _, _ = bc.bricks()
    ebytes = {"f32": 4, "f16": 2, "fp8": 1}[args.storage]
    core_bytes = np.prod((lohi[:, 3:] - lohi[:, :3]).astype(np.int64), axis=1) * ebytes
    samples, evaluated, algo_bytes, tiles = [], [], [], []
    for vs in sets:
        bc.set_views(vs)
        bc.render(out)
        st = bc.stats()
        live = np.zeros(len(core_bytes), bool)
        for j in range(len(vs)):
            r = bc.rects(j)
            live |= (r[:, 2] > r[:, 0]) & (r[:, 3] > r[:, 1])
        samples.append(st["nominal_samples"])
        evaluated.append(st["evaluated_samples"])
        tiles.append(st["n_tiles"])
        # each voxel of a brick any view needs is read once per launch; on the
        # paper-shape workloads, whose frames take far fewer samples than
        # their bricks hold voxels, at most one voxel per sample
        vox_bytes = int(core_bytes[live].sum())
        if args.workload in SAMPLE_CAPPED:
            vox_bytes = min(vox_bytes, st["nominal_samples"] * ebytes)
        algo_bytes.append(vox_bytes + st["n_tiles"] * 64 * 16)
    log(f"orbit: mean {np.mean(samples) / 1e6:.1f} M samples/frame, {np.mean(tiles):.0f} tiles/frame")

    precision = None
    if ref is not None:
        pix, ref_img, branches = ref
        bc.set_views([views[0]])
        img = bc.render(out)[0].cpu().numpy().astype(np.float64)
        precision = precision_report(img[pix[:, 1], pix[:, 0]], ref_img, branches)
        log(f"precision vs FP64 oracle: {precision}")

    learned = None
    if args.learned:
        learned = setup_learned(bc, args, views, out, W, H)

    tuned = None
    if args.autotune:
        bc.set_views(sets[0])
        tuned = bc.autotune(out, frames=3)
        log(f"autotune: chunk {tuned[0]}, workgroups {tuned[1]}, tile width {tuned[2]}")
    stage_ms_eager = None
    if args.graph:
        # stage split from eager frames first (a graph is timed as a whole)
        bc.enable_timing(True)
        for i in range(min(args.steps, nf)):
            bc.set_views(sets[i % nf])
            bc.render(out)
        ms, k = bc.timing()
        stage_ms_eager = [m / k for m in ms]
        bc.enable_timing(False)
        bc.set_option(binding.BC_OPT_GRAPH, 1)

    for i in range(args.warmup):
        bc.set_views(sets[i % nf])
        bc.render(out)
    torch.cuda.synchronize()
    # the timed frames carry only the two HIP events around the ray-casting
    # kernel (events between every stage add a few microseconds per frame)
    bc.enable_timing(True, stages=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bc.set_views(sets[i % nf])
        bc.render(out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, n_timed = bc.timing()
    bc.enable_timing(False)
    assert n_timed == args.steps, (n_timed, args.steps)
    # set-up and compositing per frame, from the same frames re-rendered
    # untimed with an event between every stage
    bc.enable_timing(True)
    for i in range(args.steps):
        bc.set_views(sets[i % nf])
        bc.render(out)
    side_ms, n_side = bc.timing()
    bc.enable_timing(False)
    stage_ms = [side_ms[0] / n_side * n_timed, stage_ms[1], side_ms[2] / n_side * n_timed]

    # the paper's statistic (untimed by the contract above): median of 10
    # frames per orbit angle, 75th percentile over the angles
    paper_stat = None
    if args.repeats > 0:
        bc.enable_timing(True)
        for i in range(nf):
            bc.set_views(sets[i])
            for _ in range(args.repeats):
                bc.render(out)
        ft = np.asarray(bc.frame_times(), np.float64).reshape(nf, args.repeats)
        bc.enable_timing(False)
        med = np.median(ft, axis=1)
        paper_stat = {"median_of": args.repeats, "p75_over_angles_ms": float(np.percentile(med, 75)),
                      "mean_ms": float(ft.mean()), "angles": nf}

    ms_step = elapsed / args.steps * 1e3
    form_legs = None
    if forms:
        form_legs = {"f32": {"ms_per_frame": ms_step, "speedup_vs_f32": 1.0}}
        if os.path.exists(args.weights):
            form_legs["learned"] = learned_leg(bc, args, sets, views, out, W, H, ms_step)
        # plain FP32 frames the other forms are compared with
        picks = list(range(0, nf, max(1, nf // 8)))[:8]
        plain_imgs = []
        for i in picks:
            bc.set_views(sets[i])
            plain_imgs.append((i, bc.render(out).clone()))
        bc.close()
        torch.cuda.empty_cache()
        for st in ("f16", "fp8"):
            form_legs[st] = storage_leg(st, args, recipe, brick, W, H, sets, vol, rgba, vmin, vmax, ref,
                                        plain_imgs, ms_step)
            torch.cuda.empty_cache()
        del plain_imgs, vol

    idx = [i % nf for i in range(args.steps)]
    tot_samples = float(sum(samples[i] for i in idx))
    tot_bytes = float(sum(algo_bytes[i] for i in idx))
    if stage_ms_eager is not None:
        stage_ms = [m * n_timed for m in stage_ms_eager]
    render_s = stage_ms[1] / 1e3
    achieved = tot_bytes / render_s / 1e9
    key = f"{args.workload}/{args.storage}/{args.op}/{args.step_policy}"
    traffic, l2_hit = measured_traffic(key), measured_traffic(key, "l2_hit_rate")
    result = {
        "metric": (f"Gsamples/s + fps @{W}x{H} on "
                   + ("1024^3 cube" if recipe.dims == (1024, 1024, 1024) else "x".join(map(str, recipe.dims)) + " cube")
                   + ("; learned/FP8 vs plain at PSNR>=40dB" if forms else ""))
                  if per_launch == 1 else
                  f"Gsamples/s + launches/s @{W}x{H}, {per_launch} views per launch, "
                  + "x".join(map(str, recipe.dims)) + " FP16 cube",
        "value": tot_samples / elapsed / 1e9,   # learned frames: nominal samples of the plain frame (equivalent)
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "fps": 1e3 / ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16 storage, f32 arithmetic",
                  "fp8": "fp8-e4m3 storage, f32 arithmetic"}[args.storage],
        "data": "synthetic",
        "config": {"workload": args.workload, "cube": list(recipe.dims), "brick": brick,
                   "image": [W, H], "operator": args.op,
                   "step_vox": "per-voxel" if args.step_policy == "voxel" else 0.5,
                   "ert": 0.99 if args.op == "composite" else "brick maximum", "storage": args.storage,
                   "orbit_frames": nf * per_launch, "views_per_launch": per_launch,
                   "graph": bool(args.graph), "autotuned": tuned, "xcd_queues": args.xcd_queues,
                   "tile": [tuned[2] if tuned else args.tile_width, 64 // (tuned[2] if tuned else args.tile_width)]},
        "stage_ms_per_frame": {"setup": stage_ms[0] / n_timed, "render": stage_ms[1] / n_timed,
                               "composite": stage_ms[2] / n_timed},
        "samples_per_frame": tot_samples / args.steps,
        "evaluated_per_frame": float(sum(evaluated[i] for i in idx)) / args.steps,
        # (a learned frame's stage times split coarse pass / network / rest,
        # so its ray-casting kernel is not timed on its own: no roofline)
        "roofline": None if args.learned else {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "render_kernel", "algo_bytes_per_launch": tot_bytes / args.steps,
            # HBM bytes actually moved (counters), as a bandwidth and a fraction of peak
            "traffic_gbs": None if traffic is None else traffic / (render_s / args.steps) / 1e9,
            "traffic_frac": None if traffic is None else traffic / (render_s / args.steps) / 1e9 / HBM_PEAK_GBS,
            "l2_hit_rate": l2_hit},
        "paper_statistic": paper_stat,
        "precision_vs_oracle": precision,
        "learned": learned,
        "forms": form_legs,
        "cpu_baseline": cpu,
    }
    if not forms:
        bc.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
