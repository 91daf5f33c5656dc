"""Trains the learned upsampler on image pairs the ray caster itself renders,
on the GPU, with the library's own forward, backward and Adam kernels.

Each pair is one view of a seeded synthetic cube rendered twice by the plain
ray caster: the coarse input at half the width and height with a 2-voxel step,
and the full-resolution target with the 0.5-voxel step.  Cubes follow the
1024^3 benchmark cube's recipe (source widths and peaks) at a chosen edge,
with the source count scaled by volume so that the fraction of voxels above
3 stays at 5%: by default one view of each of 2000 cubes of 256^3 (seeds 1000
to 2999); ``--cube 1024 --views-per-cube 100`` trains on 20 cubes at the
bench cube's own voxel-to-pixel scale.  Views are random azimuths and
elevations at the benchmark's orbit distance.  Cubes of other seeds are held
out for validation; every ``--curve-every`` steps the network's PSNR against
the full render is taken on the validation pairs and on a reservoir of
training pairs (its fit to the data it sees), beside the bilinear upsampling
of the same coarse renders.  At the end the network is measured on orbit
frames of the 1024^3 bench cube, the frames learned frames are judged on.
``--overfit N`` instead trains N steps on one pair: the PSNR it reaches there
bounds what the network can represent.

    python -m paper_1205_0282_amd.train_upsampler --pairs 2000 --out weights.npy

Writes the FP32 parameters (numpy .npy, no pickle) and a JSON summary beside
them.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_1205_0282_amd import binding, synth  # noqa: E402

N_PARAMS = binding.CNN_N_PARAMS
LAYERS = ((4, 32), (32, 32), (32, 16))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases; the last layer scaled by 0.1 so that
    training starts near the bilinear upsampling."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(LAYERS):
        w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        if k == len(LAYERS) - 1:
            w *= 0.1
        parts += [w.reshape(-1), np.zeros(co)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == N_PARAMS
    return p


def log(*a):
    print(*a, flush=True)


class PairMaker:
    """Renders (coarse, fine) pairs of random views of one loaded cube."""

    def __init__(self, width, height, brick=256):
        import torch
        self.W, self.H = width, height
        self.brick = brick
        self.fine = binding.BrickCaster(0)
        self.coarse = binding.BrickCaster(0)
        self.torch = torch
        self.dims = None

    def load(self, recipe, workers):
        self.load_volume(recipe, synth.make_cube(recipe, workers=workers))

    def load_volume(self, recipe, vol):
        torch = self.torch
        vmin, vmax = float(vol.min()), float(vol.max())
        rgba = synth.ramp_tf(vmin, vmax)
        if self.dims != recipe.dims:
            for bc, (w, h) in ((self.fine, (self.W, self.H)), (self.coarse, (self.W // 2, self.H // 2))):
                bc.close()
            self.fine = binding.BrickCaster(0)
            self.coarse = binding.BrickCaster(0)
            for bc, (w, h) in ((self.fine, (self.W, self.H)), (self.coarse, (self.W // 2, self.H // 2))):
                bc.plan(recipe.dims, (self.brick,) * 3, max_views=1, max_w=w, max_h=h)
                bc.bind()
            self.dims = recipe.dims
        src = torch.from_numpy(vol).cuda()
        for bc in (self.fine, self.coarse):
            bc.load(src)
            bc.set_transfer_function(rgba, vmin, vmax)
        del src, vol

    def pair(self, rng):
        az = float(rng.uniform(0.0, 360.0))
        el = float(rng.uniform(-60.0, 60.0))
        fv = synth.orbit_view(self.dims, 0, width=self.W, height=self.H, elevation_deg=el,
                              azimuth_offset_deg=az, step=0.5)
        cv = synth.orbit_view(self.dims, 0, width=self.W // 2, height=self.H // 2, elevation_deg=el,
                              azimuth_offset_deg=az, step=2.0)
        self.fine.set_views([fv])
        self.coarse.set_views([cv])
        return self.coarse.render(), self.fine.render()

    def close(self):
        self.fine.close()
        self.coarse.close()


def psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def bilinear2(x):
    """Bilinear x2 (half-pixel centres, clamped) of an (n, h, w, 4) tensor, for
    the baseline only."""
    import torch.nn.functional as F
    y = F.interpolate(x.permute(0, 3, 1, 2), scale_factor=2, mode="bilinear", align_corners=False)
    return y.permute(0, 2, 3, 1).contiguous()


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--pairs", type=int, default=2000)
    p.add_argument("--views-per-cube", type=int, default=1)
    p.add_argument("--width", type=int, default=1920)
    p.add_argument("--height", type=int, default=1080)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--val-views", type=int, default=8)
    p.add_argument("--val-seeds", default="998,999", help="held-out cube seeds")
    p.add_argument("--cube", type=int, default=256, help="cube edge of the training and validation cubes")
    p.add_argument("--curve-every", type=int, default=100)
    p.add_argument("--reservoir", type=int, default=8, help="training pairs kept for the training-set PSNR")
    p.add_argument("--bench-frames", type=int, default=8, help="bench-cube orbit frames measured at the end (0: none)")
    p.add_argument("--overfit", type=int, default=0, help="train this many steps on one pair instead")
    p.add_argument("--init", default="", help="start from these parameters (.npy) instead of a fresh init")
    p.add_argument("--out", required=True)
    a = p.parse_args()
    import torch
    workers = min(16, os.cpu_count() or 1)
    base = synth.RECIPE_1024
    scale = a.cube / 1024.0
    n_src = max(1, int(round(base.n_sources * scale ** 3)))

    def recipe(seed):
        return dataclasses.replace(base, dims=(a.cube,) * 3, seed=seed, n_sources=n_src)

    maker = PairMaker(a.width, a.height)
    trainer = binding.BrickCaster(0)
    trainer.cnn_setup(1, a.height // 2, a.width // 2)
    params = np.load(a.init, allow_pickle=False).astype(np.float32) if a.init else init_params(a.seed)
    trainer.cnn_set_weights(params)
    t0 = time.perf_counter()

    def measure(pairs):
        ps, pb = [], []
        for c, f in pairs:
            up = trainer.cnn_forward(c)
            ps.append(psnr(up, f))
            pb.append(psnr(bilinear2(c), f))
        torch.cuda.synchronize()
        return float(np.mean(ps)), float(np.mean(pb))

    rng = np.random.default_rng(a.seed)
    if a.overfit:
        maker.load(recipe(1000), workers)
        pair = [tuple(t.clone() for t in maker.pair(rng))]
        curve = []
        for step in range(a.overfit):
            lr = a.lr * 0.5 * (1.0 + math.cos(math.pi * step / a.overfit))
            trainer.cnn_train_step(pair[0][0], pair[0][1], lr=lr, want_loss=False)
            if step % a.curve_every == 0 or step == a.overfit - 1:
                net, bil = measure(pair)
                curve.append((step, net))
                log(f"overfit step {step}: network {net:.2f} dB, bilinear {bil:.2f} dB")
        summary = {"overfit_steps": a.overfit, "cube_edge": a.cube, "sources": n_src, "frame": [a.width, a.height],
                   "psnr_curve_db": curve, "bilinear_db": bil, "seconds": time.perf_counter() - t0}
        with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
            json.dump(summary, fh, indent=1)
        trainer.close()
        maker.close()
        return

    # held-out validation views
    vrng = np.random.default_rng(a.seed + 12345)
    val = []
    seeds = [int(x) for x in a.val_seeds.split(",") if x]
    for vs in seeds:
        maker.load(recipe(vs), workers)
        val += [tuple(t.clone() for t in maker.pair(vrng)) for _ in range(max(1, a.val_views // len(seeds)))]
    psnr0, psnr_bil = measure(val)
    log(f"validation before training: network {psnr0:.2f} dB, bilinear {psnr_bil:.2f} dB "
        f"({time.perf_counter() - t0:.1f} s)")
    n_cubes = (a.pairs + a.views_per_cube - 1) // a.views_per_cube
    # cubes are generated ahead on host threads while the GPU renders and trains
    import concurrent.futures as cf
    pool = cf.ThreadPoolExecutor(max_workers=min(8, workers))
    ahead = 8 if a.cube <= 256 else 1
    gen_workers = 1 if a.cube <= 256 else workers
    futs = {ci: pool.submit(synth.make_cube, recipe(1000 + ci), np.float32, gen_workers)
            for ci in range(min(ahead, n_cubes))}
    losses, curve, reservoir = [], [], []
    step = 0
    t_train = time.perf_counter()
    for ci in range(n_cubes):
        vol = futs.pop(ci).result()
        if ci + ahead < n_cubes:
            futs[ci + ahead] = pool.submit(synth.make_cube, recipe(1000 + ci + ahead), np.float32, gen_workers)
        maker.load_volume(recipe(1000 + ci), vol)
        del vol
        for _ in range(min(a.views_per_cube, a.pairs - step)):
            c, f = maker.pair(rng)
            # reservoir sample of the training pairs, for the fit on seen data
            if len(reservoir) < a.reservoir:
                reservoir.append((c.clone(), f.clone()))
            else:
                k = int(rng.integers(0, step + 1))
                if k < a.reservoir:
                    reservoir[k] = (c.clone(), f.clone())
            lr = a.lr * 0.5 * (1.0 + math.cos(math.pi * step / a.pairs))
            want = step % 50 == 0
            loss = trainer.cnn_train_step(c, f, lr=lr, want_loss=want)
            if want:
                losses.append((step, loss))
            if step % a.curve_every == 0:
                vn, _ = measure(val)
                tn, tb = measure(reservoir)
                curve.append((step, vn, tn))
                log(f"step {step}: loss {loss:.3e} lr {lr:.2e}; validation {vn:.2f} dB, "
                    f"training pairs {tn:.2f} dB (bilinear {tb:.2f}); {time.perf_counter() - t_train:.0f} s")
            step += 1
    pool.shutdown()
    w, m, v, st = trainer.cnn_get_weights()
    psnr1, _ = measure(val)
    train1, train_bil = measure(reservoir)
    curve.append((step, psnr1, train1))
    log(f"validation after training: network {psnr1:.2f} dB, bilinear {psnr_bil:.2f} dB; "
        f"training pairs {train1:.2f} dB (bilinear {train_bil:.2f})")
    bench = None
    if a.bench_frames > 0:
        # the bench cube (seed 2, 1024^3) and its orbit: coarse 960x540 at step 2
        # against the full 1920x1080 render at step 0.5
        maker.load(synth.RECIPE_1024, workers)
        bp = []
        for k in range(a.bench_frames):
            fv = synth.orbit_view(maker.dims, k * 64 // a.bench_frames, width=a.width, height=a.height, step=0.5)
            cv = synth.orbit_view(maker.dims, k * 64 // a.bench_frames, width=a.width // 2, height=a.height // 2,
                                  step=2.0)
            maker.fine.set_views([fv])
            maker.coarse.set_views([cv])
            bp.append((maker.coarse.render().clone(), maker.fine.render().clone()))
        bn, bb = measure(bp)
        bench = {"frames": a.bench_frames, "network_db": bn, "bilinear_db": bb}
        log(f"bench cube orbit: network {bn:.2f} dB, bilinear {bb:.2f} dB")
    np.save(a.out, w, allow_pickle=False)
    summary = {"pairs": step, "cubes": n_cubes, "cube_edge": a.cube, "sources": n_src,
               "frame": [a.width, a.height], "coarse_step": 2.0, "fine_step": 0.5, "lr": a.lr,
               "schedule": "cosine", "adam_steps": st, "val_cube_seeds": seeds,
               "train_cube_seeds": f"1000..{999 + n_cubes}",
               "val_psnr_db": {"network_before": psnr0, "network_after": psnr1, "bilinear": psnr_bil},
               "train_psnr_db": {"network_after": train1, "bilinear": train_bil},
               "bench_cube_psnr_db": bench,
               "psnr_curve_db": {"columns": ["step", "validation", "training pairs"], "rows": curve},
               "loss_curve": losses, "seconds": time.perf_counter() - t0}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(summary, fh, indent=1)
    log(json.dumps({k: summary[k] for k in ("val_psnr_db", "train_psnr_db", "bench_cube_psnr_db")}))
    trainer.close()
    maker.close()


if __name__ == "__main__":
    main()
