"""Trains the learned upsampler on image pairs the ray caster itself renders,
on the GPU, with the library's own forward, backward and Adam kernels.

Each pair is one view of a seeded synthetic cube rendered twice by the plain
ray caster: the coarse input at half the width and height with a 2-voxel step,
and the full-resolution target with the 0.5-voxel step.  Cubes follow the
1024^3 benchmark cube's recipe (same size, source count and widths) with other
seeds, so the network sees the voxel-to-pixel scale it will be used at; views
are random azimuths and elevations on the benchmark's orbit distance.  One
cube is held out for validation: the PSNR of the network's output and of the
plain bilinear upsampling, both against the full render, is reported.

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
        torch = self.torch
        vol = synth.make_cube(recipe, workers=workers)
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
    p.add_argument("--views-per-cube", type=int, default=100)
    p.add_argument("--width", type=int, default=1920)
    p.add_argument("--height", type=int, default=1080)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--val-views", type=int, default=8)
    p.add_argument("--cube", type=int, default=1024, help="cube edge of the training cubes")
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

    # held-out validation views (seed 999)
    t0 = time.perf_counter()
    maker.load(recipe(999), workers)
    vrng = np.random.default_rng(a.seed + 12345)
    val = [tuple(t.clone() for t in maker.pair(vrng)) for _ in range(a.val_views)]

    def evaluate():
        ps, pb = [], []
        for c, f in val:
            up = trainer.cnn_forward(c)
            ps.append(psnr(up, f))
            pb.append(psnr(bilinear2(c), f))
        torch.cuda.synchronize()
        return float(np.mean(ps)), float(np.mean(pb))

    psnr0, psnr_bil = evaluate()
    log(f"validation before training: network {psnr0:.2f} dB, bilinear {psnr_bil:.2f} dB "
        f"({time.perf_counter() - t0:.1f} s)")
    rng = np.random.default_rng(a.seed)
    losses = []
    n_cubes = (a.pairs + a.views_per_cube - 1) // a.views_per_cube
    step = 0
    t_train = time.perf_counter()
    for ci in range(n_cubes):
        maker.load(recipe(1000 + ci), workers)
        for _ in range(min(a.views_per_cube, a.pairs - step)):
            c, f = maker.pair(rng)
            lr = a.lr * 0.5 * (1.0 + math.cos(math.pi * step / a.pairs))
            want = step % 50 == 0
            loss = trainer.cnn_train_step(c, f, lr=lr, want_loss=want)
            if want:
                losses.append((step, loss))
                log(f"step {step}: loss {loss:.3e} lr {lr:.2e}")
            step += 1
        log(f"cube {ci + 1}/{n_cubes} done, {step} pairs, {time.perf_counter() - t_train:.1f} s")
    w, m, v, st = trainer.cnn_get_weights()
    psnr1, _ = evaluate()
    log(f"validation after training: network {psnr1:.2f} dB, bilinear {psnr_bil:.2f} dB")
    np.save(a.out, w, allow_pickle=False)
    summary = {"pairs": step, "cubes": n_cubes, "cube_edge": a.cube, "sources": n_src,
               "frame": [a.width, a.height], "coarse_step": 2.0, "fine_step": 0.5, "lr": a.lr,
               "schedule": "cosine", "adam_steps": st, "val_cube_seed": 999, "train_cube_seeds": f"1000..{999 + n_cubes}",
               "val_psnr_db": {"network_before": psnr0, "network_after": psnr1, "bilinear": psnr_bil},
               "loss_curve": losses, "seconds": time.perf_counter() - t0}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(summary, fh, indent=1)
    log(json.dumps(summary["val_psnr_db"]))
    trainer.close()
    maker.close()


if __name__ == "__main__":
    main()
