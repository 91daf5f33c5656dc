"""Parity at the benchmark's full size: the 1024^3 FP32 cube (4x4x4 bricks of
256^3), perspective 1920x1080, rendered by the same launch configuration
bench.py times, against the FP64 oracle at sampled pixels (each computed one
by one by the oracle): compositing with step 0.5 and termination at 0.99, and
maximum intensity projection with the per-voxel step; and the same cube stored
FP16 and FP8 (the precision workload) against the oracle on the stored
values."""
import numpy as np
import pytest

from oracle import mip
from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

from gpu_util import TOL, cam_of, compare, compare_mip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube1024():
    import torch
    recipe = synth.RECIPE_1024
    vol = synth.make_cube(recipe, workers=16)
    vmin, vmax = float(vol.min()), float(vol.max())
    rgba = synth.ramp_tf(vmin, vmax)
    dims = recipe.dims
    bc = binding.BrickCaster(0)
    bc.plan(dims, (256, 256, 256), storage="f32", max_views=1, max_w=1920, max_h=1080)
    bc.bind()
    src = torch.from_numpy(vol).cuda()
    bc.load(src)
    del src
    bc.set_transfer_function(rgba, vmin, vmax)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (256, 256, 256)))
    tf = rc.TransferFunction(rgba, vmin, vmax)
    yield dict(bc=bc, stored=stored, tf=tf, dims=dims, vol=vol, rgba=rgba, vmin=vmin, vmax=vmax)
    bc.close()


def _pixels(cam, dims, seed):
    rng = np.random.default_rng(seed)
    cand = np.stack([rng.integers(0, 1920, 2000), rng.integers(0, 1080, 2000)], axis=1)
    o, d = cam.rays(cand[:, 0], cand[:, 1])
    _, _, hit = rc.global_interval(o, d, dims)
    return np.concatenate([cand[hit][:96], cand[~hit][:16]])


def test_cube1024_frame_sampled_pixels(cube1024):
    bc, stored, tf, dims = cube1024["bc"], cube1024["stored"], cube1024["tf"], cube1024["dims"]
    bc.set_operator("composite", "fixed")
    for frame in (0, 23):
        v = synth.orbit_view(dims, frame)
        bc.set_views([v])
        img = bc.render()[0].cpu().numpy().astype(np.float64)
        cam = cam_of(v)
        pix = _pixels(cam, dims, 100 + frame)
        res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.99, pixels=pix)
        err, _, _ = compare(img[pix[:, 1], pix[:, 0]], res, f"frame {frame}")
        assert err <= TOL
        assert res.image[:, 3].max() > 0.1


def test_cube1024_mip_per_voxel_sampled_pixels(cube1024):
    bc, stored, tf, dims = cube1024["bc"], cube1024["stored"], cube1024["tf"], cube1024["dims"]
    bc.set_operator("mip", "voxel")
    try:
        for frame in (5, 40):
            v = synth.orbit_view(dims, frame)
            bc.set_views([v])
            img = bc.render()[0].cpu().numpy().astype(np.float64)
            cam = cam_of(v)
            pix = _pixels(cam, dims, 200 + frame)
            res = mip.render_mip_bricked(stored, dims, cam, tf, "voxel", pixels=pix)
            assert compare_mip(img[pix[:, 1], pix[:, 0]], res, f"mip frame {frame}") <= TOL
            assert np.unique(res.image[res.samples > 0, 0]).size > 20
    finally:
        bc.set_operator("composite", "fixed")


def _window(cam, dims, seed, n=32, side=24):
    """``n`` pixels of one ``side`` x ``side`` block whose rays hit the cube
    (rays that share bricks), and up to 4 pixels whose rays miss it."""
    rng = np.random.default_rng(seed)
    for _ in range(100):
        x0, y0 = int(rng.integers(1920 // 5, 4 * 1920 // 5 - side)), int(rng.integers(1080 // 5, 4 * 1080 // 5 - side))
        cand = np.unique(np.stack([x0 + rng.integers(0, side, 200), y0 + rng.integers(0, side, 200)], axis=1), axis=0)
        o, d = cam.rays(cand[:, 0], cand[:, 1])
        _, _, hit = rc.global_interval(o, d, dims)
        if hit.sum() >= n:
            break
    far = np.stack([rng.integers(0, 1920, 400), rng.integers(0, 1080, 400)], axis=1)
    o, d = cam.rays(far[:, 0], far[:, 1])
    _, _, fhit = rc.global_interval(o, d, dims)
    return cand[hit][:n], far[~fhit][:4]


@pytest.mark.parametrize("storage", ["f16", "fp8"])
def test_cube1024_stored_forms_sampled_pixels(cube1024, storage):
    """The benchmark frame with FP16 or FP8 storage, rendered in the launch
    configuration bench.py times, against the oracle on the values each brick
    stores; the oracle encodes only the bricks that the checked rays cross."""
    import torch
    vol, dims, tf = cube1024["vol"], cube1024["dims"], cube1024["tf"]
    bc = binding.BrickCaster(0)
    try:
        bc.plan(dims, (256, 256, 256), storage=storage, max_views=1, max_w=1920, max_h=1080)
        bc.bind()
        src = torch.from_numpy(vol).cuda()
        bc.load(src)
        torch.cuda.synchronize()
        del src
        bc.set_transfer_function(cube1024["rgba"], cube1024["vmin"], cube1024["vmax"])
        v = synth.orbit_view(dims, 11)
        bc.set_views([v])
        img = bc.render()[0].cpu().numpy().astype(np.float64)
    finally:
        bc.close()
    cam = cam_of(v)
    hits, misses = _window(cam, dims, 400 + len(storage))
    assert len(hits) >= 24
    pix = np.concatenate([hits, misses])
    bricks = rc.brick_grid(dims, (256, 256, 256))
    o, d = cam.rays(pix[:, 0], pix[:, 1])
    crossed = set()
    for b in bricks:
        tb0, tb1 = rc.slab(o, d, tuple(float(x) for x in b.lo), tuple(float(x) for x in b.hi))
        if np.any(tb0 < tb1):
            crossed.add(b.index)
    stored = rc.store_bricks(vol, bricks, storage, only=crossed)
    res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.99, pixels=pix)
    err, _, _ = compare(img[pix[:, 1], pix[:, 0]], res, f"{storage}, {len(crossed)} of {len(bricks)} bricks encoded")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.1
    assert np.all(img[misses[:, 1], misses[:, 0]] == 0.0)
