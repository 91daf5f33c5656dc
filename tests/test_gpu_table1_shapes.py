"""Parity on one of the paper's cube shapes at its real size (Table 1: the
HIPASS cube, 1721 x 1721 x 1025 voxels, FP32, 12 GB), split into 256^3 bricks
(7 x 7 x 5, with 185-voxel edge bricks along x and y and a 1-voxel-thick edge
brick along z), rendered perspective at 1024x1024 (the paper's frame size) in
the launch configuration bench.py times, against the FP64 oracle at blocks of
pixels.  The cube is a seeded synthetic stand-in with the bench cube's source
density (the survey data are not available).  The oracle stores only the
bricks the checked rays cross."""
import numpy as np
import pytest

from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

from gpu_util import TOL, cam_of, compare

pytestmark = pytest.mark.gpu

SIZE = 1024
BRICK = (256, 256, 256)


@pytest.fixture(scope="module")
def hipass():
    import time

    import torch
    recipe = synth.RECIPE_HIPASS
    t = time.perf_counter()
    vol = synth.make_cube(recipe, workers=16)
    vmin, vmax = float(vol.min()), float(vol.max())
    print(f"hipass cube {recipe.dims} generated in {time.perf_counter() - t:.0f} s", flush=True)
    rgba = synth.ramp_tf(vmin, vmax)
    dims = recipe.dims
    bc = binding.BrickCaster(0)
    bc.plan(dims, BRICK, storage="f32", max_views=1, max_w=SIZE, max_h=SIZE)
    bc.bind()
    src = torch.from_numpy(vol).cuda()
    bc.load(src)
    torch.cuda.synchronize()
    del src
    torch.cuda.empty_cache()
    bc.set_transfer_function(rgba, vmin, vmax)
    print(f"hipass cube loaded, {time.perf_counter() - t:.0f} s", flush=True)
    yield dict(bc=bc, vol=vol, dims=dims, tf=rc.TransferFunction(rgba, vmin, vmax))
    bc.close()


def _block(cam, dims, x0, y0, side=16):
    """The pixels of a side x side block, split into rays that hit the cube and
    rays that miss it."""
    pix = np.stack(np.meshgrid(np.arange(x0, x0 + side), np.arange(y0, y0 + side)), -1).reshape(-1, 2)
    o, d = cam.rays(pix[:, 0], pix[:, 1])
    _, _, hit = rc.global_interval(o, d, dims)
    return pix, hit


@pytest.mark.parametrize("frame", [0, 37])
def test_hipass_shape_frame_blocks(hipass, frame):
    """Frame 0 looks at the cube's +z face (every ray enters through the
    1-voxel brick), frame 37 from behind (the rays leave through it).  Two
    16x16 blocks: one at the frame centre, one across the silhouette edge on
    the middle row."""
    bc, vol, dims, tf = hipass["bc"], hipass["vol"], hipass["dims"], hipass["tf"]
    v = synth.orbit_view(dims, frame, kind="persp", width=SIZE, height=SIZE)
    bc.set_views([v])
    img = bc.render()[0].cpu().numpy().astype(np.float64)
    cam = cam_of(v)
    o, d = cam.rays(np.arange(SIZE), np.full(SIZE, SIZE // 2))
    _, _, row_hit = rc.global_interval(o, d, dims)
    x_edge = int(np.argmax(row_hit))
    centre, chit = _block(cam, dims, SIZE // 2 - 8, SIZE // 2 - 8)
    edge, ehit = _block(cam, dims, max(x_edge - 8, 0), SIZE // 2 - 8)
    assert chit.all() and 0 < ehit.sum() < len(ehit)
    pix = np.concatenate([centre, edge])
    bricks = rc.brick_grid(dims, BRICK)
    o, d = cam.rays(pix[:, 0], pix[:, 1])
    crossed = set()
    for b in bricks:
        tb0, tb1 = rc.slab(o, d, tuple(float(x) for x in b.lo), tuple(float(x) for x in b.hi))
        if np.any(tb0 < tb1):
            crossed.add(b.index)
    thin = {b.index for b in bricks if b.hi[2] - b.lo[2] == 1}
    assert crossed & thin                                  # the 1-voxel bricks are on the checked rays
    stored = rc.store_bricks(vol, bricks, only=crossed)
    res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.99, pixels=pix)
    err, _, _ = compare(img[pix[:, 1], pix[:, 0]], res,
                        f"hipass frame {frame}: {len(pix)} pixels, {len(crossed)} of {len(bricks)} bricks crossed")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.1
    miss = pix[~np.concatenate([chit, ehit])]
    assert np.all(img[miss[:, 1], miss[:, 0]] == 0.0)
