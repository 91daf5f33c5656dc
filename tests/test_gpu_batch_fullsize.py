"""Parity of the batching workload at its full size: the 3000 x 3000 x 1500
cube (noise + 5000 sources, about 27 GB) from an FP16 source, stored FP16 in
256^3 bricks with uneven edge bricks (12 x 12 x 6 of them), four orbit views
90 degrees apart rendered by one launch at 1920x1080 (the launch configuration
bench.py times for this workload, eager and replayed as a captured graph),
against the FP64 oracle at sampled pixels of every view.

FP16 storage of an FP16 source is an exact copy, so the oracle stores the host
FP16 cube as it is: each gathered value converts exactly to FP64, and no FP32
or FP64 copy of the cube is made.  The sampled pixels of each view are a block of
neighbours (rays that share bricks and cells), pixels scattered over the
image, and pixels whose rays miss the cube."""
import time

import numpy as np
import pytest

from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

from gpu_util import TOL, cam_of, compare

pytestmark = pytest.mark.gpu

W, H, BRICK, PER_LAUNCH, ORBIT = 1920, 1080, 256, 4, 64


@pytest.fixture(scope="module")
def batch_cube(request):
    import torch
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(m):   # progress lines, shown while the cube is generated
        if capman is None:
            print(m, flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(m, flush=True)

    recipe = synth.RECIPE_BATCH
    t = time.perf_counter()
    last = [0.0]

    def progress(done, total):
        if time.perf_counter() - last[0] > 20.0 or done == total:
            last[0] = time.perf_counter()
            say(f"  batch cube: {done}/{total} generation blocks, {last[0] - t:.0f} s")

    vol = synth.make_cube(recipe, out_dtype=np.float16, workers=16, progress=progress)
    dims = recipe.dims
    bc = binding.BrickCaster(0)
    bc.plan(dims, (BRICK,) * 3, storage="f16", src_dtype="f16", max_views=PER_LAUNCH, max_w=W, max_h=H)
    bc.bind()
    bc.set_option(binding.BC_OPT_XCD_QUEUES, 1)
    src = torch.from_numpy(vol).cuda()
    bc.load(src)
    # the cube's range (exact FP16 values), as the host reduction would give it
    vmin, vmax = float(src.min()), float(src.max())
    rgba = synth.ramp_tf(vmin, vmax)
    torch.cuda.synchronize()
    del src
    torch.cuda.empty_cache()
    bc.set_transfer_function(rgba, vmin, vmax)
    say(f"  batch cube: generated and loaded in {time.perf_counter() - t:.0f} s")
    # FP16 storage of an FP16 source holds exactly the source's values: the
    # oracle stores the source as it is, shared by every brick
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (BRICK,) * 3))
    assert stored[0].values is vol
    tf = rc.TransferFunction(rgba, vmin, vmax)
    yield dict(bc=bc, stored=stored, tf=tf, dims=dims, say=say)
    bc.close()


def _views(first):
    """Launch ``first`` of the orbit: frames first, first + 16, first + 32, first + 48."""
    stride = ORBIT // PER_LAUNCH
    return [synth.orbit_view(synth.RECIPE_BATCH.dims, first + j * stride, ORBIT, kind="persp",
                             width=W, height=H, step=0.5, ert=0.99) for j in range(PER_LAUNCH)]


def _pixels(cam, dims, seed):
    """24 pixels in a 24 x 24 window and 40 scattered pixels whose rays hit the
    cube, and up to 4 pixels whose rays miss it: (hit pixels, missing pixels)."""
    rng = np.random.default_rng(seed)
    for _ in range(100):
        x0, y0 = int(rng.integers(W // 5, 4 * W // 5 - 24)), int(rng.integers(H // 5, 4 * H // 5 - 24))
        cand = np.stack([x0 + rng.integers(0, 24, 200), y0 + rng.integers(0, 24, 200)], axis=1)
        cand = np.unique(cand, axis=0)
        o, d = cam.rays(cand[:, 0], cand[:, 1])
        _, _, hit = rc.global_interval(o, d, dims)
        if hit.sum() >= 24:
            break
    far = np.stack([rng.integers(0, W, 400), rng.integers(0, H, 400)], axis=1)
    o, d = cam.rays(far[:, 0], far[:, 1])
    _, _, fhit = rc.global_interval(o, d, dims)
    return np.concatenate([cand[hit][:24], far[fhit][:40]]), far[~fhit][:4]


def test_four_view_launch_matches_oracle_at_sampled_pixels(batch_cube):
    import torch
    bc, stored, tf, dims, say = (batch_cube[k] for k in ("bc", "stored", "tf", "dims", "say"))
    views = _views(0)
    bc.set_views(views)
    out = torch.empty((PER_LAUNCH, H, W, 4), dtype=torch.float32, device="cuda")
    bc.render(out)
    img = out.cpu().numpy().astype(np.float64)
    for j, v in enumerate(views):
        cam = cam_of(v)
        hits, misses = _pixels(cam, dims, 300 + j)
        assert len(hits) >= 48
        pix = np.concatenate([hits, misses])
        t = time.perf_counter()
        res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.99, pixels=pix)
        err, _, _ = compare(img[j, pix[:, 1], pix[:, 0]], res, f"  view {j} (orbit frame {j * ORBIT // PER_LAUNCH})")
        say(f"  view {j}: oracle {time.perf_counter() - t:.0f} s")
        assert err <= TOL
        assert res.image[:, 3].max() > 0.1
        assert np.all(img[j, misses[:, 1], misses[:, 0]] == 0.0)   # rays that miss stay clear


def test_four_view_graph_replay_equals_eager_launch(batch_cube):
    import torch
    bc = batch_cube["bc"]
    views = _views(5)
    bc.set_views(views)
    eager = torch.empty((PER_LAUNCH, H, W, 4), dtype=torch.float32, device="cuda")
    bc.render(eager)
    torch.cuda.synchronize()
    # one output buffer, so the graph is captured once and then replayed
    out = torch.empty_like(eager)
    bc.set_option(binding.BC_OPT_GRAPH, 1)
    try:
        for _ in range(3):
            out.fill_(-1.0)
            bc.render(out)
            torch.cuda.synchronize()
            assert torch.equal(out, eager)
    finally:
        bc.set_option(binding.BC_OPT_GRAPH, 0)
    assert float(eager[..., 3].max()) > 0.1
