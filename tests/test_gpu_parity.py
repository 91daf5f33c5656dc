"""Parity of the HIP ray caster (through the C ABI) with the FP64 oracle on
the same seeded inputs.  Images: max |GPU - oracle| <= 2e-5 per RGBA channel
(near-tie rays may match any of their branches); brick order, brick table and
encoded bricks bit-exact; rendering rectangles cover every pixel whose ray has
a sample in the brick."""
import numpy as np
import pytest

from oracle import encoders
from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

from gpu_util import TOL, cam_of, compare, compare_mip, gpu_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_cube():
    return synth.make_cube(synth.RECIPE_SMALL, workers=4)


def _ramp(vol):
    vmin, vmax = float(vol.min()), float(vol.max())
    return synth.ramp_tf(vmin, vmax), vmin, vmax


@pytest.mark.parametrize("tau", [1.0, 0.99])
def test_small_plain_full_frame(small_cube, tau):
    """128^3 cube, 2x2x2 bricks of 64^3, orthographic 256x256, step 0.5."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(vol.shape[::-1], 7, kind="ortho", width=256, height=256, ert=tau)
    img, bc = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, keep=True)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    stored = rc.store_bricks(vol, rc.brick_grid(vol.shape[::-1], (64, 64, 64)))
    res = rc.render_bricked(stored, vol.shape[::-1], cam_of(v), tf, 0.5, tau)
    err, n_tie, n_ovf = compare(img[0].reshape(-1, 4), res, f"128^3 tau {tau}")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.5           # the frame is not trivially empty
    assert np.array_equal(bc.visibility_order(0), np.asarray(res.order, np.int32))
    rects = bc.rects(0)
    py, px = np.divmod(np.arange(256 * 256), 256)
    for b, fp in res.footprint.items():
        x0, y0, x1, y1 = rects[b]
        assert np.all((px[fp] >= x0) & (px[fp] < x1) & (py[fp] >= y0) & (py[fp] < y1))
    st = bc.stats()
    assert abs(st["nominal_samples"] - int(res.samples.sum())) <= 64 * n_tie
    bc.close()


@pytest.mark.parametrize("n,brick,kind,seed", [
    (8, (3, 5, 2), "persp", 1), (8, (8, 8, 8), "ortho", 2), (16, (5, 7, 6), "persp", 3),
    (16, (16, 4, 9), "ortho", 4)])
def test_brute_force_cubes_four_views(n, brick, kind, seed):
    """Tiny random cubes with uneven bricks, four views in one launch."""
    rng = np.random.default_rng(seed)
    dims = (n, n + 1, n - 1)
    vol = rng.uniform(-1, 1, dims[::-1]).astype(np.float32)
    rgba = synth.random_tf(rng, 16, alpha_max=0.7)
    views = [synth.orbit_view(dims, f, kind=kind, width=40, height=32, elevation_deg=25.0, step=0.37, ert=0.8)
             for f in (3, 19, 35, 51)]
    img, bc = gpu_render(vol, brick, views, rgba, -1.0, 1.0, keep=True)
    tf = rc.TransferFunction(rgba, -1.0, 1.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, brick))
    for i, v in enumerate(views):
        res = rc.render_bricked(stored, dims, cam_of(v), tf, 0.37, 0.8)
        err, n_tie, n_ovf = compare(img[i].reshape(-1, 4), res, f"view {i}")
        assert err <= TOL, (i, err)
        assert np.array_equal(bc.visibility_order(i), np.asarray(res.order, np.int32))
    bc.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("src", ["f32 host", "f16 host", "f16 device"])
def test_stored_bricks_bit_exact(storage, src):
    """GPU bricking, ghosts and encoders against the oracle's, element by
    element, from FP32 and FP16 sources in host or device memory (an FP16
    source widens exactly to the FP32 values the encoders take)."""
    import torch
    rng = np.random.default_rng(11)
    dims = (37, 29, 21)
    vol = (rng.standard_normal(dims[::-1]) * 3).astype(np.float32)
    dtype, place = src.split()
    if dtype == "f16":
        vol16 = vol.astype(np.float16)
        vol = vol16.astype(np.float32)
    bc = binding.BrickCaster(0)
    bc.plan(dims, (16, 16, 8), storage=storage, src_dtype=dtype, max_w=16, max_h=16)
    bc.bind()
    source = vol16 if dtype == "f16" else vol
    bc.load(torch.from_numpy(source).cuda() if place == "device" else source)
    lohi, so, mm = bc.bricks()
    bricks = rc.brick_grid(dims, (16, 16, 8))
    for b in bricks:
        g = rc.ghosted_region(vol, b)
        buf, pdims = bc.read_brick(b.index)
        arr = binding.unswizzle(buf, pdims)[:g.shape[0], :g.shape[1], :g.shape[2]]
        tails, repeated = binding.row_tails(buf, pdims)
        assert np.array_equal(tails, repeated)
        assert list(lohi[b.index]) == list(b.lo) + list(b.hi)
        assert mm[b.index, 0] == g.min() and mm[b.index, 1] == g.max()
        if storage == "f32":
            assert np.array_equal(arr, g)
        elif storage == "f16":
            assert np.array_equal(arr, encoders.f16_bits(g))
        else:
            s, o = encoders.brick_scale_offset(float(g.min()), float(g.max()))
            assert so[b.index, 0] == s and so[b.index, 1] == o
            assert np.array_equal(arr, encoders.fp8_encode_brick(g, s, o))
    bc.close()


@pytest.mark.parametrize("storage", ["f16", "fp8"])
def test_precision_forms_match_oracle_on_stored_values(small_cube, storage):
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(vol.shape[::-1], 21, kind="ortho", width=256, height=256, ert=0.99)
    img = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, storage=storage)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    stored = rc.store_bricks(vol, rc.brick_grid(vol.shape[::-1], (64, 64, 64)), storage)
    res = rc.render_bricked(stored, vol.shape[::-1], cam_of(v), tf, 0.5, 0.99)
    err, n_tie, _ = compare(img[0].reshape(-1, 4), res, storage)
    assert err <= TOL, err
    # and the error of the storage form against FP32 data, reported
    ref = rc.render_bricked(rc.store_bricks(vol, rc.brick_grid(vol.shape[::-1], (64, 64, 64))),
                            vol.shape[::-1], cam_of(v), tf, 0.5, 0.99)
    print(storage, "max abs vs FP32 data", np.abs(img[0].reshape(-1, 4) - ref.image).max(),
          "PSNR", rc.psnr(img[0].reshape(-1, 4), ref.image))


def test_uneven_bricks_host_and_device_loads_agree():
    rng = np.random.default_rng(12)
    dims = (70, 50, 45)
    base = synth.CubeRecipe(dims, seed=5, n_sources=8, sigma_lo=2, sigma_hi=6)
    vol = synth.make_cube(base, workers=2)
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(dims, 40, kind="persp", width=96, height=80, ert=0.99)
    a = gpu_render(vol, (32, 32, 32), [v], rgba, vmin, vmax, src="device")
    b = gpu_render(vol, (32, 32, 32), [v], rgba, vmin, vmax, src="host")
    assert np.array_equal(a, b)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    res = rc.render_bricked(rc.store_bricks(vol, rc.brick_grid(dims, (32, 32, 32))), dims, cam_of(v), tf, 0.5, 0.99)
    err, _, _ = compare(a[0].reshape(-1, 4), res, "uneven bricks")
    assert err <= TOL


def test_without_termination_equals_unbricked(small_cube):
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(vol.shape[::-1], 50, kind="persp", width=160, height=120, ert=1.0)
    img = gpu_render(vol, (48, 48, 48), [v], rgba, vmin, vmax)
    res = rc.render_full(vol, cam_of(v), rc.TransferFunction(rgba, vmin, vmax), 0.5, 1.0)
    err = np.abs(img[0].reshape(-1, 4) - res.image).max(axis=1)
    assert err[~res.tie].max() <= TOL


def test_degenerate_inputs(small_cube):
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    zero = rgba.copy()
    zero[:, 3] = 0.0
    v = synth.orbit_view(vol.shape[::-1], 9, kind="persp", width=64, height=48)
    assert np.all(gpu_render(vol, (64, 64, 64), [v], zero, vmin, vmax) == 0.0)
    # the cube behind the viewer: every pixel transparent
    away = synth.orbit_view(vol.shape[::-1], 9, kind="persp", width=64, height=48)
    M = rc.mat_from_col_major(away.modelview)
    M[:3, :] = np.diag([-1.0, 1.0, -1.0]) @ M[:3, :]
    away.modelview = np.ascontiguousarray(M.T).reshape(16)
    assert np.all(gpu_render(vol, (64, 64, 64), [away], rgba, vmin, vmax) == 0.0)


def test_batched_views_equal_single_views_and_repeat(small_cube):
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=120, height=90) for f in (0, 16, 32, 48)]
    batch, bc = gpu_render(vol, (64, 64, 64), views, rgba, vmin, vmax, keep=True)
    again = bc.render().cpu().numpy()
    assert np.array_equal(again, batch.astype(np.float32))
    bc.close()
    for i, v in enumerate(views):
        single = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax)
        assert np.array_equal(single[0], batch[i])


@pytest.mark.parametrize("storage", ["f32", "fp8"])
def test_empty_space_skipping_is_bit_identical(small_cube, storage):
    """Skipping samples in cells whose values map to zero-opacity entries
    changes nothing in the image and only lowers the evaluated count."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=160, height=120) for f in (5, 37)]
    on, bc_on = gpu_render(vol, (48, 40, 64), views, rgba, vmin, vmax, storage=storage, keep=True,
                           options={binding.BC_OPT_EMPTY_SKIP: 1})
    off, bc_off = gpu_render(vol, (48, 40, 64), views, rgba, vmin, vmax, storage=storage, keep=True,
                             options={binding.BC_OPT_EMPTY_SKIP: 0})
    assert np.array_equal(on, off)
    s_on, s_off = bc_on.stats(), bc_off.stats()
    assert s_on["nominal_samples"] == s_off["nominal_samples"]
    assert s_off["evaluated_samples"] == s_off["nominal_samples"]
    assert s_on["evaluated_samples"] < 0.5 * s_on["nominal_samples"]
    # a new table (different opacity) re-classifies the cells
    rgba2 = rgba.copy()
    rgba2[:, 3] = np.where(rgba2[:, 3] > 0, rgba2[:, 3], 0.02)
    bc_on.set_transfer_function(rgba2, vmin, vmax)
    bc_off.set_transfer_function(rgba2, vmin, vmax)
    a = bc_on.render().cpu().numpy()
    b = bc_off.render().cpu().numpy()
    assert np.array_equal(a, b)
    assert bc_on.stats()["evaluated_samples"] == bc_on.stats()["nominal_samples"]
    bc_on.close()
    bc_off.close()


def test_fp8_decode_of_every_code():
    """A brick holding every finite E4M3 value (scale 1, offset 0, so the codes
    are the values themselves), seen along z with samples on voxel centres and
    a steep table around 0: subnormal, normal and negative codes all reach the
    image, which must match the oracle's table-based decoding."""
    codes = np.arange(256)
    vals = encoders.e4m3_value(codes)
    vals[np.isnan(vals)] = 0.0
    vol = np.zeros((2, 16, 16), np.float32)
    vol.reshape(-1)[:256] = vals
    vol.reshape(-1)[256:] = vals[::-1]
    vol[0, 0, 0], vol[1, 15, 15] = -448.0, 448.0        # brick range [-448, 448]: s = 1, o = 0
    dims = (16, 16, 2)
    rng = np.random.default_rng(13)
    rgba = synth.random_tf(rng, 64, alpha_max=0.9)
    v = synth.axis_view(dims, "z", 16, 16, step=1.0, ert=1.0)
    img, bc = gpu_render(vol, (16, 16, 2), [v], rgba, -0.03, 0.03, storage="fp8", keep=True)
    lohi, so, _ = bc.bricks()
    assert so[0, 0] == 1.0 and so[0, 1] == 0.0
    bc.close()
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (16, 16, 2)), "fp8")
    res = rc.render_bricked(stored, dims, cam_of(v), rc.TransferFunction(rgba, -0.03, 0.03), 1.0, 1.0)
    err, _, _ = compare(img[0].reshape(-1, 4), res, "fp8 subnormal codes")
    assert err <= TOL, err
    # the subnormal codes matter: decoding them as zero changes the oracle image
    flushed = vol.copy()
    sub = (np.abs(flushed) < 2.0 ** -6) & (flushed != 0)
    assert sub.sum() >= 10
    flushed[sub] = 0.0
    res0 = rc.render_bricked(rc.store_bricks(flushed, rc.brick_grid(dims, (16, 16, 2)), "fp8"), dims, cam_of(v),
                             rc.TransferFunction(rgba, -0.03, 0.03), 1.0, 1.0)
    assert np.abs(res0.image - res.image).max() > 100 * TOL


def test_graph_frames_match_eager_frames(small_cube):
    """Captured frames replayed many times, with eager frames and host syncs in
    between, give the eager frames bit for bit (one graph per input slot)."""
    import torch
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=96, height=72) for f in range(0, 64, 9)]
    _, eager = gpu_render(vol, (64, 64, 64), views[:1], rgba, vmin, vmax, keep=True)
    refs = []
    for v in views:
        eager.set_views([v])
        refs.append(eager.render().clone())
    _, g = gpu_render(vol, (64, 64, 64), views[:1], rgba, vmin, vmax, keep=True,
                      options={binding.BC_OPT_GRAPH: 1})
    out = torch.empty_like(refs[0])
    for rep in range(3):
        for i, v in enumerate(views):
            g.set_views([v])
            g.render(out)
            torch.cuda.synchronize()
            assert torch.equal(out, refs[i]), (rep, i)
            eager.set_views([views[-1 - i]])
            eager.render()
    g.close()
    eager.close()


def test_autotune_keeps_the_image(small_cube):
    """The launch shape changes only FP32 rounding inside a sample chunk (the
    chunk size sets the base the in-chunk positions are measured from); the
    screen tile shape changes nothing."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(vol.shape[::-1], 11, kind="persp", width=128, height=96)
    img, bc = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, keep=True)
    chunk, wgs, tile_w = bc.autotune(frames=2)
    assert chunk in (32, 64) and wgs > 0 and tile_w in (4, 8, 16)
    again = bc.render().cpu().numpy()
    assert np.abs(again - img).max() <= 1e-6
    bc.close()


def test_xcd_queues_and_chunks_do_not_change_the_image(small_cube):
    """Work queues, workgroup counts and the screen tile shape (8x8, 16x4,
    4x16; the 90-pixel-high frame leaves partial tiles) only regroup
    independent rays: bit-identical.  The chunk size changes FP32 rounding
    inside a chunk only."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=120, height=90) for f in (2, 40)]
    ref = {ch: gpu_render(vol, (40, 48, 56), views, rgba, vmin, vmax,
                          options={binding.BC_OPT_XCD_QUEUES: 0, binding.BC_OPT_SAMPLE_CHUNK: ch})
           for ch in (32, 64)}
    for q, ch, wg, tw in ((1, 64, 64, 8), (1, 32, 3, 16), (0, 64, 1000, 4), (1, 32, 2000, 8), (1, 32, 1024, 4),
                          (0, 64, 512, 16)):
        img = gpu_render(vol, (40, 48, 56), views, rgba, vmin, vmax,
                         options={binding.BC_OPT_XCD_QUEUES: q, binding.BC_OPT_SAMPLE_CHUNK: ch,
                                  binding.BC_OPT_RENDER_WORKGROUPS: wg, binding.BC_OPT_TILE_WIDTH: tw})
        assert np.array_equal(img, ref[ch]), (q, ch, wg, tw)
    assert np.abs(ref[32] - ref[64]).max() <= 1e-6
    tf = rc.TransferFunction(rgba, vmin, vmax)
    stored = rc.store_bricks(vol, rc.brick_grid(vol.shape[::-1], (40, 48, 56)))
    res = rc.render_bricked(stored, vol.shape[::-1], cam_of(views[0]), tf, 0.5, 0.99)
    err, _, _ = compare(ref[64][0].reshape(-1, 4), res, "xcd queues and chunks")
    assert err <= TOL


@pytest.mark.parametrize("kind", ["persp", "ortho"])
def test_thin_edge_bricks_like_table1_shapes(kind):
    """The paper's cube shapes split into 256^3 bricks leave thin edge bricks
    (1025 = 4 x 256 + 1 for the HIPASS cube).  A cube of 300 x 260 x 257 in
    128^3 bricks has edge bricks 44, 4 and 1 voxels thick: compositing and
    maximum intensity projection both match the oracle.

    A few rays of this view end with opacity just under the termination
    threshold for dozens of nearly transparent samples, each an early-
    termination near-tie (stop there or go on); the oracle lists such a ray's
    reachable ends linearly, so every ray is compared."""
    from oracle import mip
    dims = (300, 260, 257)
    recipe = synth.CubeRecipe(dims, seed=21, n_sources=60, sigma_lo=4.0, sigma_hi=12.0)
    vol = synth.make_cube(recipe, workers=8)
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(dims, 27, kind=kind, width=160, height=120, elevation_deg=35.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (128, 128, 128)))
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img = gpu_render(vol, (128, 128, 128), [v], rgba, vmin, vmax)
    res = rc.render_bricked(stored, dims, cam_of(v), tf, 0.5, 0.99)
    err, _, n_ovf = compare(img[0].reshape(-1, 4), res, f"thin edge bricks {kind}")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.3
    img = gpu_render(vol, (128, 128, 128), [v], rgba, vmin, vmax, op=("mip", "voxel"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, "voxel")
    assert compare_mip(img[0].reshape(-1, 4), res, f"thin edge bricks {kind} mip") <= TOL


def test_more_than_64_bricks_per_block_of_tiles():
    """4096 bricks of 4^3 voxels (the brick limit) over a 64^3 cube: each 4x4
    block of screen tiles meets hundreds of brick rectangles, so the sort-last
    fold walks its brick list in several slices of 64.  Compositing and
    maximum intensity projection both match the oracle."""
    from oracle import mip
    dims = (64, 64, 64)
    vol = synth.make_cube(synth.CubeRecipe(dims, seed=31, n_sources=12, sigma_lo=2.0, sigma_hi=5.0), workers=4)
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(dims, 5, kind="persp", width=64, height=48, elevation_deg=30.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (4, 4, 4)))
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img, bc = gpu_render(vol, (4, 4, 4), [v], rgba, vmin, vmax, keep=True)
    rects = bc.rects(0)   # pixel bounds, whole 8x8 tiles
    bc.close()
    # bricks whose rectangle meets each 4x4 block of tiles (32x32 pixels)
    most = 0
    for y0 in range(0, 48, 32):
        for x0 in range(0, 64, 32):
            meet = (rects[:, 0] < x0 + 32) & (rects[:, 2] > x0) & (rects[:, 1] < y0 + 32) & (rects[:, 3] > y0)
            most = max(most, int(meet.sum()))
    assert most > 64
    res = rc.render_bricked(stored, dims, cam_of(v), tf, 0.5, 0.99)
    err, _, n_ovf = compare(img[0].reshape(-1, 4), res, "4096 bricks")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.3
    img = gpu_render(vol, (4, 4, 4), [v], rgba, vmin, vmax, op=("mip", "voxel"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, "voxel")
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL


def test_between_64_and_128_bricks():
    """100 bricks (5x5x4 of 8x8x10 voxels over a 40^3 cube): the per-tile
    compositing kernel (up to 128 bricks) walks the visibility order in two
    slices of 64.  Compositing and maximum intensity projection match the
    oracle at every pixel of a partial-tile frame."""
    from oracle import mip
    dims = (40, 40, 40)
    vol = synth.make_cube(synth.CubeRecipe(dims, seed=17, n_sources=10, sigma_lo=2.0, sigma_hi=5.0), workers=4)
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(dims, 11, kind="persp", width=70, height=50, elevation_deg=25.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (8, 8, 10)))
    assert len(rc.brick_grid(dims, (8, 8, 10))) == 100
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img = gpu_render(vol, (8, 8, 10), [v], rgba, vmin, vmax)
    res = rc.render_bricked(stored, dims, cam_of(v), tf, 0.5, 0.99)
    err, _, _ = compare(img[0].reshape(-1, 4), res, "100 bricks")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.3
    img = gpu_render(vol, (8, 8, 10), [v], rgba, vmin, vmax, op=("mip", "fixed"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, 0.5)
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL


@pytest.mark.parametrize("dims,brick", [((1, 1, 1), (1, 1, 1)), ((2, 1, 3), (1, 1, 2)), ((5, 1, 1), (2, 1, 1)),
                                        ((3, 4, 1), (3, 4, 1))])
def test_smallest_cubes_bricks_and_frames(dims, brick):
    """The smallest geometry the method has: cubes one voxel thick, bricks of a
    single voxel (ghosts on every side are clamped copies), frames of 1x1,
    3x2 and 9x7 pixels, and an axis-aligned orthographic view with one pixel
    per voxel column.  Compositing and maximum intensity projection against
    the oracle."""
    from oracle import mip
    rng = np.random.default_rng(41 + sum(dims))
    vol = rng.uniform(-1, 1, dims[::-1]).astype(np.float32)
    rgba = synth.random_tf(rng, 16, alpha_max=0.7)
    tf = rc.TransferFunction(rgba, -1.0, 1.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, brick))
    views = [synth.orbit_view(dims, f, kind=k, width=w, height=h, elevation_deg=25.0, step=0.37, ert=0.8)
             for f, k, w, h in ((3, "persp", 1, 1), (19, "ortho", 3, 2), (35, "persp", 9, 7))]
    views.append(synth.axis_view(dims, "z", dims[0], dims[1], step=0.5, ert=1.0))
    lit = 0
    for v in views:
        img = gpu_render(vol, brick, [v], rgba, -1.0, 1.0)
        res = rc.render_bricked(stored, dims, cam_of(v), tf, v.step, v.ert)
        err, _, n_ovf = compare(img[0].reshape(-1, 4), res, f"{dims} {v.width}x{v.height}")
        assert err <= TOL, (v.width, v.height, err)
        lit += int(res.image[:, 3].max() > 0.2)
    assert lit >= 3
    v = views[2]
    img = gpu_render(vol, brick, [v], rgba, -1.0, 1.0, op=("mip", "voxel"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, "voxel")
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL


def _two_entry_tf(rgb, alpha):
    return np.array([[0.0, 0.0, 0.0, 0.0], list(rgb) + [alpha]], np.float32)


def test_constructed_exact_ties_match_an_enumerated_result():
    """The oracle's exact-tie constructions rendered by the GPU: a sample on
    the face between two FP8 bricks with different scale and offset (two
    reachable pixels), opacity reaching tau exactly at a brick's second sample
    (the GPU stops there, as FP32 reaches 3/4 exactly), and opacity held
    within the tie margin of tau over 148 transparent samples."""
    # face tie between FP8 bricks
    dims = (2, 2, 6)
    zcol = np.array([0.0, 1.0, 3.0, 2.0, 0.5, 0.25], np.float32)
    vol = np.ascontiguousarray(np.broadcast_to(zcol[:, None, None], (6, 2, 2)))
    rgba = _two_entry_tf((1.0, 0.5, 0.25), 0.75)
    v = synth.axis_view(dims, "z", 2, 2, step=2.0, ert=1.0)
    img = gpu_render(vol, (2, 2, 3), [v], rgba, 0.0, 4.0, storage="fp8", dt_ref=2.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (2, 2, 3)), "fp8")
    res = rc.render_bricked(stored, dims, cam_of(v), rc.TransferFunction(rgba, 0.0, 4.0, 2.0), 2.0, 1.0)
    assert all(len(res.branches[r]) == 2 for r in range(4))
    err, _, _ = compare(img[0].reshape(-1, 4), res, "fp8 face tie")
    assert err <= TOL
    # exact termination tie: the FP32 opacity is 0.5, then 0.75 = tau
    dims = (1, 1, 8)
    vol = np.ones((8, 1, 1), np.float32)
    rgba = _two_entry_tf((0.75, 0.5, 0.25), 0.5)
    v = synth.axis_view(dims, "z", 1, 1, step=1.0, ert=0.75)
    img = gpu_render(vol, (1, 1, 4), [v], rgba, 0.0, 1.0)
    assert np.array_equal(img[0, 0, 0], np.array([0.75, 0.5, 0.25, 1.0], np.float32) * 0.9375)
    # a long run of transparent samples within the tie margin of tau
    dims = (1, 1, 400)
    col = np.zeros(400, np.float32)
    col[0:2] = 1.0
    col[150:] = 1.0
    vol = col.reshape(400, 1, 1)
    tau = 0.75 + 2.0 ** -15
    v = synth.axis_view(dims, "z", 1, 1, step=1.0, ert=tau)
    img = gpu_render(vol, (1, 1, 200), [v], rgba, 0.0, 1.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (1, 1, 200)))
    res = rc.render_bricked(stored, dims, cam_of(v), rc.TransferFunction(rgba, 0.0, 1.0), 1.0, tau)
    err, _, _ = compare(img[0].reshape(-1, 4), res, "transparent run at tau")
    assert err <= TOL


def test_timing_windows(small_cube):
    """Stage timing: every stage positive with events between all stages; with
    only the ray caster's two events, set-up and compositing read zero and the
    per-frame times are the ray caster's; an enable outside {0, 1, 2} is refused."""
    import torch
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=160, height=120) for f in (3, 9, 21)]
    img, bc = gpu_render(vol, (48, 40, 64), views[:1], rgba, vmin, vmax, keep=True)
    out = torch.empty((1, 120, 160, 4), device="cuda")
    for stages in (True, False):
        bc.enable_timing(True, stages=stages)
        for v in views:
            bc.set_views([v])
            bc.render(out)
        ms, n = bc.timing()
        ft = bc.frame_times()
        bc.enable_timing(False)
        assert n == len(views) and len(ft) == len(views)
        assert ms[1] > 0
        if stages:
            assert ms[0] > 0 and ms[2] > 0
            assert sum(ft) >= ms[1]
        else:
            assert ms[0] == 0 and ms[2] == 0
            assert abs(sum(ft) - ms[1]) <= 1e-6 * max(ms[1], 1.0)
    with pytest.raises(binding.BrickcastError):
        bc._check(bc.lib.bc_enable_timing(bc.h, 3))
    bc.set_views(views[:1])
    assert np.array_equal(bc.render(out).cpu().numpy().astype(np.float64), img)
    bc.close()


@pytest.mark.parametrize("K,kind", [(2, "random"), (2, "ramp"), (1024, "ramp"), (1025, "ramp"), (4096, "ramp")])
def test_table_sizes_at_the_limits(small_cube, K, kind):
    """Tables of 2 entries (the smallest), 1024 (the largest the ray caster
    stages in LDS), 1025 (read from device memory) and 4096 (the limit):
    compositing and maximum intensity projection match the oracle at every
    pixel of a partial-tile frame.  The large tables are smooth (the ramp of
    the workloads, opacity zero below 3 so skipping stays in play): the table
    coordinate is FP32, so the interpolated value's rounding reaches the
    colour multiplied by (K-1)/(vmax-vmin) and by the step between
    neighbouring entries, and a random 1024-entry table exceeds the 2e-5 bar
    (2.8e-5 on this frame) while a smooth one stays far below it."""
    from oracle import mip
    vol = small_cube
    vmin, vmax = float(vol.min()), float(vol.max())
    if kind == "random":
        rgba = synth.random_tf(np.random.default_rng(100 + K), K, alpha_max=0.5)
    else:
        rgba = synth.ramp_tf(vmin, vmax, K=K)
    v = synth.orbit_view(vol.shape[::-1], 13, kind="persp", width=90, height=70)
    dims = vol.shape[::-1]
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (64, 64, 64)))
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax)
    res = rc.render_bricked(stored, dims, cam_of(v), tf, 0.5, 0.99)
    err, _, _ = compare(img[0].reshape(-1, 4), res, f"K = {K} ({kind})")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.05
    img = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, op=("mip", "fixed"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, 0.5)
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL


@pytest.mark.parametrize("eye,target", [((70.3, 61.7, 45.2), (20.0, 90.0, 120.0)),    # inside a brick
                                        ((64.0, 64.0, 64.0), (128.0, 20.0, 10.0)),    # on a brick corner
                                        ((30.5, 140.0, 64.2), (64.0, 0.0, 64.0))])    # outside, close
def test_eye_inside_or_next_to_the_cube(small_cube, eye, target):
    """Fly-through views: the eye inside a brick (rays start at the eye, that
    brick's rectangle is the whole frame and its order key is negative, bricks
    behind the eye take no samples), on the corner shared by eight bricks, and
    just outside with a wide field of view (brick corners behind the near
    plane).  Compositing and maximum intensity projection match the oracle at
    every pixel, and the visibility order matches bit for bit."""
    from oracle import mip
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    W, H = 72, 54
    v = synth.ViewSpec(synth.look_at(eye, target, (0.0, 1.0, 0.0)), synth.perspective(80.0, W / H, 0.1, 500.0), W, H)
    dims = vol.shape[::-1]
    bricks = rc.brick_grid(dims, (64, 64, 64))
    stored = rc.store_bricks(vol, bricks)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img, bc = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, keep=True)
    cam = cam_of(v)
    assert np.array_equal(bc.visibility_order(0), np.asarray(rc.visibility_order(bricks, cam)[0], np.int32))
    bc.close()
    res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.99)
    err, _, _ = compare(img[0].reshape(-1, 4), res, f"eye {eye}")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.05
    img = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, op=("mip", "fixed"))
    res = mip.render_mip_bricked(stored, dims, cam, tf, 0.5)
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL


@pytest.mark.parametrize("step,brick,size", [(0.05, (20, 18, 22), (32, 24)), (3.3, (6, 6, 6), (44, 36)),
                                             (7.9, (6, 6, 6), (44, 36))])
def test_steps_far_below_a_voxel_and_above_a_brick(step, brick, size):
    """Sample steps of 0.05 voxels (up to about 750 samples, two dozen chunks,
    per ray in a brick) and of 3.3 and 7.9 voxels against 6-voxel bricks (most
    bricks take zero or one sample of a ray, and a sample's owner brick is
    decided far from the previous one): compositing with opacity correction
    for the step, and maximum intensity projection, against the oracle."""
    from oracle import mip
    dims = (60, 54, 66)
    vol = synth.make_cube(synth.CubeRecipe(dims, seed=41, n_sources=9, sigma_lo=2.0, sigma_hi=6.0), workers=4)
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(dims, 19, kind="persp", width=size[0], height=size[1], elevation_deg=-15.0, step=step,
                         ert=0.95)
    bricks = rc.brick_grid(dims, brick)
    stored = rc.store_bricks(vol, bricks)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    img = gpu_render(vol, brick, [v], rgba, vmin, vmax)
    res = rc.render_bricked(stored, dims, cam_of(v), tf, step, 0.95)
    err, _, _ = compare(img[0].reshape(-1, 4), res, f"step {step}")
    assert err <= TOL
    assert res.image[:, 3].max() > 0.05
    img = gpu_render(vol, brick, [v], rgba, vmin, vmax, op=("mip", "fixed"))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, step)
    assert mip.max_abs_with_branches(img[0].reshape(-1, 4), res).max() <= TOL
