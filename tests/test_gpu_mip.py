"""Maximum intensity projection on the HIP path (through the C ABI) against
the FP64 oracle on the same seeded inputs: max |GPU - oracle| <= 2e-5 per RGBA
channel of the colour-mapped image (near-tie rays may match any of their
branches), fixed and per-voxel steps, every storage form; empty-space
skipping bit-identical; early termination at the brick maximum."""
import numpy as np
import pytest

from oracle import mip
from oracle import raycast as rc
from paper_1205_0282_amd import binding, synth

from gpu_util import TOL, cam_of, gpu_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_cube():
    return synth.make_cube(synth.RECIPE_SMALL, workers=4)


def _ramp(vol):
    vmin, vmax = float(vol.min()), float(vol.max())
    return synth.ramp_tf(vmin, vmax), vmin, vmax


def _check(img, res, tol=TOL):
    err = mip.max_abs_with_branches(img.reshape(-1, 4), res)
    return float(err.max()), int(res.tie.sum())


@pytest.mark.parametrize("storage", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("kind,step", [("ortho", 0.5), ("persp", "voxel"), ("ortho", "voxel")])
def test_small_cube_matches_oracle(small_cube, storage, kind, step):
    """128^3 cube, 2x2x2 bricks of 64^3, 256x256: per-brick maxima from the
    stored values, merged, colour-mapped."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    dims = vol.shape[::-1]
    v = synth.orbit_view(dims, 13, kind=kind, width=256, height=256, step=0.5 if step == "voxel" else step)
    img, bc = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, storage=storage, keep=True,
                         op=("mip", "voxel" if step == "voxel" else "fixed"))
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (64, 64, 64)), storage)
    res = mip.render_mip_bricked(stored, dims, cam_of(v), rc.TransferFunction(rgba, vmin, vmax), step)
    err, n_tie = _check(img[0], res)
    print(f"{storage} {kind} {step}: max err {err:.3g}, near-tie rays {n_tie}")
    assert err <= TOL
    assert (res.samples > 0).sum() > 10000
    assert np.unique(res.image[res.samples > 0, 0]).size > 100     # not a flat image
    st = bc.stats()
    assert 0 < st["nominal_samples"] <= int(res.samples.sum())
    bc.close()


@pytest.mark.parametrize("n,brick,kind,seed,step", [
    (8, (3, 5, 2), "persp", 1, 0.37), (8, (8, 8, 8), "ortho", 2, "voxel"), (16, (5, 7, 6), "persp", 3, "voxel"),
    (16, (16, 4, 9), "ortho", 4, 0.61)])
def test_brute_force_cubes_four_views(n, brick, kind, seed, step):
    """Tiny random cubes with uneven bricks, random colour maps, four views in
    one launch."""
    rng = np.random.default_rng(seed)
    dims = (n, n + 1, n - 1)
    vol = rng.uniform(-1, 1, dims[::-1]).astype(np.float32)
    rgba = synth.random_tf(rng, 16, alpha_max=1.0)
    views = [synth.orbit_view(dims, f, kind=kind, width=40, height=32, elevation_deg=25.0,
                              step=0.37 if step == "voxel" else step) for f in (3, 19, 35, 51)]
    img = gpu_render(vol, brick, views, rgba, -1.0, 1.0, op=("mip", "voxel" if step == "voxel" else "fixed"))
    tf = rc.TransferFunction(rgba, -1.0, 1.0)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, brick))
    for i, v in enumerate(views):
        res = mip.render_mip_bricked(stored, dims, cam_of(v), tf, step)
        err, _ = _check(img[i], res)
        assert err <= TOL, (i, err)


@pytest.mark.parametrize("storage", ["f32", "fp8"])
def test_empty_space_skipping_is_bit_identical(small_cube, storage):
    """Cells whose values all map to the colour map's leading run of equal
    entries are skipped: same image bit for bit, far fewer evaluations."""
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=160, height=120) for f in (5, 37)]
    on, bc_on = gpu_render(vol, (48, 40, 64), views, rgba, vmin, vmax, storage=storage, keep=True,
                           options={binding.BC_OPT_EMPTY_SKIP: 1}, op=("mip", "voxel"))
    off, bc_off = gpu_render(vol, (48, 40, 64), views, rgba, vmin, vmax, storage=storage, keep=True,
                             options={binding.BC_OPT_EMPTY_SKIP: 0}, op=("mip", "voxel"))
    assert np.array_equal(on, off)
    s_on, s_off = bc_on.stats(), bc_off.stats()
    assert s_off["evaluated_samples"] <= s_off["nominal_samples"]
    assert s_on["evaluated_samples"] < 0.5 * s_off["evaluated_samples"]
    # a colour map with no constant leading run skips nothing
    rgba2 = rgba.copy()
    rgba2[:, 0] = np.linspace(0.0, 1.0, len(rgba2))
    for bc in (bc_on, bc_off):
        bc.set_transfer_function(rgba2, vmin, vmax)
    a = bc_on.render().cpu().numpy()
    b = bc_off.render().cpu().numpy()
    assert np.array_equal(a, b)
    assert bc_on.stats()["evaluated_samples"] == bc_off.stats()["evaluated_samples"]
    bc_on.close()
    bc_off.close()


def test_rays_stop_at_the_brick_maximum():
    """A constant cube: every sample equals each brick's maximum, so every ray
    stops after its first sample in each brick it enters."""
    dims = (24, 20, 16)
    vol = np.full(dims[::-1], 2.5, np.float32)
    rgba = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 0.5, 0.25, 1.0]], np.float32)
    v = synth.orbit_view(dims, 9, kind="persp", width=64, height=48)
    img, bc = gpu_render(vol, (8, 8, 8), [v], rgba, 0.0, 5.0, keep=True, op=("mip", "fixed"),
                         options={binding.BC_OPT_EMPTY_SKIP: 0})
    st = bc.stats()
    bc.close()
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (8, 8, 8)))
    res = mip.render_mip_bricked(stored, dims, cam_of(v), rc.TransferFunction(rgba, 0.0, 5.0), 0.5,
                                 want_subimages=True)
    entered = sum(int(np.isfinite(s).sum()) for s in res.subimages.values())
    n_tie = int(res.tie.sum())
    assert abs(st["nominal_samples"] - entered) <= 2 * n_tie
    assert st["evaluated_samples"] == st["nominal_samples"]
    assert entered > 2 * int((res.samples > 0).sum())          # most rays cross several bricks
    hit = res.samples > 0
    assert np.allclose(img[0].reshape(-1, 4)[hit], [0.5, 0.25, 0.125, 0.5], atol=1e-7)
    assert np.all(img[0].reshape(-1, 4)[~hit] == 0.0)


def test_operator_switches_between_frames_and_graphs(small_cube):
    """Composite and MIP frames alternate on one context, eager and captured:
    each matches a fresh context's frame bit for bit."""
    import torch
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    views = [synth.orbit_view(vol.shape[::-1], f, kind="persp", width=96, height=72) for f in (3, 30)]
    ref_c = gpu_render(vol, (64, 64, 64), views, rgba, vmin, vmax)
    ref_m = gpu_render(vol, (64, 64, 64), views, rgba, vmin, vmax, op=("mip", "voxel"))
    assert not np.array_equal(ref_c, ref_m)
    for graph in (0, 1):
        _, bc = gpu_render(vol, (64, 64, 64), views, rgba, vmin, vmax, keep=True,
                           options={binding.BC_OPT_GRAPH: graph})
        for rep in range(2):
            bc.set_operator("mip", "voxel")
            a = bc.render().cpu().numpy()
            bc.set_operator("composite", "fixed")
            b = bc.render().cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(a, ref_m.astype(np.float32)), (graph, rep)
            assert np.array_equal(b, ref_c.astype(np.float32)), (graph, rep)
        bc.close()


def test_learned_frames_refuse_mip(small_cube):
    vol = small_cube
    rgba, vmin, vmax = _ramp(vol)
    v = synth.orbit_view(vol.shape[::-1], 3, kind="persp", width=64, height=48)
    _, bc = gpu_render(vol, (64, 64, 64), [v], rgba, vmin, vmax, keep=True)
    bc.cnn_setup(1, 24, 32)
    bc.cnn_set_weights(np.zeros(binding.CNN_N_PARAMS, np.float32))
    bc.set_learned(True)
    bc.set_operator("mip", "fixed")
    with pytest.raises(binding.BrickcastError) as e:
        bc.render()
    assert e.value.code == binding.BC_E_UNSUPPORTED
    bc.close()
