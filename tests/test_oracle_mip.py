"""Pins for the maximum-intensity-projection oracle: textbook discrete rays
(axis-aligned and 45-degree views through voxel centres), a closed form for a
linear field, brute force with an independent scalar formulation, and the
order-free merge of bricks."""
import math

import numpy as np
import pytest

from oracle import mip
from oracle import raycast as rc
from paper_1205_0282_amd import synth


def _cam(v: synth.ViewSpec):
    return rc.Camera(v.modelview, v.projection, v.width, v.height)


def _identity_map(vmin, vmax):
    """Colour map whose red channel is (m - vmin) / (vmax - vmin), clamped."""
    rgba = np.array([[0.0, 0.0, 0.0, 1.0], [1.0, 1.0, 1.0, 1.0]], np.float32)
    return rc.TransferFunction(rgba, vmin, vmax)


def _diag_view(dims, width):
    """Orthographic view along (1, 0, 1)/sqrt(2) with pixel columns 1/sqrt(2)
    apart (odd width), so every ray lies on a line x - z = m through voxel
    centres; rows on voxel centres in y."""
    nx, ny, nz = dims
    assert width % 2 == 1
    f = np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
    # eye on the plane x = z, outside the cube; screen right is (-1, 0, 1)/sqrt(2)
    h = (nx + nz) / 4.0
    eye = np.array([h, ny / 2.0, h]) - f * (nx + nz)
    mv = synth.look_at(eye, eye + f, (0.0, 1.0, 0.0))
    half_w = width / (2.0 * math.sqrt(2.0))
    pr = synth.ortho(-half_w, half_w, -ny / 2.0, ny / 2.0, 0.5, 4.0 * (nx + nz))
    return synth.ViewSpec(mv, pr, width, ny, math.sqrt(2.0), 1.0)


# -------------------------------------------------------------- textbook views
@pytest.mark.parametrize("step", [1.0, "voxel"])
def test_axis_view_is_max_along_z(step):
    """Axis-aligned orthographic view with pixel centres on voxel centres and a
    one-voxel step (fixed, or the per-voxel policy, which is one voxel here):
    every sample is a voxel centre, so the projection is the array maximum
    along z."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 7, 6, 11
    vol = rng.uniform(-2, 3, (nz, ny, nx)).astype(np.float32)
    tf = _identity_map(-2.0, 3.0)
    cam = _cam(synth.axis_view((nx, ny, nz), "z", nx, ny, step=1.0))
    res = mip.render_mip_full(vol, cam, tf, step)
    m = res.vmax.reshape(ny, nx)
    exp = vol.max(axis=0)[::-1, ::-1].astype(np.float64)    # row 0 at the top, px -> column nx-1-px
    assert np.allclose(m, exp, atol=1e-12, rtol=0)
    assert np.all(res.samples == nz)
    assert np.allclose(res.image[:, 0], (res.vmax + 2.0) / 5.0, atol=1e-12)


def test_diagonal_view_visits_one_voxel_per_slice():
    """45-degree view in the xz plane with the per-voxel step: dt = sqrt(2), so
    the samples of the ray on the line z = x + m are the voxel centres
    (j, m + j) -- the discrete ray of the textbook -- and the projection is the
    maximum over that diagonal of the array."""
    rng = np.random.default_rng(6)
    nx, ny, nz = 9, 3, 7
    vol = rng.uniform(0, 1, (nz, ny, nx)).astype(np.float32)
    W = 2 * (nx + nz) + 1
    v = _diag_view((nx, ny, nz), W)
    cam = _cam(v)
    tf = _identity_map(0.0, 1.0)
    res = mip.render_mip_full(vol, cam, tf, "voxel")
    o, d = cam.rays(np.arange(W), np.zeros(W, int))
    assert np.allclose(mip.per_voxel_step(d), math.sqrt(2.0), atol=1e-12)
    m = res.vmax.reshape(ny, W)
    checked = 0
    for px in range(W):
        # the ray's line: z - x = mm (an integer up to rounding)
        mm = o[px, 2] - o[px, 0]
        k = int(round(mm))
        assert abs(mm - k) < 1e-9
        # the textbook diagonal through voxel centres (i, k + i) inside the cube
        cells = [(i, k + i) for i in range(nx) if 0 <= k + i < nz]
        for py in range(ny):
            yy = ny - 1 - py
            if not cells:
                assert res.samples.reshape(ny, W)[py, px] == 0
                continue
            exp = max(float(vol[z, yy, x]) for x, z in cells)
            assert abs(m[py, px] - exp) < 1e-9
            assert res.samples.reshape(ny, W)[py, px] == len(cells)
            checked += 1
    assert checked == ny * (nx + nz - 1)   # every diagonal that meets the cube


def test_fixed_step_matches_per_voxel_where_equal():
    """On the diagonal view the fixed step sqrt(2) and the per-voxel policy
    place the same samples."""
    rng = np.random.default_rng(7)
    dims = (8, 3, 8)
    vol = rng.normal(size=dims[::-1]).astype(np.float32)
    v = _diag_view(dims, 2 * 16 + 1)
    cam = _cam(v)
    tf = _identity_map(-3.0, 3.0)
    a = mip.render_mip_full(vol, cam, tf, "voxel")
    b = mip.render_mip_full(vol, cam, tf, math.sqrt(2.0))
    assert np.allclose(a.vmax, b.vmax, atol=1e-9)


# -------------------------------------------------------------- closed form
def _slab_scalar(o, d, n):
    t0, t1 = -math.inf, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (0.0 <= o[a] < n[a]):
                return None
            continue
        ta, tb = (0.0 - o[a]) / d[a], (n[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    t0 = max(t0, 0.0)
    return (t0, t1) if t0 < t1 else None


@pytest.mark.parametrize("step", [0.5, 0.8, "voxel"])
@pytest.mark.parametrize("frame", [3, 21, 40])
def test_linear_field_maximum_is_the_last_sample(step, frame):
    """v = g . clamp(p, 1/2, N - 1/2) + c with g_a d_a >= 0 increases along every
    ray of an orthographic view, so the projection is the value at the ray's
    last sample t_in + (n - 1/2) dt (trilinear interpolation is exact for a
    linear field; the clamp is the edge addressing)."""
    dims = (10, 8, 12)
    v = synth.orbit_view(dims, frame, kind="ortho", width=24, height=20, elevation_deg=25.0)
    cam = _cam(v)
    dvec = np.asarray(cam.view_dir)
    g = np.sign(dvec) * np.array([0.7, 1.3, 0.4])
    c0 = 0.25
    n = np.asarray(dims, float)
    zc, yc, xc = [np.arange(k) + 0.5 for k in dims[::-1]]
    vol = (g[0] * xc[None, None, :] + g[1] * yc[None, :, None] + g[2] * zc[:, None, None] + c0)
    res = mip.render_mip_full(vol.astype(np.float64), cam, _identity_map(-20.0, 20.0), step)
    px, py = np.meshgrid(np.arange(v.width), np.arange(v.height))
    o, d = cam.rays(px.ravel(), py.ravel())
    hits = 0
    for r in range(len(o)):
        seg = _slab_scalar(o[r], d[r], n)
        dt = 1.0 / max(abs(x) for x in d[r]) if step == "voxel" else step
        if seg is None:
            assert res.samples[r] == 0 and np.all(res.image[r] == 0)
            continue
        t_in, t_out = seg
        cnt = 0
        while t_in + (cnt + 0.5) * dt < t_out:
            cnt += 1
        assert res.samples[r] == cnt
        if cnt == 0:
            assert np.all(res.image[r] == 0)
            continue
        p = o[r] + (t_in + (cnt - 0.5) * dt) * d[r]
        exp = float(np.dot(g, np.clip(p, 0.5, n - 0.5))) + c0
        assert abs(res.vmax[r] - exp) < 1e-9
        hits += 1
    assert hits > 100


# --------------------------------------------------------------- brute force
def _brute_mip_ray(vol, cam, dt_or_voxel, px, py):
    """Scalar formulation: slab entry, explicit sample loop, 8 explicit
    clamped corners per sample."""
    nz, ny, nx = vol.shape
    o, d = cam.rays(np.array([px]), np.array([py]))
    o, d = o[0], d[0]
    seg = _slab_scalar(o, d, (nx, ny, nz))
    if seg is None:
        return None, 0
    t_in, t_out = seg
    dt = 1.0 / max(abs(x) for x in d) if dt_or_voxel == "voxel" else dt_or_voxel
    best, cnt = -math.inf, 0
    while t_in + (cnt + 0.5) * dt < t_out:
        p = o + (t_in + (cnt + 0.5) * dt) * d
        u = [p[a] - 0.5 for a in range(3)]
        i0 = [math.floor(x) for x in u]
        f = [u[a] - i0[a] for a in range(3)]
        val = 0.0
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    w = (f[0] if cx else 1 - f[0]) * (f[1] if cy else 1 - f[1]) * (f[2] if cz else 1 - f[2])
                    x = min(max(i0[0] + cx, 0), nx - 1)
                    y = min(max(i0[1] + cy, 0), ny - 1)
                    z = min(max(i0[2] + cz, 0), nz - 1)
                    val += w * float(vol[z, y, x])
        best = max(best, val)
        cnt += 1
    return (best if cnt else None), cnt


@pytest.mark.parametrize("kind", ["persp", "ortho"])
@pytest.mark.parametrize("step", [0.37, "voxel"])
def test_bricked_and_full_match_brute_force(kind, step):
    rng = np.random.default_rng(11)
    dims = (9, 7, 8)
    vol = rng.normal(size=dims[::-1]).astype(np.float32)
    tf = _identity_map(-3.0, 3.0)
    v = synth.orbit_view(dims, 13, kind=kind, width=20, height=16)
    cam = _cam(v)
    bricks = rc.brick_grid(dims, (4, 3, 5))
    stored = rc.store_bricks(vol, bricks, "f32")
    full = mip.render_mip_full(vol, cam, tf, step)
    br = mip.render_mip_bricked(stored, dims, cam, tf, step)
    n_hit = n_tie = 0
    for r in range(v.width * v.height):
        px, py = r % v.width, r // v.width
        m, cnt = _brute_mip_ray(vol, cam, step, px, py)
        if r in br.branches:
            # a near-tie ray: the brute force takes one of its listed results
            exp = np.zeros(4) if m is None else mip.colour_map(tf, np.array([m]))[0]
            assert min(np.max(np.abs(a - exp)) for a in br.branches[r]) < 1e-12
            n_tie += 1
            continue
        assert full.samples[r] == cnt and br.samples[r] == cnt
        if m is None:
            assert np.all(full.image[r] == 0) and np.all(br.image[r] == 0)
            continue
        n_hit += 1
        assert abs(full.vmax[r] - m) < 1e-12
        assert abs(br.vmax[r] - m) < 1e-12
        assert abs(br.image[r, 0] - min(max((m + 3.0) / 6.0, 0.0), 1.0)) < 1e-12
    assert n_hit > 50


def test_brick_maxima_merge_in_any_order():
    """Per-brick maxima folded in a shuffled order give the merged result; the
    merged maximum equals the unbricked one exactly for shared FP32 values."""
    rng = np.random.default_rng(12)
    dims = (12, 10, 9)
    vol = rng.normal(size=dims[::-1]).astype(np.float32)
    tf = _identity_map(-3.0, 3.0)
    cam = _cam(synth.orbit_view(dims, 7, width=24, height=18))
    bricks = rc.brick_grid(dims, (5, 4, 4))
    stored = rc.store_bricks(vol, bricks, "f32")
    br = mip.render_mip_bricked(stored, dims, cam, tf, 0.5, want_subimages=True)
    full = mip.render_mip_full(vol, cam, tf, 0.5)
    keys = list(br.subimages)
    rng.shuffle(keys)
    m = np.full(len(br.vmax), -np.inf)
    for k in keys:
        m = np.maximum(m, br.subimages[k])
    assert np.array_equal(m, br.vmax)
    ok = ~br.tie
    assert np.array_equal(br.vmax[ok], full.vmax[ok])


def test_colour_map_is_straight_entries_and_background_is_clear():
    """The colour map interpolates the given entries (no opacity correction,
    no premultiplication); rays without samples stay (0, 0, 0, 0)."""
    K = 5
    rgba = np.array([[0.1, 0.2, 0.3, 0.0], [0.5, 0.5, 0.5, 0.2], [0.9, 0.1, 0.4, 0.6],
                     [0.2, 0.8, 0.6, 0.9], [1.0, 1.0, 1.0, 1.0]], np.float32)
    tf = rc.TransferFunction(rgba, 0.0, 4.0)
    vals = np.array([-1.0, 0.0, 0.5, 1.0, 2.25, 4.0, 9.0])
    out = mip.colour_map(tf, vals)
    for c in range(4):
        assert np.allclose(out[:, c], np.interp(vals, np.arange(K), rgba[:, c].astype(np.float64)), atol=1e-7)
    dims = (6, 6, 6)
    vol = np.ones(dims[::-1], np.float32)
    cam = _cam(synth.orbit_view(dims, 0, width=40, height=30, fovy_deg=60.0))
    res = mip.render_mip_full(vol, cam, tf, 0.5)
    miss = res.samples == 0
    assert miss.any() and (~miss).any()
    assert np.all(res.image[miss] == 0)
    assert np.allclose(res.image[~miss], np.asarray(rgba[1], np.float64), atol=1e-7)


def test_fp8_bricks_decode_with_their_own_quantisation():
    """FP8 storage: each brick's maximum comes from its own decoded codes, so
    the merged projection differs from the FP32 one by at most the largest
    per-brick quantisation step on the values it takes."""
    rng = np.random.default_rng(13)
    dims = (10, 9, 8)
    vol = rng.normal(size=dims[::-1]).astype(np.float32) * 2.0
    tf = _identity_map(-8.0, 8.0)
    cam = _cam(synth.orbit_view(dims, 9, width=20, height=16))
    bricks = rc.brick_grid(dims, (5, 5, 4))
    s8 = rc.store_bricks(vol, bricks, "fp8")
    s32 = rc.store_bricks(vol, bricks, "f32")
    a = mip.render_mip_bricked(s8, dims, cam, tf, 0.5)
    b = mip.render_mip_bricked(s32, dims, cam, tf, 0.5)
    hit = b.samples > 0
    # e4m3 keeps 3 mantissa bits: relative step 1/8 of the code's binade,
    # at most 32 of 896 scale units at the largest codes
    bound = max(sb.scale for sb in s8) * 32.0
    assert np.max(np.abs(a.vmax[hit] - b.vmax[hit])) <= bound
    assert np.max(np.abs(a.vmax[hit] - b.vmax[hit])) > 0.0


def test_sample_on_a_face_between_fp8_bricks_lists_both_maxima():
    """A sample lands exactly on the face z = 3 between two FP8 bricks with
    different scale and offset, and it is the largest of the ray.  The ray's
    results are the colour map of its value decoded from either brick (codes
    worked out by hand from the E4M3 grid) and nothing else."""
    dims = (2, 2, 6)
    zcol = np.array([0.0, 1.0, 3.0, 2.0, 0.5, 0.25], np.float32)
    vol = np.broadcast_to(zcol[:, None, None], (6, 2, 2)).astype(np.float32)
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (2, 2, 3)), "fp8")
    a, b = stored
    assert [float(rc._E4M3_LUT[c]) for c in a.codes[:, 0, 0]] == [-448.0, -448.0, -144.0, 448.0, 144.0]
    assert [float(rc._E4M3_LUT[c]) for c in b.codes[:, 0, 0]] == [448.0, 120.0, -352.0, -448.0, -448.0]
    v3a = 0.5 * ((448.0 * a.scale + a.offset) + (144.0 * a.scale + a.offset))
    v3b = 0.5 * ((120.0 * b.scale + b.offset) + (448.0 * b.scale + b.offset))
    v5 = 0.5 * ((-352.0 * b.scale + b.offset) + (-448.0 * b.scale + b.offset))
    assert abs(v3a - v3b) > 1e-3 and v5 < min(v3a, v3b)
    tf = _identity_map(0.0, 4.0)
    cam = _cam(synth.axis_view(dims, "z", 2, 2, step=2.0))
    res = mip.render_mip_bricked(stored, dims, cam, tf, 2.0)
    assert res.tie.all()
    for r in range(4):
        reds = sorted(float(x[0]) for x in res.branches[r])
        assert len(reds) == 2
        assert abs(reds[0] - min(v3a, v3b) / 4.0) < 1e-12 and abs(reds[1] - max(v3a, v3b) / 4.0) < 1e-12
        # the FP64 default: the half-open box puts z = 3 in brick 1
        assert abs(res.image[r, 0] - v3b / 4.0) < 1e-12
