"""Pins for the FP64 ray-casting oracle: closed forms, a textbook special case,
brute force with an independent formulation, invariants and bounds.  None of
these re-types the oracle's own code path."""
import math

import numpy as np
import pytest

from oracle import raycast as rc
from paper_1205_0282_amd import synth


def _cam(v: synth.ViewSpec):
    return rc.Camera(v.modelview, v.projection, v.width, v.height)


def _const_tf(rgba, K=8, vmin=-1.0, vmax=1.0):
    return rc.TransferFunction(np.tile(np.asarray(rgba, np.float32), (K, 1)), vmin, vmax)


# ------------------------------------------------------------------- camera
def test_camera_unprojects_through_pixel_centres():
    """Points on each ray project back (P M) onto the pixel's NDC centre."""
    for kind in ("persp", "ortho"):
        v = synth.orbit_view((40, 30, 20), 5, kind=kind, width=64, height=48)
        cam = _cam(v)
        M, P = rc.mat_from_col_major(v.modelview), rc.mat_from_col_major(v.projection)
        py, px = np.mgrid[0:48:7, 0:64:5]
        px, py = px.ravel(), py.ravel()
        o, d = cam.rays(px, py)
        x, y = (2 * px + 1) / 64 - 1, 1 - (2 * py + 1) / 48
        for t in (3.0, 50.0):
            q = np.concatenate([o + t * d, np.ones((len(px), 1))], axis=1) @ (P @ M).T
            ndc = q[:, :3] / q[:, 3:4]
            assert np.allclose(ndc[:, 0], x, atol=1e-12) and np.allclose(ndc[:, 1], y, atol=1e-12)
        assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)


def test_camera_eye_and_direction():
    dims = (40, 30, 20)
    v = synth.orbit_view(dims, 9, kind="persp", width=32, height=32)
    cam = _cam(v)
    n = np.asarray(dims, float)
    R = 0.5 * np.linalg.norm(n)
    D = R / math.sin(math.radians(15))
    az, el = 2 * math.pi * 9 / 64, math.radians(20)
    eye = n / 2 + D * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    assert np.allclose(cam.eye, eye, atol=1e-10)
    o, d = cam.rays(np.array([0, 31]), np.array([0, 31]))
    assert np.allclose(o, eye, atol=1e-10)
    vo = synth.orbit_view(dims, 9, kind="ortho", width=32, height=32)
    camo = _cam(vo)
    fwd = (n / 2 - eye) / np.linalg.norm(n / 2 - eye)
    assert np.allclose(camo.view_dir, fwd, atol=1e-12)
    _, do = camo.rays(np.array([3, 20]), np.array([7, 1]))
    assert np.allclose(do, fwd[None, :], atol=1e-12)


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("dt", [0.5, 0.25, 1.0])
def test_constant_density_opacity(dt):
    """v == c0 everywhere: opacity after a chord of length L is
    1 - (1 - a)^(n dt / dt_ref) with n = #{j : (j+1/2) dt < L}; colour = rgb * A."""
    dims = (12, 10, 16)
    vol = np.full(dims[::-1], 0.3, dtype=np.float32)
    rgba = (0.9, 0.4, 0.2, 0.35)
    tf = _const_tf(rgba)
    v = synth.axis_view(dims, "z", 12, 10, step=dt, ert=1.0)
    cam = _cam(v)
    res = rc.render_full(vol, cam, tf, dt, 1.0)
    L = dims[2]
    n = math.ceil(L / dt - 0.5)
    A = 1 - (1 - rgba[3]) ** (n * dt)
    exp = np.array([rgba[0] * A, rgba[1] * A, rgba[2] * A, A])
    assert np.allclose(res.image, exp[None, :], atol=1e-12)
    assert np.all(res.samples == n)


def test_constant_density_oblique_chord():
    """Oblique orthographic rays: n from the analytic chord length of each ray."""
    dims = (16, 16, 16)
    vol = np.full(dims[::-1], -0.2, dtype=np.float32)
    rgba = (0.5, 0.6, 0.7, 0.2)
    tf = _const_tf(rgba)
    v = synth.orbit_view(dims, 3, kind="ortho", width=24, height=24, elevation_deg=31.0)
    cam = _cam(v)
    dt = 0.5
    res = rc.render_full(vol, cam, tf, dt, 1.0)
    py, px = np.mgrid[0:24, 0:24]
    o, d = cam.rays(px.ravel(), py.ravel())
    # chord by brute geometry: clip the line against the six planes (independent of slab())
    lo_t, hi_t = np.zeros(len(o)), np.full(len(o), np.inf)
    for a in range(3):
        ta = (0 - o[:, a]) / d[:, a]
        tb = (16 - o[:, a]) / d[:, a]
        lo_t = np.maximum(lo_t, np.minimum(ta, tb))
        hi_t = np.minimum(hi_t, np.maximum(ta, tb))
    L = np.maximum(hi_t - lo_t, 0)
    n = np.where(L > 0, np.ceil(L / dt - 0.5), 0)
    A = 1 - (1 - rgba[3]) ** (n * dt)
    assert np.allclose(res.image[:, 3], A, atol=1e-12)
    assert np.allclose(res.image[:, :3], np.asarray(rgba[:3])[None, :] * A[:, None], atol=1e-12)


def test_constant_density_early_termination():
    dims = (8, 8, 40)
    vol = np.full(dims[::-1], 0.0, dtype=np.float32)
    rgba = (1.0, 1.0, 1.0, 0.3)
    tf = _const_tf(rgba)
    dt, tau = 0.5, 0.9
    cam = _cam(synth.axis_view(dims, "z", 8, 8, step=dt, ert=tau))
    res = rc.render_full(vol, cam, tf, dt, tau)
    a1 = 1 - (1 - 0.3) ** dt
    m = next(m for m in range(1, 1000) if 1 - (1 - a1) ** m >= tau)
    A = 1 - (1 - a1) ** m
    assert np.allclose(res.image[:, 3], A, atol=1e-12)
    assert np.all(res.samples == m)


def test_linear_ramp_axis_view_closed_form():
    """v = a + b z (voxel centres), view straight down z, constant opacity and
    colour linear in v: C = sum_j a'(1-a')^j (c0 + c1 v_j), v_j linear in j in
    the interior and clamped flat in the first and last half voxel."""
    nx, ny, nz = 6, 5, 20
    a, b = -2.0, 0.25
    z = np.arange(nz) + 0.5
    vol = np.broadcast_to((a + b * z)[:, None, None], (nz, ny, nx)).astype(np.float32).copy()
    vmin, vmax = a, a + b * nz
    K = 33
    vk = vmin + np.arange(K) / (K - 1) * (vmax - vmin)
    c0, c1 = 0.1, 0.05
    col = np.clip(c0 + c1 * vk, 0, 1)
    assert np.all((c0 + c1 * vk >= 0) & (c0 + c1 * vk <= 1))
    alpha = 0.15
    rgba = np.stack([col, col, col, np.full(K, alpha)], axis=1).astype(np.float32)
    tf = rc.TransferFunction(rgba, vmin, vmax)
    dt = 0.5
    cam = _cam(synth.axis_view((nx, ny, nz), "z", nx, ny, step=dt, ert=1.0))
    res = rc.render_full(vol, cam, tf, dt, 1.0)
    ap = 1 - (1 - alpha) ** dt
    q = 1 - ap
    n = 2 * nz
    zj = (np.arange(n) + 0.5) * dt
    # closed form: first and last sample clamped; interior samples j=1..n-2 linear
    v_first, v_last = a + b * 0.5, a + b * (nz - 0.5)
    # sum over j=1..n-2 of q^j (c0 + c1 (a + b z_j)), z_j = (j + 1/2) dt
    m0, m1 = 1, n - 2
    S0 = (q ** m0 - q ** (m1 + 1)) / (1 - q)
    def sjq(k):  # sum_{j=0}^{k} j q^j
        return q * (1 - (k + 1) * q ** k + k * q ** (k + 1)) / (1 - q) ** 2
    S1 = sjq(m1) - sjq(m0 - 1)
    inner = (c0 + c1 * (a + b * 0.5 * dt)) * S0 + c1 * b * dt * S1
    C = ap * ((c0 + c1 * v_first) + inner + q ** (n - 1) * (c0 + c1 * v_last))
    assert np.allclose(res.image[:, 0], C, atol=1e-12)
    assert np.allclose(res.image[:, 3], 1 - q ** n, atol=1e-12)
    assert zj[0] < 0.5 and zj[1] >= 0.5 and zj[-1] > nz - 0.5 and zj[-2] <= nz - 0.5


def test_textbook_voxel_centred_axis_view():
    """dt = 1, axis-aligned orthographic view with pixel centres on voxel
    centres: samples land on voxel centres and the image is the cumulative
    front-to-back composite of TF(V[:, y, x]) along z in product form."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 7, 6, 9
    vol = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    K = 16
    rgba = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    tf = rc.TransferFunction(rgba, -1.0, 1.0)
    cam = _cam(synth.axis_view((nx, ny, nz), "z", nx, ny, step=1.0, ert=1.0))
    o, _ = cam.rays(np.arange(nx), np.zeros(nx, int))
    assert np.allclose(o[:, 0], nx - np.arange(nx) - 0.5, atol=1e-12)   # px -> column nx-1-px
    res = rc.render_full(vol, cam, tf, 1.0, 1.0)
    img = res.image.reshape(ny, nx, 4)
    # independent table lookup: piecewise-linear interpolation of each channel
    x = np.linspace(-1.0, 1.0, K)
    a_corr = rgba[:, 3].astype(np.float64)  # dt == dt_ref: no correction
    for py in range(ny):
        for px in range(nx):
            col = vol[:, ny - 1 - py, nx - 1 - px].astype(np.float64)
            alpha = np.interp(col, x, a_corr)
            rgb = np.stack([np.interp(col, x, rgba[:, c] * a_corr) for c in range(3)], axis=1)
            trans = np.concatenate([[1.0], np.cumprod(1 - alpha)[:-1]])
            exp = np.concatenate([(rgb * trans[:, None]).sum(0), [(alpha * trans).sum()]])
            assert np.allclose(img[py, px], exp, atol=1e-12)


# --------------------------------------------------------------- brute force
def _brute_bricked_ray(vol, bricks, cam, tf, dt, tau, px, py):
    """Independent formulation: sample membership by point-in-box, explicit
    8-weight trilinear with clamped corners, transmittance products, bricks
    composited in the order of first visit along the ray."""
    o, d = cam.rays(np.array([px]), np.array([py]))
    o, d = o[0], d[0]
    nz, ny, nx = vol.shape
    # global chord from plane crossings
    ts = []
    for a, N in enumerate((nx, ny, nz)):
        if d[a] != 0:
            ts.append(sorted(((0 - o[a]) / d[a], (N - o[a]) / d[a])))
    t0 = max([0.0] + [t[0] for t in ts])
    t1 = min(t[1] for t in ts)
    if not t0 < t1:
        return np.zeros(4)
    K = tf.rgba.shape[0]
    base = tf.rgba.astype(np.float64)
    ac = 1 - (1 - base[:, 3]) ** (dt / tf.dt_ref)
    per_brick = {}
    first_seen = []
    j = 0
    while True:
        t = t0 + (j + 0.5) * dt
        if not t < t1:
            break
        p = o + t * d
        owner = None
        for b in bricks:
            if all(b.lo[a] <= p[a] < b.hi[a] for a in range(3)):
                owner = b.index
        if owner is None:   # on the far faces of the cube (closed): take the last brick containing it
            for b in bricks:
                if all(b.lo[a] <= p[a] <= b.hi[a] for a in range(3)):
                    owner = b.index
        u = p - 0.5
        i0 = np.floor(u).astype(int)
        f = u - i0
        val = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                    ix = min(max(i0[0] + dx, 0), nx - 1)
                    iy = min(max(i0[1] + dy, 0), ny - 1)
                    iz = min(max(i0[2] + dz, 0), nz - 1)
                    val += w * float(vol[iz, iy, ix])
        s = min(max((val - tf.vmin) / (tf.vmax - tf.vmin), 0.0), 1.0) * (K - 1)
        i = min(int(math.floor(s)), K - 2)
        fr = s - i
        a_s = (1 - fr) * ac[i] + fr * ac[i + 1]
        rgb = (1 - fr) * base[i, :3] * ac[i] + fr * base[i + 1, :3] * ac[i + 1]
        if owner not in per_brick:
            per_brick[owner] = []
            first_seen.append(owner)
        per_brick[owner].append((rgb, a_s))
        j += 1
    F_rgb, F_a = np.zeros(3), 0.0
    for b in first_seen:
        S_rgb, S_a, trans = np.zeros(3), 0.0, 1.0
        for rgb, a_s in per_brick[b]:
            S_rgb += trans * rgb
            S_a += trans * a_s
            trans *= 1 - a_s
            if S_a >= tau:
                break
        F_rgb += (1 - F_a) * S_rgb
        F_a += (1 - F_a) * S_a
    return np.concatenate([F_rgb, [F_a]])


@pytest.mark.parametrize("kind,brick,tau,frame", [
    ("persp", (3, 3, 3), 1.0, 5), ("persp", (3, 5, 2), 0.9, 17), ("ortho", (4, 3, 5), 0.8, 40),
    ("ortho", (8, 8, 8), 0.95, 11), ("persp", (5, 4, 3), 0.7, 29)])
def test_bricked_matches_brute_force_8cube(kind, brick, tau, frame):
    rng = np.random.default_rng(frame)
    dims = (8, 8, 8)
    vol = rng.uniform(-1, 1, dims[::-1]).astype(np.float32)
    tf = rc.TransferFunction(synth.random_tf(rng, 12, alpha_max=0.6), -1.0, 1.0)
    v = synth.orbit_view(dims, frame, kind=kind, width=20, height=16, elevation_deg=27.0)
    cam = _cam(v)
    bricks = rc.brick_grid(dims, brick)
    stored = rc.store_bricks(vol, bricks)
    dt = 0.37
    res = rc.render_bricked(stored, dims, cam, tf, dt, tau)
    k = 0
    n_tie = 0
    for py in range(16):
        for px in range(20):
            exp = _brute_bricked_ray(vol, bricks, cam, tf, dt, tau, px, py)
            if res.tie[k]:
                # the brute force takes one of the ray's enumerated results
                n_tie += 1
                assert not res.overflow[k]
                assert min(np.max(np.abs(a - exp)) for a in res.branches[k]) < 1e-12, (px, py)
            else:
                assert np.allclose(res.image[k], exp, atol=1e-12), (px, py)
            k += 1
    assert res.image[:, 3].max() > 0.3


def test_bricked_equals_unbricked_without_termination():
    """Sort-last of per-brick renders equals the unbricked render when early
    termination is off, for uneven bricks and several views."""
    rng = np.random.default_rng(5)
    dims = (19, 14, 11)
    vol = rng.standard_normal(dims[::-1]).astype(np.float32)
    tf = rc.TransferFunction(synth.random_tf(rng, 20, alpha_max=0.4), -3.0, 3.0)
    for kind, frame, brick in (("persp", 3, (5, 4, 4)), ("ortho", 22, (7, 7, 3)), ("persp", 50, (19, 14, 11))):
        cam = _cam(synth.orbit_view(dims, frame, kind=kind, width=40, height=30))
        full = rc.render_full(vol, cam, tf, 0.5, 1.0)
        stored = rc.store_bricks(vol, rc.brick_grid(dims, brick))
        br = rc.render_bricked(stored, dims, cam, tf, 0.5, 1.0)
        assert np.allclose(full.image, br.image, atol=1e-12)
        assert np.array_equal(full.samples, br.samples)


def test_single_brick_equals_unbricked_with_termination():
    rng = np.random.default_rng(6)
    dims = (10, 12, 9)
    vol = rng.standard_normal(dims[::-1]).astype(np.float32)
    tf = rc.TransferFunction(synth.random_tf(rng, 16, alpha_max=0.9), -3.0, 3.0)
    cam = _cam(synth.orbit_view(dims, 7, kind="persp", width=30, height=30))
    full = rc.render_full(vol, cam, tf, 0.5, 0.8)
    br = rc.render_bricked(rc.store_bricks(vol, rc.brick_grid(dims, dims)), dims, cam, tf, 0.5, 0.8)
    ok = ~(full.tie | br.tie)
    assert np.allclose(full.image[ok], br.image[ok], atol=1e-12)


def test_termination_bound_and_degenerate_tfs():
    rng = np.random.default_rng(7)
    dims = (16, 16, 16)
    vol = rng.standard_normal(dims[::-1]).astype(np.float32)
    cam = _cam(synth.orbit_view(dims, 12, kind="persp", width=32, height=24))
    tf = rc.TransferFunction(synth.random_tf(rng, 32, alpha_max=0.8), -3.0, 3.0)
    for tau in (0.5, 0.9, 0.99):
        a = rc.render_full(vol, cam, tf, 0.5, tau).image
        b = rc.render_full(vol, cam, tf, 0.5, 1.0).image
        assert np.all(np.abs(a - b) <= (1 - tau) + 1e-12)
    zero = rc.TransferFunction(np.concatenate([rng.uniform(0, 1, (8, 3)), np.zeros((8, 1))], 1).astype(np.float32), -3, 3)
    assert np.all(rc.render_full(vol, cam, zero, 0.5, 0.99).image == 0.0)
    one = rc.TransferFunction(np.array([[0.2, 0.4, 0.6, 1.0]] * 8, np.float32), -3, 3)
    img = rc.render_full(vol, cam, one, 0.5, 0.99)
    hit = img.samples > 0
    assert np.allclose(img.image[hit], [0.2, 0.4, 0.6, 1.0], atol=1e-15)
    assert np.all(img.samples[hit] == 1)


def test_opacity_correction_is_step_independent():
    """Opacity over a fixed chord does not depend on the step (constant density)."""
    dims = (4, 4, 6)
    vol = np.zeros(dims[::-1], np.float32)
    tf = _const_tf((0.3, 0.3, 0.3, 0.45))
    vals = []
    for dt in (1.0, 0.5, 0.25, 0.125):
        cam = _cam(synth.axis_view(dims, "z", 4, 4, step=dt))
        vals.append(rc.render_full(vol, cam, tf, dt, 1.0).image[0, 3])
    assert np.allclose(vals, 1 - (1 - 0.45) ** 6, atol=1e-12)


def test_over_is_associative():
    rng = np.random.default_rng(8)
    def rnd():
        a = rng.uniform(0, 1, (100, 1))
        return np.concatenate([rng.uniform(0, 1, (100, 3)) * a, a], 1)
    x, y, z = rnd(), rnd(), rnd()
    assert np.allclose(rc.over(rc.over(x, y), z), rc.over(x, rc.over(y, z)), atol=1e-15)


# -------------------------------------------------------- visibility order
@pytest.mark.parametrize("kind", ["persp", "ortho"])
def test_visibility_order_brute_force(kind):
    """Along every ray, the bricks met are met in increasing visibility rank,
    on grids with uneven edge bricks (the eye outside the cube)."""
    rng = np.random.default_rng(9)
    dims = (23, 17, 19)
    for trial in range(12):
        brick = tuple(int(x) for x in rng.integers(3, 9, 3))
        bricks = rc.brick_grid(dims, brick)
        v = synth.orbit_view(dims, int(rng.integers(0, 64)), kind=kind, width=24, height=24,
                             elevation_deg=float(rng.uniform(-60, 60)))
        cam = _cam(v)
        order, _ = rc.visibility_order(bricks, cam)
        rank = {b: r for r, b in enumerate(order)}
        py, px = np.mgrid[0:24, 0:24]
        o, d = cam.rays(px.ravel(), py.ravel())
        t_in, t_out, hit = rc.global_interval(o, d, dims)
        for r in np.nonzero(hit)[0]:
            ts = np.linspace(t_in[r], t_out[r], 400, endpoint=False)[1:]
            p = o[r] + ts[:, None] * d[r]
            bi = np.minimum((p // np.asarray(brick)).astype(int), (np.asarray(dims) - 1) // np.asarray(brick))
            nb = [(dims[a] + brick[a] - 1) // brick[a] for a in range(3)]
            lin = bi[:, 0] + nb[0] * (bi[:, 1] + nb[1] * bi[:, 2])
            seq = [int(lin[0])] + [int(x) for k, x in enumerate(lin[1:]) if x != lin[k]]
            ranks = [rank[b] for b in seq]
            assert ranks == sorted(ranks), (trial, r)


def test_centre_distance_order_fails_where_power_distance_holds():
    """With the eye just outside the cube, the centre-distance order is wrong
    for some rays through uneven bricks while the power-distance order holds
    for every ray (the reason for the power key)."""
    dims = np.array((8, 9, 7))
    brick = (6, 6, 6)
    bricks = rc.brick_grid(tuple(dims), brick)
    nb = [(dims[a] + brick[a] - 1) // brick[a] for a in range(3)]
    cen = {b.index: np.array([(b.lo[a] + b.hi[a]) / 2 for a in range(3)]) for b in bricks}
    rng = np.random.default_rng(10)
    bad_centre = 0
    for trial in range(60):
        while True:
            eye = rng.uniform(-3, dims + 3)
            if np.any((eye < 0) | (eye >= dims)):
                break
        key_c = {i: np.linalg.norm(c - eye) for i, c in cen.items()}
        key_p = {b.index: sum((eye[a] - b.lo[a]) * (eye[a] - b.hi[a]) for a in range(3)) for b in bricks}
        for _ in range(60):
            d = rng.uniform(0, dims) - eye
            d /= np.linalg.norm(d)
            p = eye + np.linspace(0, 40, 8000)[:, None] * d
            inside = np.all((p >= 0) & (p < dims), axis=1)
            bi = (p[inside] // np.asarray(brick)).astype(int)
            lin = bi[:, 0] + nb[0] * (bi[:, 1] + nb[1] * bi[:, 2])
            seq = [int(lin[0])] + [int(x) for k, x in enumerate(lin[1:]) if x != lin[k]]
            kp = [key_p[b] for b in seq]
            kc = [key_c[b] for b in seq]
            assert kp == sorted(kp)
            bad_centre += kc != sorted(kc)
    assert bad_centre > 0


# ----------------------------------------------------------- storage forms
def test_fp8_bricks_use_own_quantisation_and_fp16_is_exact_cast():
    rng = np.random.default_rng(11)
    dims = (9, 8, 7)
    vol = (rng.standard_normal(dims[::-1]) * 4).astype(np.float32)
    bricks = rc.brick_grid(dims, (5, 4, 4))
    s16 = rc.store_bricks(vol, bricks, "f16")
    s8 = rc.store_bricks(vol, bricks, "fp8")
    assert np.array_equal(s16[0].values, vol.astype(np.float16).astype(np.float32))
    for b in s8:
        g = rc.ghosted_region(vol, b.brick)
        dec = b.decode(b.codes)
        assert dec.shape == g.shape
        assert np.max(np.abs(dec - g)) <= (g.max() - g.min()) / 896 * 16 + 1e-9
        assert b.offset == np.float32((np.float32(g.min()) + np.float32(g.max())) / np.float32(2))
        assert b.origin == tuple(x - 1 for x in b.brick.lo)


def test_storing_only_crossed_bricks_keeps_the_sampled_pixels():
    """Storing only the bricks that the checked rays cross gives those pixels
    as storing every brick does (FP16: the brick's own ghosted region instead
    of the shared cube, so up to the rounding of the origin shift); a brick
    left out raises when a ray reads it."""
    rng = np.random.default_rng(21)
    dims = (20, 18, 16)
    vol = (rng.standard_normal(dims[::-1]) * 3).astype(np.float32)
    tf = rc.TransferFunction(synth.random_tf(rng, 16, alpha_max=0.4), -6.0, 6.0)
    cam = _cam(synth.orbit_view(dims, 7, kind="persp", width=24, height=20))
    bricks = rc.brick_grid(dims, (8, 8, 8))
    pix = np.array([[x, y] for x in range(9, 13) for y in range(8, 11)])
    o, d = cam.rays(pix[:, 0], pix[:, 1])
    crossed = set()
    for b in bricks:
        tb0, tb1 = rc.slab(o, d, tuple(float(x) for x in b.lo), tuple(float(x) for x in b.hi))
        if np.any(tb0 < tb1):
            crossed.add(b.index)
    assert 0 < len(crossed) < len(bricks)
    for storage in ("f16", "fp8"):
        full = rc.render_bricked(rc.store_bricks(vol, bricks, storage), dims, cam, tf, 0.5, 0.95, pixels=pix)
        part = rc.render_bricked(rc.store_bricks(vol, bricks, storage, only=crossed), dims, cam, tf, 0.5,
                                 0.95, pixels=pix)
        assert full.image[:, 3].max() > 0.05
        assert np.max(np.abs(full.image - part.image)) <= 1e-12
    with pytest.raises(RuntimeError, match="not stored"):
        rc.render_bricked(rc.store_bricks(vol, bricks, "fp8", only=set()), dims, cam, tf, 0.5, 0.95, pixels=pix)


def test_fp16_source_is_stored_without_a_copy_and_renders_as_its_float32_widening():
    rng = np.random.default_rng(22)
    dims = (12, 10, 9)
    v16 = (rng.standard_normal(dims[::-1]) * 3).astype(np.float16)
    bricks = rc.brick_grid(dims, (5, 4, 4))
    s16 = rc.store_bricks(v16, bricks)
    s32 = rc.store_bricks(v16.astype(np.float32), bricks)
    assert s16[0].values is v16
    tf = rc.TransferFunction(synth.random_tf(rng, 16, alpha_max=0.4), -6.0, 6.0)
    cam = _cam(synth.orbit_view(dims, 3, kind="persp", width=16, height=14))
    a = rc.render_bricked(s16, dims, cam, tf, 0.5, 0.95)
    b = rc.render_bricked(s32, dims, cam, tf, 0.5, 0.95)
    assert a.image[:, 3].max() > 0.05
    assert np.array_equal(a.image, b.image)


def test_branch_enumeration_consistent_with_vectorised_path():
    """Rays without near ties give one branch equal to the vectorised result;
    an exact exit tie gives two branches that differ by one sample."""
    rng = np.random.default_rng(12)
    dims = (8, 8, 8)
    vol = rng.uniform(-1, 1, dims[::-1]).astype(np.float32)
    tf = rc.TransferFunction(synth.random_tf(rng, 12, alpha_max=0.5), -1, 1)
    cam = _cam(synth.orbit_view(dims, 13, kind="persp", width=12, height=12))
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (3, 4, 5)))
    res = rc.render_bricked(stored, dims, cam, tf, 0.5, 0.9)
    for k in range(0, 144, 7):
        if res.tie[k]:
            continue
        br, ovf = rc.ray_branches(stored, dims, cam, tf, 0.5, 0.9, k % 12, k // 12)
        assert len(br) == 1 and not ovf
        assert np.allclose(br[0], res.image[k], atol=1e-12)
    # exit tie: axis view, (j + 1/2) dt == 8 for j = 7
    dt = 8 / 7.5
    cam2 = _cam(synth.axis_view(dims, "z", 8, 8, step=dt))
    st1 = rc.store_bricks(vol, rc.brick_grid(dims, dims))
    r2 = rc.render_bricked(st1, dims, cam2, tf, dt, 1.0)
    assert r2.tie.all()
    # the exit sample sits on the cube's far face: included or not, two distinct pixels
    for alts in r2.branches.values():
        distinct = {tuple(np.round(a, 14)) for a in alts}
        assert len(distinct) == 2


# ----------------------------------------------- near ties with known results
def _dyadic_tf(rgb, alpha, vmin=0.0, vmax=1.0, dt_ref=1.0):
    """Two entries over [vmin, vmax]: transparent black, then (rgb, alpha)."""
    rgba = np.array([[0.0, 0.0, 0.0, 0.0], list(rgb) + [alpha]], np.float32)
    return rc.TransferFunction(rgba, vmin, vmax, dt_ref)


def _alpha_set(results):
    return sorted({float(r[3]) for r in results})


def test_exact_termination_tie_two_bricks_closed_form():
    """A column of constant density with opacity 1/2 per sample and tau = 3/4:
    each brick's opacity reaches tau exactly (in binary) at its second sample.
    A brick may stop there (opacity 3/4) or one sample later (7/8), never
    elsewhere, so two bricks composite to exactly three distinct pixels,
    alpha 1 - 2^-4, 1 - 2^-5, 1 - 2^-6, each with colour rgb * alpha."""
    dims = (1, 1, 8)
    vol = np.ones(dims[::-1], np.float32)
    rgb = (0.75, 0.5, 0.25)
    tf = _dyadic_tf(rgb, 0.5)
    cam = _cam(synth.axis_view(dims, "z", 1, 1, step=1.0))
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (1, 1, 4)))
    res = rc.render_bricked(stored, dims, cam, tf, 1.0, 0.75)
    assert res.tie[0] and not res.overflow[0]
    assert res.image[0, 3] == 0.9375                       # the FP64 decisions: both bricks stop at 3/4
    alts = res.branches[0]
    assert _alpha_set(alts) == [1 - 2.0 ** -4, 1 - 2.0 ** -5, 1 - 2.0 ** -6]
    assert len(alts) == 3
    for a in alts:
        assert np.array_equal(a[:3], np.asarray(rgb) * a[3])


def test_termination_tie_over_a_long_transparent_run_is_enumerated_without_cap():
    """Opacity sits within the tie margin of tau across 148 transparent
    samples: every stop among them gives the same sub-image, so the ray has
    as many distinct results as the two-brick closed form (three), and the
    enumeration does not overflow."""
    dims = (1, 1, 400)
    col = np.zeros(400, np.float32)
    col[0:2] = 1.0
    col[150:] = 1.0
    vol = col.reshape(400, 1, 1)
    tf = _dyadic_tf((0.75, 0.5, 0.25), 0.5)
    tau = 0.75 + 2.0 ** -15
    cam = _cam(synth.axis_view(dims, "z", 1, 1, step=1.0))
    stored = rc.store_bricks(vol, rc.brick_grid(dims, (1, 1, 200)))
    res = rc.render_bricked(stored, dims, cam, tf, 1.0, tau)
    assert res.tie[0] and not res.overflow[0]
    # FP64: brick 0 never reaches tau before sample 150 (opacity 7/8), brick 1 at its third sample
    assert res.image[0, 3] == 0.875 + 0.125 * 0.875
    alts, ovf = rc.ray_branches(stored, dims, cam, tf, 1.0, tau, 0, 0)
    assert not ovf
    assert _alpha_set(alts) == [1 - 2.0 ** -4, 1 - 2.0 ** -5, 1 - 2.0 ** -6]


def test_sample_on_a_face_between_fp8_bricks_closed_form():
    """A sample lands exactly on the face z = 3 between two FP8 bricks with
    different scale and offset.  It belongs to either brick; its value is the
    mean of voxels 2 and 3 decoded with that brick's codes, scale and offset
    (codes worked out by hand from the E4M3 grid).  The ray has exactly the
    two results composited from those values."""
    dims = (2, 2, 6)
    zcol = np.array([0.0, 1.0, 3.0, 2.0, 0.5, 0.25], np.float32)
    vol = np.broadcast_to(zcol[:, None, None], (6, 2, 2)).astype(np.float32)
    bricks = rc.brick_grid(dims, (2, 2, 3))
    stored = rc.store_bricks(vol, bricks, "fp8")
    a, b = stored
    # brick 0 stores z = 0, 0, 1, 2, 3 (ghost below clamps): min 0, max 3;
    # brick 1 stores z = 2, 3, 4, 5, 5: min 0.25, max 3
    assert a.offset == 1.5 and a.scale == float(np.float32(np.float32(3.0) / np.float32(896.0)))
    assert b.offset == 1.625 and b.scale == float(np.float32(np.float32(2.75) / np.float32(896.0)))
    # codes: (v - o) / s on the E4M3 grid (binades [64, 128), [128, 256), [256, 448] have steps 8, 16, 32)
    assert [float(rc._E4M3_LUT[c]) for c in a.codes[:, 0, 0]] == [-448.0, -448.0, -144.0, 448.0, 144.0]
    assert [float(rc._E4M3_LUT[c]) for c in b.codes[:, 0, 0]] == [448.0, 120.0, -352.0, -448.0, -448.0]
    dec_a = lambda q: q * a.scale + a.offset
    dec_b = lambda q: q * b.scale + b.offset
    v1 = 0.5 * (dec_a(-448.0) + dec_a(-144.0))          # sample z = 1, brick 0
    v3 = {"a": 0.5 * (dec_a(448.0) + dec_a(144.0)),      # sample z = 3 in brick 0 (voxel 3 = its ghost)
          "b": 0.5 * (dec_b(120.0) + dec_b(448.0))}      # ... in brick 1 (voxel 2 = its ghost)
    v5 = 0.5 * (dec_b(-352.0) + dec_b(-448.0))           # sample z = 5, brick 1
    assert abs(v3["a"] - v3["b"]) > 1e-3
    rgb = np.array([1.0, 0.5, 0.25])
    tf = _dyadic_tf(rgb, 0.75, vmin=0.0, vmax=4.0, dt_ref=2.0)
    expected = []
    for k in ("a", "b"):
        al = [0.75 * v / 4.0 for v in (v1, v3[k], v5)]
        A = al[0] + (1 - al[0]) * al[1] + (1 - al[0]) * (1 - al[1]) * al[2]
        expected.append(np.concatenate([rgb * A, [A]]))
    cam = _cam(synth.axis_view(dims, "z", 2, 2, step=2.0))
    res = rc.render_bricked(stored, dims, cam, tf, 2.0, 1.0)
    assert res.tie.all() and not res.overflow.any()
    for r in range(4):
        alts = res.branches[r]
        assert len(alts) == 2
        for e in expected:
            assert min(np.max(np.abs(x - e)) for x in alts) < 1e-12
        # the FP64 default: the half-open box puts z = 3 in brick 1
        assert np.max(np.abs(res.image[r] - expected[1])) < 1e-12


def test_psnr_peak_one_decibels_base_ten():
    """PSNR = 10 log10(1 / MSE) with peak 1 over every pixel and channel."""
    a = np.zeros((10, 10, 4))
    b = a.copy()
    b[3, 4, 2] = 0.4                                      # MSE = 0.16 / 400 = 4e-4
    assert abs(rc.psnr(a, b) - (40.0 - 10.0 * math.log10(4.0))) < 1e-9
    b[:] = 0.01                                           # MSE = 1e-4 -> 40 dB
    assert abs(rc.psnr(a, b) - 40.0) < 1e-9
    assert abs(rc.psnr(np.zeros(8), np.full(8, 0.5)) - 10.0 * math.log10(4.0)) < 1e-12   # 6.02 dB
    assert rc.psnr(np.zeros(8), np.ones(8)) == 0.0
    assert rc.psnr(b, b) == math.inf
