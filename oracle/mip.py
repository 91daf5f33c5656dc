"""FP64 reference for maximum intensity projection (TEST INFRASTRUCTURE ONLY --
see oracle/__init__).

The paper's adopted operator (Section 2.3.3): each ray keeps the largest data
value it samples; because the maximum is associative and commutative the
per-brick results merge in any order; the colour map is applied once, after
the merge.  Its early termination at the data maximum (Section 2.3.2) cannot
change the maximum, so this reference does not model it.

Readings used here besides C0-C6 of ``oracle.raycast`` (the same rays, clipping,
sample anchoring at the cube entry, trilinear values and bricks):

M1  The colour map is the K straight RGBA entries given for the transfer
    function, interpolated linearly over [vmin, vmax] and clamped (C4 without
    the opacity correction and premultiplication, which only compositing
    needs).
M2  A pixel whose ray takes no sample is transparent black (0, 0, 0, 0); any
    other pixel is colourmap(max).
M3  Step policy "per voxel" (Section 2.3.2: at least one sample for each voxel
    the ray crosses, by discrete ray casting): the ray's step is
    dt = 1 / max_a |d_a|, so consecutive samples advance exactly one voxel
    along the ray's dominant axis and at most one along the others.  The
    samples keep the C2 anchoring t_j = t_in + (j + 1/2) dt.
"""
from __future__ import annotations

import numpy as np

from . import raycast as rc


def per_voxel_step(d):
    """M3: one sample per voxel slice along each ray's dominant axis."""
    return 1.0 / np.max(np.abs(d), axis=-1)


def colour_map(tf: rc.TransferFunction, m):
    """M1: straight entries interpolated at value(s) m."""
    return tf.lookup(np.asarray(tf.rgba, dtype=np.float64), m)


def _steps(step, d):
    if isinstance(step, str):
        if step != "voxel":
            raise ValueError(step)
        return per_voxel_step(d)
    return np.full(d.shape[0], float(step))


class MipResult:
    def __init__(self, image, vmax, samples, tie, branches=None):
        self.image = image          # (R, 4) colour-mapped maximum (M2)
        self.vmax = vmax            # (R,) maximum sample value, -inf without samples
        self.samples = samples      # (R,) samples taken
        self.tie = tie              # (R,) a sample-membership decision was near its threshold
        self.branches = branches or {}


def _finish(tf, m, n):
    img = np.where((n > 0)[:, None], colour_map(tf, np.where(n > 0, m, tf.vmin)), 0.0)
    return img


def render_mip_full(vol, cam: rc.Camera, tf: rc.TransferFunction, step, pixels=None, chunk=2048):
    """Unbricked maximum intensity projection of the cube vol[z][y][x]."""
    px, py = rc._pixels(cam, pixels)
    R = len(px)
    dims = (vol.shape[2], vol.shape[1], vol.shape[0])
    m = np.full(R, -np.inf)
    used = np.zeros(R, dtype=np.int64)
    tie = np.zeros(R, dtype=bool)
    for s, e in rc._chunks(R, chunk):
        o, d = cam.rays(px[s:e], py[s:e])
        dt = _steps(step, d)
        t_in, t_out, hit = rc.global_interval(o, d, dims)
        n = rc.sample_count(t_in, t_out, dt, hit)
        used[s:e] = n
        last = t_in + (n - 0.5) * dt
        nxt = t_in + (n + 0.5) * dt
        tie[s:e] = hit & ((np.abs(last - t_out) < rc.DELTA_T) | (np.abs(nxt - t_out) < rc.DELTA_T))
        J = int(n.max()) if len(n) else 0
        if J == 0:
            continue
        j = np.arange(J)
        t = t_in[:, None] + (j[None, :] + 0.5) * dt[:, None]
        valid = j[None, :] < n[:, None]
        p = o[:, None, :] + np.where(valid, t, 0.0)[..., None] * d[:, None, :]
        v = rc.trilinear(vol, p)
        m[s:e] = np.max(np.where(valid, v, -np.inf), axis=1)
    return MipResult(_finish(tf, m, used), m, used, tie)


def render_mip_bricked(stored, dims, cam: rc.Camera, tf: rc.TransferFunction, step, pixels=None,
                       chunk=1024, want_subimages=False):
    """Per-brick maxima from each brick's stored values, merged with max in
    brick-index order (any order gives the same result), then colour-mapped
    (Sections 2.1, 2.3.2, 2.3.3)."""
    px, py = rc._pixels(cam, pixels)
    R = len(px)
    m = np.full(R, -np.inf)
    used = np.zeros(R, dtype=np.int64)
    tie = np.zeros(R, dtype=bool)
    subs = {sb.brick.index: np.full(R, -np.inf) for sb in stored} if want_subimages else None
    for s, e in rc._chunks(R, chunk):
        o, d = cam.rays(px[s:e], py[s:e])
        dt = _steps(step, d)
        t_in, t_out, hit = rc.global_interval(o, d, dims)
        n = rc.sample_count(t_in, t_out, dt, hit)
        last = t_in + (n - 0.5) * dt
        nxt = t_in + (n + 0.5) * dt
        tie[s:e] |= hit & ((np.abs(last - t_out) < rc.DELTA_T) | (np.abs(nxt - t_out) < rc.DELTA_T))
        for sb in stored:
            j0, j1, j0u, j1u, tb0, tb1, hit_b = rc._brick_sample_range(t_in, n, dt, o, d, sb.brick)
            for tb, cand in ((tb0, (j0u - 1, j0u)), (tb1, (j1u - 1, j1u))):
                for jj in cand:
                    tj = t_in + (jj + 0.5) * dt
                    with np.errstate(invalid="ignore"):
                        near = np.abs(tj - tb) < rc.DELTA_T
                    tie[s:e] |= hit_b & np.isfinite(tb) & (jj >= 0) & (jj < n) & near
            cnt = j1 - j0
            J = int(cnt.max()) if len(cnt) else 0
            if J == 0:
                continue
            k = np.arange(J)
            valid = k[None, :] < cnt[:, None]
            t = t_in[:, None] + (j0[:, None] + k[None, :] + 0.5) * dt[:, None]
            p = o[:, None, :] + np.where(valid, t, 0.0)[..., None] * d[:, None, :]
            pc = np.where(valid[..., None], p, np.asarray(sb.brick.lo) + 0.5)
            v = rc.trilinear(sb.values, pc, origin=sb.origin, decode=sb.decode)
            mb = np.max(np.where(valid, v, -np.inf), axis=1)
            if subs is not None:
                subs[sb.brick.index][s:e] = mb
            m[s:e] = np.maximum(m[s:e], mb)
            used[s:e] += cnt
    branches = {}
    for r in np.nonzero(tie)[0]:
        branches[int(r)] = mip_ray_branches(stored, dims, cam, tf, step, int(px[r]), int(py[r]))
    out = MipResult(_finish(tf, m, used), m, used, tie, branches)
    out.subimages = subs
    return out


def mip_ray_branches(stored, dims, cam, tf, step, px, py):
    """Colour-mapped results of one ray over its near-tie decisions: the last
    sample of the ray taken or not, and every sample near a brick face decoded
    with the stored values of any brick whose face it is near.  For a maximum
    the reachable results are exactly the candidate values that are not below
    the largest per-sample minimum, so they are listed without enumerating
    the combinations."""
    o, d = cam.rays(np.array([px]), np.array([py]))
    dt = float(_steps(step, d)[0])
    t_in, t_out, hit = rc.global_interval(o, d, dims)
    if not bool(hit[0]):
        return [np.zeros(4)]
    t_in, t_out = float(t_in[0]), float(t_out[0])
    n = int(rc.sample_count(np.array([t_in]), np.array([t_out]), dt, np.array([True]))[0])
    o1, d1 = o[0], d[0]
    # per sample: the values it can take (owner brick, and a neighbour across a near face)
    options = []
    for j in range(n + 1):
        tj = t_in + (j + 0.5) * dt
        p = o1 + tj * d1
        vals = []
        for sb in stored:
            br = sb.brick
            tb0, tb1 = rc.slab(o, d, tuple(float(x) for x in br.lo), tuple(float(x) for x in br.hi))
            tb0, tb1 = float(tb0[0]), float(tb1[0])
            if not tb0 < tb1:
                continue
            inside = tb0 <= tj < tb1
            near = abs(tj - tb0) < rc.DELTA_T or abs(tj - tb1) < rc.DELTA_T
            if inside or near:
                vals.append(float(rc.trilinear(sb.values, p[None, :], origin=sb.origin, decode=sb.decode)[0]))
        options.append(vals)
    exit_near = [jj for jj in (n - 1, n) if jj >= 0 and abs(t_in + (jj + 0.5) * dt - t_out) < rc.DELTA_T]
    counts = {n} | {jj for jj in exit_near} | {jj + 1 for jj in exit_near}
    out = []
    for cnt in sorted(counts):
        opts = [v for v in options[:cnt] if v]
        if cnt <= 0 or not opts:
            out.append(np.zeros(4))
            continue
        # the maxima reachable by some choice per sample: every option value
        # at or above the largest per-sample minimum
        lo = max(min(v) for v in opts)
        reach = sorted({x for v in opts for x in v if x >= lo})
        out.extend(colour_map(tf, np.array(reach)))
    return out


def max_abs_with_branches(gpu, res: MipResult):
    """Per-pixel max |gpu - oracle|, for near-tie rays the closest branch."""
    err = np.max(np.abs(gpu - res.image), axis=1)
    for r, alts in res.branches.items():
        if alts:
            err[r] = min(err[r], min(float(np.max(np.abs(gpu[r] - a))) for a in alts))
    return err
