"""FP64 reference ray caster (TEST INFRASTRUCTURE ONLY -- see oracle/__init__).

Plain, slow and single-threaded per ray batch; numpy float64 throughout.  It
follows the paper's ray casting (Sections 1.2, 2.1 and 2.3.2), its rendering
rectangle (Section 2.3.2, Figure 4), its compositing of independently rendered
sub-volumes and the associativity of alpha blending (Section 2.3.3), bricking
(Section 2.1) and the data minimum/maximum (Section 2.3.1).  Where the paper is
silent the readings below are used (they are listed again in the design notes):

C0  World space is the texel space of the global cube: voxel (i, j, k) has its
    centre at (i+1/2, j+1/2, k+1/2); the cube is [0,Nx] x [0,Ny] x [0,Nz];
    memory order is data[z][y][x].  Membership in boxes is half-open.
    Pixel (px, py), row 0 at the top: x = (2px+1)/W - 1, y = 1 - (2py+1)/H.
    The modelview must be rigid [R t; 0 1]; the eye is -R^T t evaluated as
    e_a = -((R0a t0 + R1a t1) + R2a t2).  Perspective iff row 3 of the
    projection is (0, 0, -1, 0); orthographic iff it is (0, 0, 0, 1).
    Perspective ray: o = e, d = normalize(dehom((PM)^-1 (x, y, 1, 1)) - e).
    Orthographic ray: o = dehom((PM)^-1 (x, y, -1, 1)),
                      d = normalize(dehom((PM)^-1 (x, y, 1, 1)) - o).
C1  Global entry/exit by the slab test; t_in = max(0, max near), t_out = min far.
C2  Samples t_j = t_in + (j + 1/2) dt while t_j < t_out (anchored at the entry
    into the global cube, so every brick sees the same sample points).
C3  Trilinear interpolation of voxel values with corner indices clamped to the
    cube (clamp-to-edge texture addressing, Section 2.3.2).
C4  Transfer function: K straight RGBA entries over [vmin, vmax] with opacity
    given per dt_ref voxels; the table is opacity-corrected and premultiplied
    entry by entry (a' = 1 - (1 - a)^(dt/dt_ref)) and then interpolated
    linearly between neighbouring entries, clamped at both ends.
C5  Front-to-back "over": C <- C + (1 - C_a) c; stop when C_a >= tau.
C6  Bricks: box [b*B, min((b+1)*B, N)) per axis, linear index
    bx + nbx*(by + nby*bz); a brick owns samples with t_in_b <= t_j < t_out_b
    and composites them from zero with its own early termination; its values
    come from the brick's own ghosted copy (1-voxel ghosts, clamp-replicated at
    cube faces).
C7  Visibility order (not needed by the paper's MIP): ascending (key, index)
    with the power distance key sum_a (e_a - lo_a)(e_a - hi_a) for perspective
    and sum_a centre_a d_a for orthographic views, FP64 without FMA.
C8  Sort-last: F <- F + (1 - F_a) S_b over bricks in visibility order.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

from . import encoders

# near-tie margins for discontinuous decisions (sample count, brick ownership,
# early termination): rays with a decision closer than this to its threshold
# get every branch evaluated.
DELTA_T = 1e-6
DELTA_ALPHA = 1e-4
MAX_CONFIGS = 256        # sample-membership configurations of one ray
MAX_BRANCHES = 1 << 14   # distinct results of one ray


# ---------------------------------------------------------------------- camera
def mat_from_col_major(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64).reshape(4, 4)
    return a.T.copy()


@dataclass
class Camera:
    """Rays of one rendering request: frame size plus OpenGL projection and
    modelview matrices (Section 2.3.2)."""
    modelview: np.ndarray
    projection: np.ndarray
    width: int
    height: int
    kind: str = field(init=False)
    inv_pm: np.ndarray = field(init=False)
    eye: tuple = field(init=False)
    view_dir: tuple = field(init=False)

    def __post_init__(self):
        M = mat_from_col_major(self.modelview)
        P = mat_from_col_major(self.projection)
        row3 = P[3]
        if np.array_equal(row3, [0.0, 0.0, -1.0, 0.0]):
            self.kind = "persp"
        elif np.array_equal(row3, [0.0, 0.0, 0.0, 1.0]):
            self.kind = "ortho"
        else:
            raise ValueError("projection is neither perspective nor orthographic")
        self.inv_pm = np.linalg.inv(P @ M)
        R = [[float(M[r, c]) for c in range(3)] for r in range(3)]
        t = [float(M[r, 3]) for r in range(3)]
        self.eye = tuple(-((R[0][a] * t[0] + R[1][a] * t[1]) + R[2][a] * t[2]) for a in range(3))
        self.view_dir = (-R[2][0], -R[2][1], -R[2][2])

    def ndc(self, px, py):
        px = np.asarray(px, dtype=np.float64)
        py = np.asarray(py, dtype=np.float64)
        return (2.0 * px + 1.0) / self.width - 1.0, 1.0 - (2.0 * py + 1.0) / self.height

    def _unproject(self, x, y, z):
        v = np.stack([x, y, np.full_like(x, z), np.ones_like(x)], axis=-1) @ self.inv_pm.T
        return v[..., :3] / v[..., 3:4]

    def rays(self, px, py):
        """(o, d) with d of unit length, FP64, for pixel arrays."""
        x, y = self.ndc(px, py)
        far = self._unproject(x, y, 1.0)
        if self.kind == "persp":
            o = np.broadcast_to(np.asarray(self.eye), far.shape).copy()
        else:
            o = self._unproject(x, y, -1.0)
        d = far - o
        d = d / np.linalg.norm(d, axis=-1, keepdims=True)
        return o, d


# ------------------------------------------------------------------ slab test
def slab(o, d, lo, hi):
    """Entry/exit parameters of rays against the box [lo, hi] (per-axis slabs).
    Returns (t_near, t_far); a ray parallel to an axis outside the slab gets
    t_near = +inf."""
    n = o.shape[0]
    t_near = np.full(n, -np.inf)
    t_far = np.full(n, np.inf)
    for a in range(3):
        da = d[:, a]
        oa = o[:, a]
        par = da == 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (lo[a] - oa) / da
            t1 = (hi[a] - oa) / da
        near = np.where(par, np.where((oa >= lo[a]) & (oa < hi[a]), -np.inf, np.inf), np.minimum(t0, t1))
        far = np.where(par, np.where((oa >= lo[a]) & (oa < hi[a]), np.inf, -np.inf), np.maximum(t0, t1))
        t_near = np.maximum(t_near, near)
        t_far = np.minimum(t_far, far)
    return t_near, t_far


def global_interval(o, d, dims):
    t_near, t_far = slab(o, d, (0.0, 0.0, 0.0), tuple(float(x) for x in dims))
    t_in = np.maximum(0.0, t_near)
    hit = t_in < t_far
    return t_in, t_far, hit


def first_index_at_or_after(t_in, dt, t):
    """Smallest j >= 0 with t_in + (j + 1/2) dt >= t (C2 sample times)."""
    j = np.ceil((t - t_in) / dt - 0.5)
    j = np.maximum(j, 0.0)
    j = np.where(np.isfinite(j), j, 0.0)
    # exact fix-up against the sample-time formula
    tj = t_in + (j + 0.5) * dt
    j = np.where(tj < t, j + 1, j)
    tjm = t_in + (j - 0.5) * dt
    j = np.where((j > 0) & (tjm >= t), j - 1, j)
    return j.astype(np.int64)


def sample_count(t_in, t_out, dt, hit):
    """n = #{j : t_j < t_out} (C2)."""
    n = first_index_at_or_after(t_in, dt, t_out)
    return np.where(hit, n, 0)


# ------------------------------------------------------------------ trilinear
def trilinear(vol, p, origin=(0, 0, 0), decode=None):
    """Trilinear value at positions p (..., 3) of the array vol[z][y][x] whose
    element [0,0,0] is voxel ``origin`` (its centre at origin + 1/2).  Corner
    indices are clamped to [0, n-1] of the array (C3).  ``decode`` maps the
    gathered stored elements to FP64 values (storage forms)."""
    nz, ny, nx = vol.shape
    u = p - 0.5 - np.asarray(origin, dtype=np.float64)
    i0 = np.floor(u)
    f = u - i0
    i0 = i0.astype(np.int64)
    lim = (nx, ny, nz)
    idx = []
    for a in range(3):
        lo = np.clip(i0[..., a], 0, lim[a] - 1)
        hi = np.clip(i0[..., a] + 1, 0, lim[a] - 1)
        idx.append((lo, hi))
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    v = 0.0
    for cz, wz in ((0, 1.0 - fz), (1, fz)):
        for cy, wy in ((0, 1.0 - fy), (1, fy)):
            for cx, wx in ((0, 1.0 - fx), (1, fx)):
                g = vol[idx[2][cz], idx[1][cy], idx[0][cx]]
                g = decode(g) if decode is not None else g.astype(np.float64)
                v = v + (wz * wy * wx) * g
    return v


# --------------------------------------------------------- transfer function
@dataclass
class TransferFunction:
    rgba: np.ndarray      # (K, 4) straight RGBA in [0, 1]
    vmin: float
    vmax: float
    dt_ref: float = 1.0

    def table(self, dt):
        """Opacity-corrected, premultiplied entries (C4)."""
        t = np.asarray(self.rgba, dtype=np.float64)
        a = 1.0 - (1.0 - t[:, 3]) ** (dt / self.dt_ref)
        return np.stack([a * t[:, 0], a * t[:, 1], a * t[:, 2], a], axis=1)

    def lookup(self, table, v):
        K = table.shape[0]
        s = np.clip((v - self.vmin) / (self.vmax - self.vmin), 0.0, 1.0)
        x = s * (K - 1)
        i = np.minimum(np.floor(x), K - 2).astype(np.int64)
        f = (x - i)[..., None]
        return (1.0 - f) * table[i] + f * table[i + 1]


# ---------------------------------------------------------------- compositing
def composite(colors, valid, tau):
    """Front-to-back over with early termination (C5).  colors (R, J, 4),
    valid (R, J).  Returns (C, n_used, tie) where n_used counts the samples
    composited and tie flags a termination decision within DELTA_ALPHA."""
    R, J = valid.shape
    cnt = valid.sum(axis=1)            # valid is a prefix mask per ray
    C = np.zeros((R, 4))
    active = np.ones(R, dtype=bool)
    used = np.zeros(R, dtype=np.int64)
    tie = np.zeros(R, dtype=bool)
    for j in range(J):
        m = active & valid[:, j]
        if not m.any():
            if not (active & (cnt > j)).any():
                break
            continue
        C[m] = C[m] + (1.0 - C[m, 3:4]) * colors[m, j]
        used[m] += 1
        ca = C[:, 3]
        tie |= m & (np.abs(ca - tau) < DELTA_ALPHA)
        active &= ~(m & (ca >= tau))
    return C, used, tie


def over(front, back):
    """front over back for premultiplied RGBA (C8)."""
    return front + (1.0 - front[..., 3:4]) * back


# -------------------------------------------------------------------- bricks
@dataclass
class Brick:
    index: int
    lo: tuple
    hi: tuple


def brick_grid(dims, brick_dims):
    nb = [(dims[a] + brick_dims[a] - 1) // brick_dims[a] for a in range(3)]
    out = []
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                lo = (bx * brick_dims[0], by * brick_dims[1], bz * brick_dims[2])
                hi = tuple(min(lo[a] + brick_dims[a], dims[a]) for a in range(3))
                out.append(Brick(bx + nb[0] * (by + nb[1] * bz), lo, hi))
    return out


def ghosted_region(vol, brick, ghost=1):
    """The brick's core plus ``ghost`` voxels per side, clamp-replicated at the
    cube faces; element [0,0,0] is voxel lo - ghost."""
    nz, ny, nx = vol.shape
    zs = np.clip(np.arange(brick.lo[2] - ghost, brick.hi[2] + ghost), 0, nz - 1)
    ys = np.clip(np.arange(brick.lo[1] - ghost, brick.hi[1] + ghost), 0, ny - 1)
    xs = np.clip(np.arange(brick.lo[0] - ghost, brick.hi[0] + ghost), 0, nx - 1)
    return vol[np.ix_(zs, ys, xs)]


@dataclass
class StoredBrick:
    """What one brick stores.  ``values`` is an array whose element [0,0,0] is
    voxel ``origin``; for FP32/FP16 storage every brick shares the (rounded)
    global cube, whose clamped edges are exactly the clamp-replicated ghosts;
    FP8 bricks hold their own ghosted codes, decoded with the brick's own
    scale and offset."""
    brick: Brick
    values: np.ndarray
    origin: tuple
    scale: float = 1.0
    offset: float = 0.0
    codes: np.ndarray | None = None

    def decode(self, g):
        if self.codes is None:
            return g.astype(np.float64)
        return _E4M3_LUT[g] * self.scale + self.offset


_E4M3_LUT = encoders.e4m3_value(np.arange(256))


class _NotStored:
    """Values of a brick left out of ``store_bricks(..., only=...)``: reading
    them is an error."""

    def __init__(self, index):
        self.index = index
        self.shape = (1, 1, 1)

    def __getitem__(self, key):
        raise RuntimeError(f"brick {self.index} was not stored (outside only=)")


def store_bricks(vol, bricks, storage="f32", ghost=1, only=None):
    """What each brick stores: f32 as given, f16 after an RNE cast, fp8 after
    per-brick affine e4m3 quantisation over its core + ghost values (ghosts
    carry the owning brick's quantisation).

    ``only``: if given, the indices of the bricks to store; every other brick
    holds values that raise when read (a large cube checked at a few rays
    needs only the bricks those rays cross).  f16 bricks are then stored as
    their own ghosted regions, which equal the shared cube wherever the
    brick's samples read it."""
    out = []
    if storage == "f32":
        # an FP16 source is kept as it is: its values widen exactly when
        # gathered, and a float32 copy of a large cube is not made
        shared = vol if isinstance(vol, np.ndarray) and vol.dtype == np.float16 else np.asarray(vol, dtype=np.float32)
        return [StoredBrick(b, shared, (0, 0, 0)) for b in bricks]
    if storage == "f16" and only is None:
        shared = encoders.f16_value(encoders.f16_bits(vol)).astype(np.float32)   # exact
        return [StoredBrick(b, shared, (0, 0, 0)) for b in bricks]
    if storage not in ("f16", "fp8"):
        raise ValueError(storage)
    for b in bricks:
        if only is not None and b.index not in only:
            out.append(StoredBrick(b, _NotStored(b.index), (0, 0, 0)))
            continue
        if storage == "f16":
            g = encoders.f16_value(encoders.f16_bits(ghosted_region(vol, b, ghost))).astype(np.float32)
            out.append(StoredBrick(b, g, tuple(int(x) - ghost for x in b.lo)))
            continue
        g = ghosted_region(vol, b, ghost).astype(np.float32)
        s, o = encoders.brick_scale_offset(float(g.min()), float(g.max()))
        codes = encoders.fp8_encode_brick(g, s, o)
        origin = tuple(int(x) - ghost for x in b.lo)
        out.append(StoredBrick(b, codes, origin, float(s), float(o), codes))
    return out


def visibility_order(bricks, cam: Camera):
    """Front-to-back brick order (C7): keys in FP64, evaluated left to right
    without fused multiply-add (plain Python floats)."""
    keys = []
    for b in bricks:
        if cam.kind == "persp":
            e = cam.eye
            k = 0.0
            for a in range(3):
                k = k + (e[a] - b.lo[a]) * (e[a] - b.hi[a])
        else:
            d = cam.view_dir
            k = 0.0
            for a in range(3):
                k = k + ((b.lo[a] + b.hi[a]) / 2.0) * d[a]
        keys.append((k, b.index))
    keys.sort()
    return [i for _, i in keys], {i: k for k, i in keys}


# ----------------------------------------------------------------- rendering
@dataclass
class RenderResult:
    image: np.ndarray                 # (R, 4) premultiplied RGBA per requested pixel
    tie: np.ndarray                   # (R,) a discontinuous decision was near its threshold
    branches: dict                    # ray index -> list of (4,) alternative results
    overflow: np.ndarray              # (R,) branch list incomplete (MAX_CONFIGS / MAX_BRANCHES exceeded)
    samples: np.ndarray               # (R,) samples composited (up to termination)
    order: list | None = None
    footprint: dict | None = None     # brick index -> bool (R,) (>= 1 sample in the brick)


def _pixels(cam, pixels):
    if pixels is None:
        py, px = np.mgrid[0:cam.height, 0:cam.width]
        return px.reshape(-1), py.reshape(-1)
    pixels = np.asarray(pixels, dtype=np.int64)
    return pixels[:, 0], pixels[:, 1]


def _chunks(n, size):
    for s in range(0, n, size):
        yield s, min(n, s + size)


def render_full(vol, cam: Camera, tf: TransferFunction, dt: float, tau: float,
                pixels=None, chunk=2048) -> RenderResult:
    """Unbricked render (R_full): one front-to-back pass per ray with global
    early termination."""
    px, py = _pixels(cam, pixels)
    R = len(px)
    table = tf.table(dt)
    img = np.zeros((R, 4))
    tie = np.zeros(R, dtype=bool)
    used = np.zeros(R, dtype=np.int64)
    dims = (vol.shape[2], vol.shape[1], vol.shape[0])
    for s, e in _chunks(R, chunk):
        o, d = cam.rays(px[s:e], py[s:e])
        t_in, t_out, hit = global_interval(o, d, dims)
        n = sample_count(t_in, t_out, dt, hit)
        J = int(n.max()) if len(n) else 0
        if J == 0:
            continue
        j = np.arange(J)
        t = t_in[:, None] + (j[None, :] + 0.5) * dt
        valid = j[None, :] < n[:, None]
        p = o[:, None, :] + np.where(valid, t, 0.0)[..., None] * d[:, None, :]
        v = trilinear(vol, p)
        c = tf.lookup(table, v)
        C, u, tt = composite(c, valid, tau)
        img[s:e], used[s:e] = C, u
        # exit decision margin
        last = t_in + (n - 0.5) * dt
        nxt = t_in + (n + 0.5) * dt
        tie[s:e] = tt | (hit & ((np.abs(last - t_out) < DELTA_T) | (np.abs(nxt - t_out) < DELTA_T)))
    return RenderResult(img, tie, {}, np.zeros(R, dtype=bool), used)


def _brick_sample_range(t_in, n, dt, o, d, brick):
    """Samples of [0, n) owned by the brick: t_in_b <= t_j < t_out_b (C6).
    Returns (j0, j1, j0 unclamped, j1 unclamped, t_in_b, t_out_b, hit_b)."""
    tb0, tb1 = slab(o, d, tuple(float(x) for x in brick.lo), tuple(float(x) for x in brick.hi))
    hit_b = tb0 < tb1
    j0u = np.where(tb0 == -np.inf, 0,
                   first_index_at_or_after(t_in, dt, np.where(np.isfinite(tb0), tb0, 0.0)))
    j1u = np.where(tb1 == np.inf, n,
                   first_index_at_or_after(t_in, dt, np.where(np.isfinite(tb1), tb1, 0.0)))
    j0 = np.minimum(j0u, n)
    j1 = np.clip(j1u, j0, n)
    j1 = np.where(hit_b, j1, j0)
    return j0, j1, j0u, j1u, tb0, tb1, hit_b


def render_bricked(stored, dims, cam: Camera, tf: TransferFunction, dt: float, tau: float,
                   pixels=None, chunk=1024, want_subimages=False) -> RenderResult:
    """Per-brick render with local early termination, then sort-last compositing
    in visibility order (R_bricked; Sections 2.1, 2.3.2, 2.3.3)."""
    px, py = _pixels(cam, pixels)
    R = len(px)
    table = tf.table(dt)
    order, _ = visibility_order([sb.brick for sb in stored], cam)
    by_index = {sb.brick.index: sb for sb in stored}
    img = np.zeros((R, 4))
    tie = np.zeros(R, dtype=bool)
    used = np.zeros(R, dtype=np.int64)
    foot = {sb.brick.index: np.zeros(R, dtype=bool) for sb in stored}
    subs = {sb.brick.index: np.zeros((R, 4)) for sb in stored} if want_subimages else None
    for s, e in _chunks(R, chunk):
        o, d = cam.rays(px[s:e], py[s:e])
        t_in, t_out, hit = global_interval(o, d, dims)
        n = sample_count(t_in, t_out, dt, hit)
        last = t_in + (n - 0.5) * dt
        nxt = t_in + (n + 0.5) * dt
        tie[s:e] |= hit & ((np.abs(last - t_out) < DELTA_T) | (np.abs(nxt - t_out) < DELTA_T))
        F = np.zeros((e - s, 4))
        for bi in order:
            sb = by_index[bi]
            j0, j1, j0u, j1u, tb0, tb1, hit_b = _brick_sample_range(t_in, n, dt, o, d, sb.brick)
            cnt = j1 - j0
            foot[bi][s:e] = cnt > 0
            # (a brick the ray grazes, entered in FP64 or nearly, counts too)
            live = tb0 < tb1 + 2.0 * DELTA_T
            for tb, cand in ((tb0, (j0u - 1, j0u)), (tb1, (j1u - 1, j1u))):
                for jj in cand:
                    tj = t_in + (jj + 0.5) * dt
                    with np.errstate(invalid="ignore"):
                        near = np.abs(tj - tb) < DELTA_T
                    tie[s:e] |= (live & np.isfinite(tb) & (jj >= 0) & (jj < n)
                                 & near)
            J = int(cnt.max()) if len(cnt) else 0
            if J == 0:
                continue
            k = np.arange(J)
            valid = k[None, :] < cnt[:, None]
            jj = j0[:, None] + k[None, :]
            t = t_in[:, None] + (jj + 0.5) * dt
            p = o[:, None, :] + np.where(valid, t, 0.0)[..., None] * d[:, None, :]
            lo = np.asarray(sb.brick.lo)
            pc = np.where(valid[..., None], p, lo + 0.5)
            v = trilinear(sb.values, pc, origin=sb.origin, decode=sb.decode)
            c = tf.lookup(table, v)
            S, u, tt = composite(c, valid, tau)
            tie[s:e] |= tt
            used[s:e] += u
            if subs is not None:
                subs[bi][s:e] = S
            F = over(F, S)
        img[s:e] = F
    branches, overflow = {}, np.zeros(R, dtype=bool)
    for r in np.nonzero(tie)[0]:
        res, ovf = ray_branches(stored, dims, cam, tf, dt, tau, int(px[r]), int(py[r]))
        branches[int(r)] = res
        overflow[r] = ovf
    out = RenderResult(img, tie, branches, overflow, used, order, foot)
    out.subimages = subs
    return out


# ------------------------------------------------- per-ray branch enumeration
# A near tie is a discontinuous decision whose FP64 margin is below DELTA_T
# (sample times against the cube exit or a brick face) or DELTA_ALPHA (the
# opacity of a brick's ray against tau).  A ray's reachable results are
# enumerated in two layers:
#   membership  every sample near a face may belong to any brick whose interval
#               it is near (one owner per sample, as the bricks partition the
#               ray), and a sample near the cube exit may be taken or not;
#               the combinations are the ray's configurations;
#   termination per brick, opacity never decreases along its samples, so the
#               reachable ends of its ray are: after each sample whose opacity
#               lies within DELTA_ALPHA of tau, after the first sample at or
#               above tau + DELTA_ALPHA, and after its last sample if none is;
#               that is linear in the number of samples, with no cap.
# Sub-images are folded over the bricks in visibility order (C8); results that
# are bit-identical are kept once (a transparent sample leaves a brick's
# sub-image unchanged, so a long transparent run near tau adds nothing).
def _ray_chord(dims, o, d, dt):
    t_in, t_out, hit = global_interval(o[None, :], d[None, :], dims)
    t_in, t_out, hit = float(t_in[0]), float(t_out[0]), bool(hit[0])
    if not hit:
        return t_in, t_out, False, 0
    n = int(sample_count(np.array([t_in]), np.array([t_out]), dt, np.array([True]))[0])
    return t_in, t_out, True, n


def _sample_owner_options(stored_sorted, o, d, t_in, dt, n_max):
    """For samples j < n_max: the owner options (tuples of positions in
    stored_sorted), the FP64 default first.  A sample inside exactly one brick
    and near no face has that brick alone."""
    tj = t_in + (np.arange(n_max) + 0.5) * dt
    claim = [[] for _ in range(n_max)]
    near = [[] for _ in range(n_max)]
    o1, d1 = o[None, :], d[None, :]
    for pos, sb in enumerate(stored_sorted):
        br = sb.brick
        tb0, tb1 = slab(o1, d1, tuple(float(x) for x in br.lo), tuple(float(x) for x in br.hi))
        tb0, tb1 = float(tb0[0]), float(tb1[0])
        if not tb0 < tb1 + 2.0 * DELTA_T:
            continue
        inside = (tb0 <= tj) & (tj < tb1)
        with np.errstate(invalid="ignore"):
            close = (np.abs(tj - tb0) < DELTA_T) | (np.abs(tj - tb1) < DELTA_T)
        for j in np.nonzero(inside)[0]:
            claim[j].append(pos)
        for j in np.nonzero(close)[0]:
            near[j].append(pos)
    options = []
    for j in range(n_max):
        default = tuple(claim[j])
        opts = [default]
        if near[j]:
            for pos in sorted(set(claim[j]) | set(near[j])):
                if (pos,) not in opts:
                    opts.append((pos,))
        options.append(opts)
    return options


def _brick_results(sb, o, d, t_in, dt, members, table, tf, tau):
    """Distinct sub-images of one brick over its reachable termination points."""
    ts = t_in + (np.asarray(members, dtype=np.float64) + 0.5) * dt
    p = o[None, :] + ts[:, None] * d[None, :]
    v = trilinear(sb.values, p, origin=sb.origin, decode=sb.decode)
    c = tf.lookup(table, v)
    S = np.zeros(4)
    prefix = []
    for m in range(len(members)):
        S = S + (1.0 - S[3]) * c[m]
        prefix.append(S)
    ends = []
    for k, Sk in enumerate(prefix):
        if abs(Sk[3] - tau) < DELTA_ALPHA:
            ends.append(k)
        elif Sk[3] >= tau + DELTA_ALPHA:
            ends.append(k)
            break
    else:
        ends.append(len(prefix) - 1)
    out = {}
    for k in ends:
        out.setdefault(tuple(prefix[k].tolist()), prefix[k])
    return list(out.values())


def ray_branches(stored, dims, cam, tf, dt, tau, px, py):
    """Every result one ray of R_bricked can take over its near-tie decisions.
    Returns (list of (4,) results, overflow); overflow is set when the ray has
    more than MAX_CONFIGS membership configurations or more than MAX_BRANCHES
    distinct results (the list is then incomplete)."""
    order, _ = visibility_order([sb.brick for sb in stored], cam)
    by_index = {sb.brick.index: sb for sb in stored}
    stored_sorted = [by_index[i] for i in order]
    o, d = cam.rays(np.array([px]), np.array([py]))
    o, d = o[0], d[0]
    t_in, t_out, hit, n0 = _ray_chord(dims, o, d, dt)
    if not hit:
        return [np.zeros(4)], False
    # exit decision: the last included sample and the first excluded one
    counts = [n0]
    for jj, inc in ((n0 - 1, n0 - 1), (n0, n0 + 1)):
        if jj >= 0 and abs(t_in + (jj + 0.5) * dt - t_out) < DELTA_T and inc not in counts:
            counts.append(inc)
    n_max = max(counts)
    options = _sample_owner_options(stored_sorted, o, d, t_in, dt, n_max)
    tie_js = [j for j in range(n_max) if len(options[j]) > 1]
    n_conf = len(counts)
    for j in tie_js:
        n_conf *= len(options[j])
    if n_conf > MAX_CONFIGS:
        return [], True
    table = tf.table(dt)
    cache = {}
    results = {}
    overflow = False
    for n in counts:
        js = [j for j in tie_js if j < n]
        for choice in itertools.product(*[options[j] for j in js]):
            owner = {j: options[j][0] for j in range(n)}
            owner.update(zip(js, choice))
            members = [[] for _ in stored_sorted]
            for j in range(n):
                for pos in owner[j]:
                    members[pos].append(j)
            partial = {(0.0, 0.0, 0.0, 0.0): np.zeros(4)}
            for pos, mem in enumerate(members):
                if not mem:
                    continue
                key = (pos, tuple(mem))
                if key not in cache:
                    cache[key] = _brick_results(stored_sorted[pos], o, d, t_in, dt, mem, table, tf, tau)
                nxt = {}
                for F in partial.values():
                    for S in cache[key]:
                        G = over(F, S)
                        nxt.setdefault(tuple(G.tolist()), G)
                if len(nxt) > MAX_BRANCHES:
                    overflow = True
                    break
                partial = nxt
            if overflow:
                break
            results.update(partial)
        if overflow or len(results) > MAX_BRANCHES:
            overflow = True
            break
    return list(results.values()), overflow


# ------------------------------------------------------------ image helpers
def to_image(result: RenderResult, cam: Camera):
    return result.image.reshape(cam.height, cam.width, 4)


def max_abs_with_branches(gpu, result: RenderResult):
    """Per-pixel max |gpu - oracle| taking, for near-tie rays, the closest
    branch.  gpu is (R, 4) for the same pixels as result."""
    err = np.max(np.abs(gpu - result.image), axis=1)
    for r, alts in result.branches.items():
        if alts:
            err[r] = min(err[r], min(float(np.max(np.abs(gpu[r] - a))) for a in alts))
    return err


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2))
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)
