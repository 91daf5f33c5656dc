"""Seeded synthetic inputs: spectral data cube stand-ins, transfer-function tables
and viewer camera matrices.

This module produces inputs only.  It holds none of the ray-casting arithmetic
(no sampling, interpolation, opacity correction or compositing), so both the
FP64 oracle and the HIP path can consume what it makes.

Workload shapes follow the paper's data cubes (Section 3.1, Table 1): spectral
cubes are noise-dominated with compact sources near or below the noise level
(Section 1.1).  The datasets themselves are not available, so a cube here is
N(0, 1) noise plus Gaussian sources:

* noise: float32 N(0, 1), drawn per 256^3 generation block from
  ``SeedSequence([seed, block_index])`` (PCG64), so any region can be
  regenerated on its own;
* sources: centres U[0, N) per axis (voxel-index coordinates), width
  sigma ~ U[sigma_lo, sigma_hi] * sigma_scale, peak ~ U[amp_lo, amp_hi];
  each adds ``peak * gx * gy * gz`` with ``g(i) = exp(-(i + 0.5 - c)^2 / 2 sigma^2)``
  over voxel centres with ``|i + 0.5 - c| <= 5 sigma`` (separable box cut).

The viewer's rendering request is the output frame size plus the OpenGL
projection and modelview matrices (Section 2.3.2); the helpers here build those
matrices (column-major, as OpenGL stores them) for an orbit around the cube.
"""
from __future__ import annotations

import concurrent.futures as _cf
import math
import os
import threading
from dataclasses import dataclass

import numpy as np

GEN_BLOCK = 256


# --------------------------------------------------------------------------- cubes
@dataclass(frozen=True)
class CubeRecipe:
    dims: tuple            # (nx, ny, nz)
    seed: int
    n_sources: int
    sigma_lo: float
    sigma_hi: float
    sigma_scale: float = 1.0
    amp_lo: float = 3.0
    amp_hi: float = 10.0


# Small plain workload: 128^3, 20 sources, sigma 2-8.
RECIPE_SMALL = CubeRecipe((128, 128, 128), seed=1, n_sources=20, sigma_lo=2.0, sigma_hi=8.0)
# 1024^3, 500 sources with sigma U[10, 30] * k; k puts 5.0% of voxels above 3
# (k = 1.0134 from calibrate_sigma_scale: seeded bisection on a stride-4 lattice).
RECIPE_1024 = CubeRecipe((1024, 1024, 1024), seed=2, n_sources=500, sigma_lo=10.0,
                         sigma_hi=30.0, sigma_scale=1.0134)
# 3000 x 3000 x 1500 (about 27 GB in FP16), 5000 sources, sigma U[10, 30].
RECIPE_BATCH = CubeRecipe((3000, 3000, 1500), seed=4, n_sources=5000, sigma_lo=10.0,
                          sigma_hi=30.0)
# The shapes of the paper's test cubes (Table 1) with the 1024^3 cube's source
# density (500 per 1024^3) and width law: HIPASS (12 GB in FP32), GASS (25 GB)
# and the scaled N-body cube (65.4 GB in FP32; stored here from an FP16 source).
RECIPE_HIPASS = CubeRecipe((1721, 1721, 1025), seed=5, n_sources=1413, sigma_lo=10.0, sigma_hi=30.0)
RECIPE_GASS = CubeRecipe((2502, 2501, 1093), seed=6, n_sources=3185, sigma_lo=10.0, sigma_hi=30.0)
RECIPE_NBODY2600 = CubeRecipe((2600, 2600, 2600), seed=7, n_sources=8185, sigma_lo=10.0, sigma_hi=30.0)


def draw_sources(recipe: CubeRecipe):
    """Source parameters, drawn in one stream from the recipe seed."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([recipe.seed, 7919])))
    n = recipe.n_sources
    dims = np.asarray(recipe.dims, dtype=np.float64)
    centres = rng.uniform(0.0, 1.0, size=(n, 3)) * dims[None, :]
    sigma = rng.uniform(recipe.sigma_lo, recipe.sigma_hi, size=n) * recipe.sigma_scale
    amp = rng.uniform(recipe.amp_lo, recipe.amp_hi, size=n)
    return centres, sigma, amp


def _block_grid(dims):
    return tuple((d + GEN_BLOCK - 1) // GEN_BLOCK for d in dims)


def block_values(recipe: CubeRecipe, sources, bidx: int):
    """Float32 values of generation block ``bidx`` (x fastest over the block
    grid), regenerated on its own; returns ((x0, y0, z0), array[z][y][x])."""
    nx, ny, nz = recipe.dims
    gbx, gby, _ = _block_grid(recipe.dims)
    bx = bidx % gbx
    by = (bidx // gbx) % gby
    bz = bidx // (gbx * gby)
    x0, y0, z0 = bx * GEN_BLOCK, by * GEN_BLOCK, bz * GEN_BLOCK
    x1, y1, z1 = min(x0 + GEN_BLOCK, nx), min(y0 + GEN_BLOCK, ny), min(z0 + GEN_BLOCK, nz)
    shape = (z1 - z0, y1 - y0, x1 - x0)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([recipe.seed, int(bidx)])))
    block = rng.standard_normal(size=shape, dtype=np.float32)
    centres, sigma, amp = sources
    acc = None
    lo = np.array([x0, y0, z0], dtype=np.float64)
    hi = np.array([x1, y1, z1], dtype=np.float64)
    reach = 5.0 * sigma
    # voxel centres at i + 0.5: the source touches [c - 5s, c + 5s]
    touch = np.all((centres + reach[:, None] >= lo[None, :] + 0.5) &
                   (centres - reach[:, None] <= hi[None, :] - 0.5), axis=1)
    for s in np.nonzero(touch)[0]:
        c, sg, a = centres[s], sigma[s], amp[s]
        prof = []
        for ax, (l, h) in enumerate(((x0, x1), (y0, y1), (z0, z1))):
            i = np.arange(l, h, dtype=np.float64) + 0.5
            dlt = i - c[ax]
            g = np.exp(-(dlt * dlt) / (2.0 * sg * sg))
            g[np.abs(dlt) > 5.0 * sg] = 0.0
            prof.append(g)
        gx, gy, gz = prof
        nzx, nzy, nzz = np.nonzero(gx)[0], np.nonzero(gy)[0], np.nonzero(gz)[0]
        if len(nzx) == 0 or len(nzy) == 0 or len(nzz) == 0:
            continue
        sx = slice(nzx[0], nzx[-1] + 1)
        sy = slice(nzy[0], nzy[-1] + 1)
        sz = slice(nzz[0], nzz[-1] + 1)
        if acc is None:
            acc = np.zeros(shape, dtype=np.float64)
        acc[sz, sy, sx] += a * (gz[sz][:, None, None] * gy[sy][None, :, None] * gx[sx][None, None, :])
    if acc is not None:
        block = (block.astype(np.float64) + acc).astype(np.float32)
    return (x0, y0, z0), block


def _fill_block(recipe, sources, bidx, out, out_dtype):
    (x0, y0, z0), block = block_values(recipe, sources, bidx)
    z1, y1, x1 = z0 + block.shape[0], y0 + block.shape[1], x0 + block.shape[2]
    out[z0:z1, y0:y1, x0:x1] = block.astype(out_dtype)


def make_cube(recipe: CubeRecipe, out_dtype=np.float32, workers: int | None = None,
              out: np.ndarray | None = None, progress=None) -> np.ndarray:
    """Cube as ``array[z][y][x]`` (x fastest).  ``float16`` output is a
    round-to-nearest-even cast of the float32 values.  ``progress(done,
    total)``, if given, is called after each generation block (from the
    generating threads)."""
    nx, ny, nz = recipe.dims
    if out is None:
        out = np.empty((nz, ny, nx), dtype=out_dtype)
    gb = _block_grid(recipe.dims)
    nblocks = gb[0] * gb[1] * gb[2]
    sources = draw_sources(recipe)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    done = [0]
    lock = threading.Lock()

    def fill(b):
        _fill_block(recipe, sources, b, out, out_dtype)
        if progress is not None:
            with lock:
                done[0] += 1
                progress(done[0], nblocks)

    if workers <= 1 or nblocks == 1:
        for b in range(nblocks):
            fill(b)
    else:
        # numpy releases the GIL in the random fill and the array arithmetic
        with _cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, range(nblocks)))
    return out


def lattice_fraction_above(recipe: CubeRecipe, threshold: float = 3.0, stride: int = 4,
                           lattice_seed: int = 99) -> float:
    """Estimate of the fraction of voxels above ``threshold`` on a stride lattice
    (fresh N(0, 1) noise per lattice point).  Used only to calibrate
    ``sigma_scale``."""
    nx, ny, nz = recipe.dims
    xs = np.arange(0, nx, stride, dtype=np.float64) + 0.5
    ys = np.arange(0, ny, stride, dtype=np.float64) + 0.5
    zs = np.arange(0, nz, stride, dtype=np.float64) + 0.5
    field = np.zeros((len(zs), len(ys), len(xs)), dtype=np.float64)
    centres, sigma, amp = draw_sources(recipe)
    for c, sg, a in zip(centres, sigma, amp):
        gs = []
        for ax, coords in enumerate((xs, ys, zs)):
            dlt = coords - c[ax]
            g = np.exp(-(dlt * dlt) / (2.0 * sg * sg))
            g[np.abs(dlt) > 5.0 * sg] = 0.0
            gs.append(g)
        gx, gy, gz = gs
        ix, iy, iz = np.nonzero(gx)[0], np.nonzero(gy)[0], np.nonzero(gz)[0]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        sx, sy, sz = slice(ix[0], ix[-1] + 1), slice(iy[0], iy[-1] + 1), slice(iz[0], iz[-1] + 1)
        field[sz, sy, sx] += a * gz[sz][:, None, None] * gy[sy][None, :, None] * gx[sx][None, None, :]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([lattice_seed])))
    field += rng.standard_normal(size=field.shape)
    return float(np.mean(field > threshold))


def calibrate_sigma_scale(recipe: CubeRecipe, target: float = 0.05, lo: float = 0.5,
                          hi: float = 2.0, iters: int = 12) -> float:
    """Seeded bisection on ``sigma_scale`` for a target fraction above 3."""
    import dataclasses
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        f = lattice_fraction_above(dataclasses.replace(recipe, sigma_scale=mid))
        if f < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ----------------------------------------------------------------- transfer function
def ramp_tf(vmin: float, vmax: float, K: int = 256, lo: float = 3.0, width: float = 7.0,
            alpha_max: float = 0.5) -> np.ndarray:
    """K straight (not premultiplied) RGBA entries in [0, 1]; entry k sits at
    ``vmin + k/(K-1) (vmax - vmin)``.  Opacity is exactly zero below ``lo`` so
    the noise floor is transparent; colour runs red-ish to yellow/white."""
    v = vmin + (np.arange(K, dtype=np.float64) / (K - 1)) * (vmax - vmin)
    s = np.clip((v - lo) / width, 0.0, 1.0)
    rgba = np.stack([0.2 + 0.8 * s, s * s, 1.0 - s, alpha_max * s], axis=1)
    return rgba.astype(np.float32)


def random_tf(rng: np.random.Generator, K: int, alpha_max: float = 1.0) -> np.ndarray:
    rgba = rng.uniform(0.0, 1.0, size=(K, 4))
    rgba[:, 3] *= alpha_max
    return rgba.astype(np.float32)


# ------------------------------------------------------------------------- cameras
def _col_major(m: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(m.T).reshape(16).astype(np.float64)


def look_at(eye, centre, up) -> np.ndarray:
    """OpenGL gluLookAt modelview matrix, 16 doubles column-major."""
    eye = np.asarray(eye, dtype=np.float64)
    centre = np.asarray(centre, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    f = centre - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3], m[1, :3], m[2, :3] = s, u, -f
    m[:3, 3] = -m[:3, :3] @ eye
    return _col_major(m)


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    """OpenGL gluPerspective projection matrix, column-major."""
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = (far + near) / (near - far)
    m[2, 3] = 2.0 * far * near / (near - far)
    m[3, 2] = -1.0
    return _col_major(m)


def ortho(left, right, bottom, top, near, far) -> np.ndarray:
    """OpenGL glOrtho projection matrix, column-major."""
    m = np.eye(4)
    m[0, 0] = 2.0 / (right - left)
    m[1, 1] = 2.0 / (top - bottom)
    m[2, 2] = -2.0 / (far - near)
    m[0, 3] = -(right + left) / (right - left)
    m[1, 3] = -(top + bottom) / (top - bottom)
    m[2, 3] = -(far + near) / (far - near)
    return _col_major(m)


@dataclass
class ViewSpec:
    modelview: np.ndarray   # 16 doubles, column-major
    projection: np.ndarray  # 16 doubles, column-major
    width: int
    height: int
    step: float = 0.5
    ert: float = 0.99


def orbit_view(dims, frame: int, n_frames: int = 64, kind: str = "persp",
               width: int = 1920, height: int = 1080, fovy_deg: float = 30.0,
               elevation_deg: float = 20.0, azimuth_offset_deg: float = 0.0,
               step: float = 0.5, ert: float = 0.99) -> ViewSpec:
    """Viewer orbiting the cube centre: the cube's bounding sphere (radius R =
    half-diagonal) fits the vertical field of view; eye distance D = R/sin(fovy/2)."""
    n = np.asarray(dims, dtype=np.float64)
    centre = n / 2.0
    R = 0.5 * float(np.linalg.norm(n))
    D = R / math.sin(math.radians(fovy_deg) / 2.0)
    az = 2.0 * math.pi * frame / n_frames + math.radians(azimuth_offset_deg)
    el = math.radians(elevation_deg)
    eye = centre + D * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    mv = look_at(eye, centre, (0.0, 1.0, 0.0))
    near, far = D - R - 1.0, D + R + 1.0
    aspect = width / height
    if kind == "persp":
        pr = perspective(fovy_deg, aspect, near, far)
    elif kind == "ortho":
        pr = ortho(-R * aspect, R * aspect, -R, R, near, far)
    else:
        raise ValueError(kind)
    return ViewSpec(mv, pr, width, height, step, ert)


def axis_view(dims, axis: str, width: int, height: int, step: float = 1.0, ert: float = 1.0,
              margin: float = 4.0) -> ViewSpec:
    """Orthographic view straight down +z ('z') with one pixel per voxel column,
    pixel centres on voxel centres (requires width = nx, height = ny)."""
    nx, ny, nz = dims
    assert axis == "z" and width == nx and height == ny
    cx, cy = nx / 2.0, ny / 2.0
    eye = np.array([cx, cy, -margin])
    mv = look_at(eye, eye + np.array([0.0, 0.0, 1.0]), (0.0, 1.0, 0.0))
    pr = ortho(-nx / 2.0, nx / 2.0, -ny / 2.0, ny / 2.0, 0.5, nz + 2 * margin)
    return ViewSpec(mv, pr, width, height, step, ert)
