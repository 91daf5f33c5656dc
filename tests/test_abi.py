"""C ABI: the built library loads, exports every entry point the header
declares, and rejects bad arguments and out-of-order calls on a host-only
context (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1205_0282_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "brickcast.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert set(_declared()) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.fixture
def host_ctx(lib):
    h = C.c_void_p()
    assert lib.bc_create(-1, C.byref(h)) == binding.BC_OK
    yield h
    lib.bc_destroy(h)


def _desc(dims=(64, 64, 64), brick=(32, 32, 32), storage=0):
    d = binding.VolumeDesc()
    d.global_dims[:] = dims
    d.share_lo[:] = (0, 0, 0)
    d.share_hi[:] = dims
    d.brick_dims[:] = brick
    d.ghost = 1
    d.storage = storage
    d.src_dtype = 0
    return d


def _plan(lib, h, d, views=1, w=64, h_=64, tiles=0):
    sizes = (C.c_size_t * 4)()
    return lib.bc_plan(h, C.byref(d), views, w, h_, tiles, sizes), [int(s) for s in sizes]


def test_create_rejects_bad_args(lib):
    assert lib.bc_create(-1, None) == binding.BC_E_ARG
    h = C.c_void_p()
    assert lib.bc_create(-7, C.byref(h)) == binding.BC_E_ARG
    assert h.value is None
    assert b"device" in lib.bc_last_error(None)


def test_plan_sizes(lib, host_ctx):
    rc, sz = _plan(lib, host_ctx, _desc())
    assert rc == 0
    # 8 bricks of 32^3 -> ghosted 34 -> padded 36 per axis = 9^3 micro-blocks of
    # 80 elements (16 rows of 5), 4 bytes each
    assert sz[0] == 8 * 9 ** 3 * 80 * 4
    assert sz[3] >= 34 ** 3 * 4
    rc, sz16 = _plan(lib, host_ctx, _desc(storage=1))
    assert rc == 0 and sz16[0] == 8 * 9 ** 3 * 80 * 2
    rc, sz8 = _plan(lib, host_ctx, _desc(storage=2))
    assert rc == 0 and sz8[0] == (8 * 9 ** 3 * 80 + 255) // 256 * 256   # rounded up to 256 B
    # uneven edge bricks: 70 = 32 + 32 + 6 -> padded 36, 36, 8 -> 9, 9, 2 micro-blocks
    rc, szu = _plan(lib, host_ctx, _desc(dims=(70, 64, 64)))
    assert rc == 0 and szu[0] == (2 * 9 + 2) * 9 * 9 * 2 * 2 * 80 * 4


@pytest.mark.parametrize("field,value", [
    ("global_dims", (0, 64, 64)), ("brick_dims", (0, 32, 32)), ("ghost", 2), ("storage", 7),
    ("src_dtype", 2), ("share_hi", (65, 64, 64)), ("share_lo", (10, 0, 0))])
def test_plan_rejects_bad_desc(lib, host_ctx, field, value):
    d = _desc()
    if field == "share_lo":
        d.share_hi[:] = (10, 64, 64)
    attr = getattr(d, field)
    if isinstance(value, tuple):
        attr[:] = value
    else:
        setattr(d, field, value)
    rc, _ = _plan(lib, host_ctx, d)
    assert rc == binding.BC_E_ARG
    assert lib.bc_last_error(host_ctx)


def test_plan_rejects_too_many_bricks_and_views(lib, host_ctx):
    rc, _ = _plan(lib, host_ctx, _desc(dims=(1024, 1024, 1024), brick=(16, 16, 16)))
    assert rc == binding.BC_E_ARG
    rc, _ = _plan(lib, host_ctx, _desc(), views=5)
    assert rc == binding.BC_E_ARG
    rc, _ = _plan(lib, host_ctx, _desc(), w=0)
    assert rc == binding.BC_E_ARG


def test_plan_rejects_bricks_past_32bit_offsets(lib, host_ctx):
    """Offsets and buffer ranges inside a brick are 32-bit: a 1024^3 FP32 brick
    (257^3 micro-blocks of 80 elements, 5.4 GB) is refused, the same brick in
    FP16 (2.7 GB) and a 944^3 FP32 brick (4.26 GB) are accepted (sizes rounded up to 256 B)."""
    rc, _ = _plan(lib, host_ctx, _desc(dims=(1024, 1024, 1024), brick=(1024, 1024, 1024)))
    assert rc == binding.BC_E_ARG and b"4 GiB" in lib.bc_last_error(host_ctx)
    rc, sz = _plan(lib, host_ctx, _desc(dims=(1024, 1024, 1024), brick=(1024, 1024, 1024), storage=1))
    assert rc == 0 and sz[0] == (257 ** 3 * 80 * 2 + 255) // 256 * 256   # rounded up to 256 B
    rc, sz = _plan(lib, host_ctx, _desc(dims=(944, 944, 944), brick=(944, 944, 944)))
    assert rc == 0 and sz[0] == (237 ** 3 * 80 * 4 + 255) // 256 * 256


def _tf(lib, h, rgba, K=None, vmin=0.0, vmax=1.0, dt_ref=1.0):
    a = np.ascontiguousarray(rgba, np.float32)
    return lib.bc_set_transfer_function(h, a.ctypes.data_as(C.POINTER(C.c_float)),
                                        a.shape[0] if K is None else K, vmin, vmax, dt_ref)


def test_transfer_function_checks(lib, host_ctx):
    good = np.full((8, 4), 0.5, np.float32)
    assert _tf(lib, host_ctx, good) == 0
    assert _tf(lib, host_ctx, good, K=1) == binding.BC_E_ARG
    assert _tf(lib, host_ctx, np.full((4097, 4), 0.5)) == binding.BC_E_ARG
    assert _tf(lib, host_ctx, good, vmin=1.0, vmax=1.0) == binding.BC_E_ARG
    assert _tf(lib, host_ctx, good, vmin=float("nan")) == binding.BC_E_ARG
    assert _tf(lib, host_ctx, good, dt_ref=0.0) == binding.BC_E_ARG
    bad = good.copy(); bad[3, 2] = 1.5
    assert _tf(lib, host_ctx, bad) == binding.BC_E_ARG
    bad[3, 2] = np.nan
    assert _tf(lib, host_ctx, bad) == binding.BC_E_ARG
    assert lib.bc_set_transfer_function(host_ctx, None, 8, 0.0, 1.0, 1.0) == binding.BC_E_ARG


def _views(*vs):
    return (binding.View * len(vs))(*[binding._view_struct(v) for v in vs])


def test_view_checks(lib, host_ctx):
    v = synth.orbit_view((64, 64, 64), 3, kind="persp", width=64, height=48)
    assert lib.bc_set_view(host_ctx, _views(v), 1) == 0
    assert lib.bc_set_view(host_ctx, _views(v, v, v, v), 4) == 0
    assert lib.bc_set_view(host_ctx, None, 1) == binding.BC_E_ARG
    assert lib.bc_set_view(host_ctx, _views(v), 0) == binding.BC_E_ARG
    assert lib.bc_set_view(host_ctx, _views(v, v, v, v, v), 5) == binding.BC_E_ARG
    for mutate in ("scale", "proj", "step", "ert", "size", "nan", "mixed"):
        w = synth.orbit_view((64, 64, 64), 3, kind="persp", width=64, height=48)
        vs = [w]
        if mutate == "scale":
            w.modelview = w.modelview.copy(); w.modelview[0] *= 2.0
        elif mutate == "proj":
            w.projection = w.projection.copy(); w.projection[11] = -0.5
        elif mutate == "step":
            w.step = 0.0
        elif mutate == "ert":
            w.ert = 1.5
        elif mutate == "size":
            w.width = 0
        elif mutate == "nan":
            w.modelview = w.modelview.copy(); w.modelview[13] = np.nan
        elif mutate == "mixed":
            u = synth.orbit_view((64, 64, 64), 3, kind="persp", width=32, height=48)
            vs = [w, u]
        assert lib.bc_set_view(host_ctx, _views(*vs), len(vs)) == binding.BC_E_ARG, mutate
        assert lib.bc_last_error(host_ctx)


def test_view_tile_budget(lib, host_ctx):
    d = _desc()
    rc, _ = _plan(lib, host_ctx, d, views=1, w=64, h_=64, tiles=4)
    assert rc == 0
    v = synth.orbit_view((64, 64, 64), 3, kind="persp", width=64, height=64)
    assert lib.bc_set_view(host_ctx, _views(v), 1) == binding.BC_E_NOMEM
    rc, _ = _plan(lib, host_ctx, d, views=1, w=64, h_=64, tiles=0)
    assert lib.bc_set_view(host_ctx, _views(v), 1) == 0


def test_step_bounded_by_the_cube_diagonal(lib, host_ctx):
    """Once planned, a view whose step would take more than 2^22 samples along
    the cube's diagonal is refused (sample indices stay exact in FP32)."""
    d = _desc()
    rc, _ = _plan(lib, host_ctx, d, views=1, w=64, h_=64, tiles=0)
    assert rc == 0
    diag = float(np.linalg.norm(np.asarray(d.global_dims[:], np.float64)))
    v = synth.orbit_view((64, 64, 64), 3, kind="persp", width=64, height=64)
    v.step = diag / 2 ** 22 * 1.01
    assert lib.bc_set_view(host_ctx, _views(v), 1) == 0
    v.step = diag / 2 ** 22 * 0.99
    assert lib.bc_set_view(host_ctx, _views(v), 1) == binding.BC_E_ARG
    assert b"2^22" in lib.bc_last_error(host_ctx)


def test_host_only_context_refuses_gpu_calls(lib, host_ctx):
    rc, _ = _plan(lib, host_ctx, _desc())
    assert rc == 0
    ptrs = (C.c_void_p * 4)()
    sizes = (C.c_size_t * 4)()
    assert lib.bc_bind_memory(host_ctx, ptrs, sizes) == binding.BC_E_STATE
    assert lib.bc_render_frame(host_ctx, None, None) == binding.BC_E_STATE
    st = binding.FrameStats()
    assert lib.bc_get_frame_stats(host_ctx, C.byref(st)) == binding.BC_E_STATE
    strides = (C.c_int64 * 3)(1, 64, 64 * 64)
    assert lib.bc_load_bricks(host_ctx, C.c_void_p(1), strides, 0) == binding.BC_E_STATE
    assert lib.bc_read_brick(host_ctx, 0, None, 0, None) == binding.BC_E_STATE


def test_get_bricks_after_plan(lib, host_ctx):
    rc, _ = _plan(lib, host_ctx, _desc(dims=(70, 64, 40), brick=(32, 32, 32)))
    assert rc == 0
    n = C.c_int()
    assert lib.bc_get_bricks(host_ctx, None, None, None, 0, C.byref(n)) == 0
    assert n.value == 3 * 2 * 2
    lohi = np.zeros((n.value, 6), np.int32)
    assert lib.bc_get_bricks(host_ctx, lohi.ctypes.data_as(C.POINTER(C.c_int32)), None, None, n.value, C.byref(n)) == 0
    from oracle import raycast as rc_
    ref = rc_.brick_grid((70, 64, 40), (32, 32, 32))
    assert np.array_equal(lohi, np.array([list(b.lo) + list(b.hi) for b in ref], np.int32))


def test_options_learned_mode_and_upsampler_argument_checks(lib, host_ctx):
    ok = {binding.BC_OPT_EMPTY_SKIP: (0, 1), binding.BC_OPT_SAMPLE_CHUNK: (32, 64),
          binding.BC_OPT_RENDER_WORKGROUPS: (1, 4096), binding.BC_OPT_XCD_QUEUES: (0, 1),
          binding.BC_OPT_TILE_WIDTH: (16, 4, 8)}
    bad = {binding.BC_OPT_EMPTY_SKIP: (2, -1), binding.BC_OPT_SAMPLE_CHUNK: (16, 0),
           binding.BC_OPT_RENDER_WORKGROUPS: (0, 1 << 21), binding.BC_OPT_XCD_QUEUES: (2,),
           binding.BC_OPT_GRAPH: (5,), binding.BC_OPT_TILE_WIDTH: (2, 32, 0), 99: (1,)}
    for opt, vals in ok.items():
        for v in vals:
            assert lib.bc_set_option(host_ctx, opt, v) == binding.BC_OK, (opt, v)
    for opt, vals in bad.items():
        for v in vals:
            assert lib.bc_set_option(host_ctx, opt, v) == binding.BC_E_ARG, (opt, v)
    assert lib.bc_set_learned(host_ctx, 1, 2.0, 40.0, 8) == binding.BC_OK
    assert lib.bc_set_learned(host_ctx, 2, 2.0, 40.0, 8) == binding.BC_E_ARG
    assert lib.bc_set_learned(host_ctx, 1, 0.0, 40.0, 8) == binding.BC_E_ARG
    assert lib.bc_set_learned(host_ctx, 1, 2.0, float("inf"), 8) == binding.BC_E_ARG
    assert lib.bc_set_learned(host_ctx, 1, 2.0, 40.0, 65) == binding.BC_E_ARG
    nb = C.c_size_t()
    assert lib.bc_cnn_plan(host_ctx, 0, 10, 10, C.byref(nb)) == binding.BC_E_ARG
    assert lib.bc_cnn_plan(host_ctx, 1, 10, 9000, C.byref(nb)) == binding.BC_E_ARG
    assert lib.bc_cnn_plan(host_ctx, 1, 10, 10, None) == binding.BC_E_ARG
    assert lib.bc_cnn_plan(host_ctx, 2, 540, 960, C.byref(nb)) == binding.BC_OK and nb.value > 0
    assert lib.bc_cnn_bind(host_ctx, C.c_void_p(256), nb.value) == binding.BC_E_STATE      # host-only
    w = np.zeros(binding.CNN_N_PARAMS, np.float32)
    assert lib.bc_cnn_set_weights(host_ctx, w.ctypes.data_as(C.POINTER(C.c_float)), None, None, w.size,
                                  0) == binding.BC_E_STATE
    assert lib.bc_autotune(host_ctx, None, None, 2, None) == binding.BC_E_STATE
    ms = (C.c_double * 3)()
    assert lib.bc_get_timing(host_ctx, ms, None) == binding.BC_E_STATE


def test_operator_argument_checks(lib, host_ctx):
    assert lib.bc_set_operator(None, 0, 0) == binding.BC_E_ARG
    assert lib.bc_set_operator(host_ctx, 2, 0) == binding.BC_E_ARG
    assert lib.bc_set_operator(host_ctx, -1, 0) == binding.BC_E_ARG
    assert lib.bc_set_operator(host_ctx, binding.BC_OP_MIP, 2) == binding.BC_E_ARG
    # compositing corrects its table for one step per frame
    assert lib.bc_set_operator(host_ctx, binding.BC_OP_COMPOSITE, binding.BC_STEP_PER_VOXEL) == binding.BC_E_UNSUPPORTED
    assert b"step" in lib.bc_last_error(host_ctx)
    for op, st in ((binding.BC_OP_MIP, binding.BC_STEP_PER_VOXEL), (binding.BC_OP_MIP, binding.BC_STEP_FIXED),
                   (binding.BC_OP_COMPOSITE, binding.BC_STEP_FIXED)):
        assert lib.bc_set_operator(host_ctx, op, st) == binding.BC_OK


def test_header_is_c99_and_a_c_program_links(lib, tmp_path):
    """The header compiles as strict C99 (no C++ in it), a C program links
    against the library and plans through it on a host-only context, and the
    C structs have the sizes the binding's ctypes structures assume."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "plan.c"
    src.write_text(r'''
#include <stdio.h>
#include "brickcast.h"
int main(void) {
  bc_ctx* h = NULL;
  if (bc_create(-1, &h) != BC_OK) return 1;
  bc_volume_desc d = {0};
  for (int a = 0; a < 3; ++a) { d.global_dims[a] = 64; d.share_hi[a] = 64; d.brick_dims[a] = 32; }
  d.ghost = 1;
  size_t sizes[4];
  const int r = bc_plan(h, &d, 1, 64, 64, 0, sizes);
  printf("%d %zu %zu %zu %zu %zu %zu %zu\n", r, sizes[0], sizes[1], sizes[2], sizes[3], sizeof(bc_view),
         sizeof(bc_volume_desc), sizeof(bc_frame_stats));
  bc_destroy(h);
  return r == BC_OK ? 0 : 2;
}
''')
    libdir = os.path.dirname(binding.LIB_PATH)
    exe = tmp_path / "plan"
    build = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                            os.path.join(ROOT, "include"), str(src), "-L", libdir, "-lbrickcast",
                            "-Wl,-rpath," + libdir, "-o", str(exe)], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stdout + run.stderr
    vals = [int(x) for x in run.stdout.split()]
    h = C.c_void_p()
    assert lib.bc_create(-1, C.byref(h)) == binding.BC_OK
    code, sizes = _plan(lib, h, _desc())
    lib.bc_destroy(h)
    assert vals[0] == code == binding.BC_OK
    assert vals[1:5] == sizes
    assert vals[5:] == [C.sizeof(binding.View), C.sizeof(binding.VolumeDesc), C.sizeof(binding.FrameStats)]
