"""FP64 CPU oracle for the bricked volume ray caster.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
rendering library never imports, links or calls it, and it shares no code,
tables or constants with the HIP path.

Modules:
  raycast   -- rays from the viewer's OpenGL matrices, slab clipping, trilinear
               sampling, transfer function, front-to-back compositing with early
               ray termination, bricking with ghosts, visibility order,
               sort-last compositing (Sections 1.2, 2.1, 2.3.2, 2.3.3).
  mip       -- maximum intensity projection (the paper's adopted operator,
               Sections 2.3.2 and 2.3.3): per-ray maximum, any-order merge of
               brick maxima, colour map after the merge, fixed or per-voxel
               step.
  encoders  -- IEEE binary16 and OCP FP8 e4m3 storage encoders, per-brick
               scale/offset (no passage in the paper: storage forms of the cube).
  cnn       -- the learned upsampler's forward/backward and Adam (no passage in
               the paper; a stated reading).
"""
