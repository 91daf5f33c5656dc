"""Bricked volume ray caster for one MI355X (gfx950).

The rendering path is the HIP library ``libbrickcast.so`` behind the C ABI in
``include/brickcast.h``; ``binding`` marshals arguments to it and ``synth``
makes seeded synthetic inputs.
"""
