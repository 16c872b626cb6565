"""MI355X (gfx950) force engine for long-range molecular dynamics.

The hot path of Rocha Filho's method (the force evaluations inside the
fourth-order Yoshida integrator for the Ring, HMF and 2D self-gravitating
models) as hand-written HIP kernels behind the C ABI of ``include/md.h``.
``paper_1212_0262_amd.md`` is the Python binding; ``inputs`` holds the seeded
initial-condition generators.
"""
