"""Plain FP64 CPU oracle of the nonhydrostatic ocean-model hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path (the
HIP library and its Python binding) never does, and this package imports
nothing from the product.  It shares no code with the GPU kernels.

Every function follows a passage of Wagner et al., "High-level,
high-resolution ocean modeling at all scales with Oceananigans"
(arXiv 2502.14148) and is written for clarity, not speed: NumPy array
expressions in float64, one array expression per step of the method, with no
blocking, fusion or reordering beyond what the passage states.  Library
primitives (FFT, DCT, dense solves) serve as single steps.

Modules
-------
fv          halo-padded C-grid arrays and halo filling
weno        fifth-order WENO-Z reconstruction (and its linear-weight limit)
tendencies  nonhydrostatic tendencies: advection, Coriolis, buoyancy, closure
pressure    divergence, FFT/DCT eigenfunction Poisson solve, projection
timestep    low-storage RK3 substages with pressure correction
diagnostics conservation sums and divergence measures
"""
