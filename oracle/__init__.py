"""Plain, slow, FP64 CPU oracle for the dual-stencil FDTD particle-in-cell hot path.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library; it is
never part of the product path.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library or its Python binding, and imports neither.

Paper: F. Li et al., "A new field solver for modeling of relativistic
particle-laser interactions using the particle-in-cell algorithm",
arXiv:2004.03754.

Modules
-------
stencil     customized coefficient fit (App. B), textbook staggered
            coefficients, k-space symbols, dispersion, F and kappa factors,
            CFL bounds (Sec. 2.1, 3.1, 3.2)
fdtd        leapfrog field step on the Yee mesh with different x1 operators in
            Faraday's and Ampere's laws (Eq. maxwell, App. B operators),
            divergence diagnostics
particles   staggered linear-shape gather (App. A), Boris pusher, exact
            constant-field pusher, leapfrog position update, Esirkepov
            charge-conserving deposit (Sec. 3.3)
current     x1 current correction for a wide Ampere stencil (Sec. 3.3)
pic         the per-step driver: push, deposit, current correction, fused
            field sweep
trajectory  closed-form electron trajectory in a plane wave, from rest or
            drifting (Sec. 4.1, canonical momentum conservation)
window      moving window along x1 (Sec. 4.1 single-particle runs)
absorb      graded damping layers at the two x1 ends of the window
precise     the three pushers evaluated at 50 digits (strong-field checks)
adjoint     FP64 adjoint of the field sweep, gather and pushers

Every function names the passage of the paper it follows.  Readings of
passages the paper leaves open are listed at the top of the module that takes
them.
"""
