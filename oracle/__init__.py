"""FP64 CPU oracle for the Fullwave 2 time stepper (Sode & Pinton, arXiv 2106.11476).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this directory: only the test suite, the smoke check of
the build entry point, and the CPU-baseline leg of the benchmark use it.

The oracle is a plain, slow, obviously correct restatement of the paper in
double precision.  It shares no code with the HIP library: every derived
coefficient (stencil weights, relaxation a/b, boundary profiles, staggered
medium values) is recomputed here from the paper's formulas.  The only thing
it has in common with the GPU path is the seeded input generator in
``workloads`` (which holds no arithmetic of the method).

Modules
-------
stencil     Staggered (2M,4) finite-difference weights (Sec. 3.1).
relaxation  Memory-variable coefficients a, b (Sec. 3.2, Eqs. relaxation_a/b)
            and the dispersion relation (Eqs. dispersion_relations, gamma1).
pml         Two-stage C-PML + transition profiles (Sec. 3.3, Table 1).
fit         Relaxation-parameter fit to a power law (Sec. 4.1, Eq.
            relaxation_parameter_optimization).
solver      Per-point coefficient maps and the time loop (C stepper in
            fw2_oracle.c, plus a vectorised NumPy twin for tiny grids).
physics     Closed-form references used as pins (Green's function, exact
            pre-shock simple wave, power-law / Kramers-Kronig targets).
adjoint     Discrete adjoint of the time-centred step (gradient of a trace
            misfit with respect to c), pinned by central differences of the
            stepper.
reflection  The two-stage C-PML's reflection measured with the stepper
            (Secs. 4.2-4.3) and the study of its settings.
"""
