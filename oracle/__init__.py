"""Plain FP64 CPU oracle for the emRKC method (test infrastructure).

This package is test infrastructure, not part of the product: only the test
suite, the smoke check of the package entry module and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the GPU library: every
formula here is written out again, in numpy, from the paper (section
"Multirate explicit stabilized methods", the RKC, mRKC and emRKC algorithms,
and the nonlinear power iteration of the appendix).

Functions whose results have no independent pin say "parity unpinned" in
their docstrings.  Nonlinear trajectories are pinned on a single cell (first
order convergence to a library ODE integrator); with diffusion they are
parity unpinned beyond the properties checked in the tests (uniform states,
convergence order, brute force on tiny meshes).
"""
