"""CPU FP64 oracle for the two-component colour-gradient lattice Boltzmann step.

This package is TEST INFRASTRUCTURE.  It is a plain, slow, whole-array numpy
statement of what one time step computes (paper: Sec. III.B "Basic ideas of
the Lattice Boltzmann method", Sec. III.C.1 "Color-gradient Lattice
Boltzmann" incl. the "Near-contact interactions" paragraph, Sec. III.D
"Boundary conditions", Sec. IV "Second group" for shifted storage).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The GPU product path never imports, links or calls anything here,
and nothing here imports the GPU package.

Modules
-------
lattice  velocity sets, weights, opposite table and the B_i coefficients
sim      ``OracleSim``: vectorised FP64 step (stream, moments, gradient,
         flags, near-contact scan, Guo-forced BGK, perturbation, recolouring)
naive    independent per-site Python-loop step for tiny lattices
ccl      connected-component droplet labels (breadth-first search)
mlp      FP64 reference of the near-contact MLP closure (forward, backward,
         Adam) used to check the GPU training kernels
fp16c    the FP16C 16-bit storage format (1 sign, 4 exponent, 11 significand
         bits) by its definition: decode, round-to-nearest-even encode
llb      ``OracleLLB``: the moment-based (regularised) colour-gradient step,
         whose state is 15 moments per site instead of populations

Parity pins: every function documents which identity, closed form or brute
force check pins it; the checks live under ``tests/`` (marker ``not gpu``).
"""
