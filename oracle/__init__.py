"""CPU oracle for the space-time BIEM convolution (test infrastructure only).

This package is the slow, plain, obviously-correct FP64 reference that the
GPU library is checked against.  It is *test infrastructure*: only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The product path (the HIP library and its Python binding) never calls
into it, and it shares no code with that path; the only common dependency is
the seeded input generator module ``synth``.

Contents
  kernel2d  closed-form step response and discrete kernel of the 2D
            anti-plane (mode III) problem, Sec. 2.1 (Eq. 4 and the
            definition of K_m under it).
  dense     Tier-A: the exact dense time-marching convolution, Eq. 4.
  fdph      Tier-B: the FDP=H-approximated kernel (FDPM split, block cluster
            tree, ART integers, degenerate waveforms, Domain S static and
            2D transient terms, inadmissible windows) assembled densely and
            applied by the same direct convolution.  No rings, no ACA.
  inplane2d closed-form 2 x 2 kernel of the 2D in-plane (P-SV) problem on a
            straight fault.
  rupture   dynamic rupture: the convolution coupled to the paper's
            friction laws (Sec. 6.2, App. A.2.3), first lag implicit.

Parity status of each function is stated in its docstring; every function
here is pinned by tests under ``tests/`` (marked ``not gpu``) against values
that do not come from the oracle itself (closed forms, physical limits,
brute-force quadrature of the Green's function, definitional identities).
"""
