"""Plain FP64 CPU oracle for the reduced implicit-Euler Newton iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library: the only
common module is the seeded input generator
(``paper_2102_11026_amd.synth``), which draws random numbers and lays out
meshes but holds none of the method's arithmetic.

Contents, each following the paper's definitions in its own order:
  multicomplex  multicomplex numbers C^n and their elementary functions
                (Sec. 4.1, the recursive definition; Appendix A)
  decoder       decoder MLP passes in multicomplex arithmetic: collective
                right contractions (Sec. 4.3) and complex-step
                backpropagation for left contractions (Sec. 4.4)
  fem           lumped mass, neo-Hookean element force / stiffness, cubature
                (Sec. 3.1, Sec. 5)
  newton        the reduced residual phi(r), its Newton matrix, LU solve and
                the implicit-Euler time step (Sec. 3.2, Sec. 3.6)
  wnet          the cubature weight-prediction MLP at inference (Sec. 5.2)

Parity status of every function is stated in its module header.
"""
