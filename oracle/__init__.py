"""Plain, slow FP64 CPU oracle for the Quantum Flow (QFlow) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under this package; only the test suite, the smoke check
and the CPU-baseline leg of the benchmark do.  It shares no code with the HIP
path: its only common input is the seeded generator in ``synth``.

The oracle works in spin orbitals (index 2*P + spin, spin 0 = alpha) and
evaluates every operator product from its textbook normal-ordered form, so that
a reader can check each step against the definitions:

* ``so``       -- normal-ordered 0/1/2-body operators and the commutator kept
                  to its 0-, 1- and 2-body parts (the "[.,.]_2" of the DUCC
                  truncation used for Eq. (6) at N=1).
* ``qflow``    -- reference quantities, the downfolded active-space
                  Hamiltonian of Eq. (6) with N=1, the CAS eigenproblem,
                  cluster analysis, the global residual and one Jacobi
                  macro-iteration of the flow.
* ``sampling`` -- Algorithm 1 (coverage-driven active-space sampling), the
                  Delta-epsilon ordering and amplitude ownership.
"""
