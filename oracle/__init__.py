"""CPU oracle for the 3D PFC second-order scheme and its FAS multigrid solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or run anything in this folder;
the HIP product path never does, and shares no code with it.

* ``cfas``       -- ctypes binding to ``pfc_oracle.c``: the FAS algorithm of
                    Section 5 step by step (plain FP64 C).
* ``definition`` -- numpy: the discrete system of scheme (1.10) solved directly
                    (dense Newton, Newton-Krylov), the energy, the Fourier
                    symbols and the adjoint of one step.

Parity status of each function is stated in its module docstring.
"""
