"""FP64 CPU oracle of the overlapping-Schwarz / Operator-Inference method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code
with the HIP path (``paper_2511_20687_amd/csrc``); the only common module is
the seeded input generator ``paper_2511_20687_amd.inputs``.

The oracle is written for reading, not for speed: plain numpy / scipy.sparse
in float64 (complex128 works too, for complex-step derivatives), following the
paper's definitions and algorithms step by step.  Each module cites the
section / equation / algorithm it implements.

Modules
-------
fem       hex8 Galerkin FE for linear elasticity (Sec. 2, App. A.1)
newmark   Newmark-beta time stepping of one FE model (Sec. 2, 4.1)
rom       OpInf reduced model, compressed Kronecker powers (Sec. 3.2, 4.2)
schwarz   multiplicative overlapping Schwarz controller (Sec. 4.1, Alg. 1;
          Sec. 4.2 OpInf-FOM / OpInf-OpInf couplings)
pod       POD bases by thin SVD and the energy criterion (Sec. 3.1, Eq. pod_energy)
opinf     OpInf regularised least squares and lambda selection (Eq. opinf_schwarz_inference,
          Alg. 3)
metrics   relative space-time error (Eq. mse) and projection error (Eq. projerr)
adjoint   discrete adjoint of the coupled rollout (no paper passage: an extension)

Parity status: every function is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or library routines.
"""
