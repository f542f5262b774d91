"""Plain FP64 CPU oracle for the POD-2G preconditioned CG method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library; the two meet only through the seeded inputs of
``paper_2207_02543_amd.inputs``.

Modules (each function cites the passage of the paper it follows):

* ``fem``      -- Galerkin FE discretisation K(theta) u = f (Sec. 2.1).
* ``pod``      -- POD by the method of snapshots (Sec. 3.3, steps 1-2).
* ``twogrid``  -- damped-Jacobi relaxation and the two-level cycle with the
                  POD basis as prolongation (Sec. 2.2 Alg. 2, Sec. 3.3).
* ``pcg``      -- PCG preconditioned by one two-grid cycle (Sec. 3.4 Alg. 3),
                  the standalone two-grid solver (Sec. 3.3, Alg. 2) and the
                  POD-Galerkin reduced solve (Sec. 3.3, step 3).
* ``problem``  -- glue: builds a workload's matrices, training snapshots,
                  basis and warm-started queries from the seeded inputs.

Everything is FP64 except the optional FP32-emulated preconditioner mode of
``twogrid.cycle``, which rounds the preconditioner's operands to binary32.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant, a textbook routine or brute force, except the
error-bound constants of Sec. 3.5, which the paper does not make computable
(parity unpinned; not implemented here).
"""
