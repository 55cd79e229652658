"""Plain FP64 CPU oracle for GenEO two-level additive Schwarz inside PCG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check the HIP path and to
time a CPU reference.  It shares no code with the HIP path; the two only
read the same seeded inputs from ``synth``.

Each step follows the paper's definitions in the paper's order, with
numpy/scipy library primitives (sparse COO->CSR, dense Cholesky, triangular
solves, a dense symmetric eigensolver) as single steps and no blocking or
fusion beyond what the definitions state:

* ``fem``        -- conforming Q1 discretisation of the Darcy and elasticity
                    forms (Sec. 2, eqs. (2)-(3)) with symmetric elimination
                    of homogeneous Dirichlet conditions;
* ``decomp``     -- overlapping subdomains, overlap zone, partition of unity
                    (Sec. 3, Def. 3; Sec. 4.3);
* ``geneo``      -- local matrices, the GenEO generalised eigenproblem (eq. 4)
                    solved through the shift-and-invert transform of Sec. 4.4,
                    the coarse space (Def. 4), the coarse matrix (Def. 2,
                    Sec. 4.5) and the two-level additive Schwarz operator
                    (Def. 2);
* ``pcg``        -- preconditioned conjugate gradients and the Lanczos
                    condition-number estimate reported beside iterations
                    (Sec. 5.3, Table 1).

Every function is pinned by ``tests/test_oracle_*.py`` to closed forms,
invariants and brute-force results; see each module's header for its pins.
"""
from . import fem, decomp, geneo, pcg  # noqa: F401
