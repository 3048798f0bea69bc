"""CPU FP64 oracle for the block epsilon-circulant (BEC) all-at-once solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute this package: only the tests, the smoke check of the graft entry point
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library; the only common dependency is the seeded input module `workloads`.

Every function here is a plain, slow, obviously correct restatement of the
paper (Lin & Ng, "An all-at-once preconditioner for evolutionary partial
differential equations", arXiv 2002.01108); each one cites the passage it
follows.  Library primitives (matrix products, sparse LU, dense LU, QR,
eigenvalues) serve as steps; no blocking or reordering beyond the definitions.
"""
from . import heat, mg, cnn  # noqa: F401
