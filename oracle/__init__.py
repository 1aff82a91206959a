"""CPU oracle for the SpMV library: TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct reference of what the GPU library computes:
COO ingest (sort, duplicate check, row pointers), the CSR / COO / ELL / HYB /
SELL-C-sigma / BELL layouts, y = alpha*A*x + beta*y in FP64, the 12 sparsity features and the
12-64-64-C selector network, C = 4 or 6 classes (forward, gradient, Adam,
training loop).

Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package. It shares no code with ``paper_2302_05662_amd`` and imports
nothing from it; the seeded generators in ``synth`` feed both.

Parity status: every function is pinned by the CPU tests
(tests/test_oracle_*.py) against dense brute force, exact rational sums,
closed forms, round trips, finite differences or printed values of the paper,
except the Mode feature: the paper's printed Mode column contradicts its own
definition, so Mode is the plain definition (modal row length, smallest on
ties) with parity unpinned by the paper.
"""
from . import formats, mlp, spmv  # noqa: F401
