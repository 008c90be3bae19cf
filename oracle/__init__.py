"""CPU oracle (FP64) -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package. The product library (``paper_2603_08499_amd``) never
imports, links or executes anything here, and this package imports nothing from
the product. Parity unpinned: none (every function is pinned by a CPU test
against closed forms, invariants, quadrature or finite differences).
"""
