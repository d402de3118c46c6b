"""CPU oracle: TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the GPU
path computes.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code
with the library under ``paper_2601_21552_amd/`` and never imports it; both
sides read the same seeded inputs from ``workloads``.

* ``oracle.cnf_ref``   - ctypes front end of ``dpll.c``: unit propagation,
  DPLL decide, #DPLL model count, canonical leaf (refuted / f / m / count /
  smallest satisfying index), plus numpy brute force for tiny CNFs.
* ``oracle.query_ref`` - exact-integer meaning of a query: evaluator, brute
  force, the oracle's own Tseitin encoder, and a word-level root check.
"""
