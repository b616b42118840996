"""CPU oracle for the IRKGL16 hot path: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  The GPU library never
imports, links or calls it.
"""
