"""FP64 CPU oracle for the hydro packet step.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product path (the HIP library and its
binding) never imports, links or runs anything here, and shares no code with
it.  The C solver lives in ``hydro_oracle.c``; ``oracle.py`` loads it;
``exact_riemann.py`` holds the exact Riemann solution used to pin it.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, textbook values and exact solutions (see the
module docstrings of those tests).  No function is parity-unpinned.
"""
