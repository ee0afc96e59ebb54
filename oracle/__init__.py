"""BHEM CPU oracle (FP64, written from the paper).  TEST INFRASTRUCTURE ONLY:
only tests/, the smoke check and the benchmark's CPU-baseline leg use it."""
