"""CPU oracle of the first-order finite-volume step (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. It shares no code with the HIP library.
"""
