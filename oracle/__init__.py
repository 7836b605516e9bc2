"""CPU oracle for BP-SF: test infrastructure, never part of the product path.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import it.
"""
