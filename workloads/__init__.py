"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

Holds code constructions, the counter-based shot generator, GF(2) scoring
helpers and the named workloads. None of the decoder's arithmetic lives here.
"""
