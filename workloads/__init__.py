"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.
Holds no arithmetic of the method itself."""
