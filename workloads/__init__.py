"""Seeded synthetic densities shaped like the paper's test problems.

Holds no arithmetic of the solver: every function samples a density at
coordinate arrays the caller supplies (cell centres from whichever side -- the
library's geometry query or the oracle), so the same generator feeds the GPU
path, the oracle and the benchmark.
"""
