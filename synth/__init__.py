"""Seeded synthetic inputs (images and formula texts) for tests and benchmarks.

Input generation only: this package evaluates no operator of the logic.  It is
the one module that both the GPU path's tests and the oracle's tests use.
"""
