"""CPU oracle of the harmonic sum (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package. The library under test never does.
"""
