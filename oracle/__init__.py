"""CPU FP64 reference implementation (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The GPU library must never depend on it.
"""
