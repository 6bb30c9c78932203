"""Plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the GPU library.
"""
