"""FP64 CPU oracle of the AQMP encoder: test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package; the GPU library and its Python binding never do.
"""
