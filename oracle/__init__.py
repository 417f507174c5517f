"""FP64 CPU oracle of the bound-driven caustic estimator (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the GPU library never does.
"""
