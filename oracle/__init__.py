"""FP64 CPU oracle of the colour-gradient LBM step with reaction-limited evaporation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the HIP product path never does.
"""
