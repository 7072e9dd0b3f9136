"""FP64 CPU oracle of the coupled phase-field / hydrodynamic LBM step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.
"""
