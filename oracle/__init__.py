"""CPU oracle for model-based iterative edge-illumination tomography.

TEST INFRASTRUCTURE ONLY: plain, slow FP64 NumPy written from the paper, used by the
test suite, the smoke check and the benchmark's CPU-baseline leg to check and time the
HIP path. Nothing in the product path imports it, and it imports nothing from the
product package (inputs reach it as arrays).

Parity pins: every function here is pinned by a test in tests/test_oracle_*.py against
closed forms, invariants, brute force or library special cases, except the learned
U-Net's trained weights (parity unpinned; judged by the measured time-to-tolerance).
"""
