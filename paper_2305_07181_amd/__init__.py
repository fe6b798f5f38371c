"""MI355X-native entropy-split SBP-SAT residual library (Python side).

The compute path lives in the HIP/C++ shared library built from ``csrc/``;
``paper_2305_07181_amd.sbp`` is the thin ctypes binding over its C ABI
(``include/sbp.h``).  ``paper_2305_07181_amd.workloads`` holds the seeded
synthetic inputs.  Importing the package loads nothing native.
"""
