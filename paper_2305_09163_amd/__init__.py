"""MI355X-native right-hand side of the two-fluid five-equation model
(WENO5-JS + HLLC + SSP-RK3) behind a C-ABI HIP library.

The HIP binding lives in ``paper_2305_09163_amd.mfc``; it is imported on
demand so that the seeded input generators in ``workloads`` can be used
without a GPU.
"""
