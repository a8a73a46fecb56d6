"""MI355X-native fused finite-volume RHS and TVD-RK3 stage (arXiv:2402.05193 hot path).

Importing the package is cheap: the HIP library is loaded on first use by
``paper_2402_05193_amd.solver``.
"""
