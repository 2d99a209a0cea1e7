"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the oracle tests, the GPU parity tests and the benchmark.  It holds
none of the method's arithmetic: only matrix generators (Haar-random factors,
prescribed spectra, noise, Gaussian-kernel matrices) and workload presets.

The paper's real matrices (smallnorb, ImageNet, Section 4) are not available;
these synthetic matrices stand in for them, including the paper's own
`polydecay` construction (Section 4: U diag(30000/i) V^T with random
orthogonal U, V).
"""
from .matrices import (haar, spectrum_matrix, lowrank_noise, psd_from_spectrum,  # noqa: F401
                       gauss_kernel, workload, WORKLOADS)
