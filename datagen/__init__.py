"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds input generation only: Gaussian-mixture point streams and
the workload descriptions (sizes, k, batch size, tunables).  It contains none
of the k-nn graph method's arithmetic, so that the oracle and the GPU path can
both draw identical inputs without sharing any of the method's code.
"""

from .gmm import GaussianMixture, u8_mixture, float_mixture, subspace_mixture  # noqa: F401
from .workloads import WORKLOADS, Workload, get_workload  # noqa: F401
