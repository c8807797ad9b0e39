"""Gaussian-mixture point streams (the synthetic data of the paper's
evaluation, "Synthetic dataset" subsection: points drawn from a mixture of
Gaussians, compared with Euclidean distance), generalised to the dimensions
and sizes of the workloads in :mod:`datagen.workloads`.

Every stream is a pure function of (mixture seed, stream seed, count), drawn
with NumPy's PCG64 ``default_rng``.  Cluster labels are uniform, so point ids
carry no information about cluster membership.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GaussianMixture:
    """A fixed mixture: ``centres[c]`` and per-cluster ``sigma[c]``.

    ``kind`` is ``"u8"`` (round half-to-even, clip to [0, 255], uint8) or
    ``"f32"`` (float32).  ``dim_scale`` (optional, shape [d]) multiplies every
    coordinate after sampling; it models heavy-tailed per-dimension scales.

    ``basis`` (optional, shape [C, d, r], orthonormal columns) makes every
    component r-dimensional: a point of component c is
    ``centres[c] + sigma[c] * basis[c] @ z`` with z ~ N(0, I_r), plus
    isotropic noise of standard deviation ``noise * sigma[c]`` in all d
    coordinates.  Without it a component is isotropic in all d coordinates.
    """

    centres: np.ndarray          # [C, d] float64
    sigma: np.ndarray            # [C] float64
    kind: str                    # "u8" | "f32"
    dim_scale: np.ndarray | None = None
    basis: np.ndarray | None = None      # [C, d, r]
    noise: float = 0.0

    @property
    def dim(self) -> int:
        return int(self.centres.shape[1])

    def sample(self, count: int, stream_seed: int, chunk: int = 1 << 16,
               with_labels: bool = False):
        """Draw ``count`` points from the mixture with its own stream seed.

        Drawing is chunked so that large streams do not need a float64 copy
        of the whole output; the chunking is part of the stream definition
        (labels, then noise, per chunk of ``chunk`` points).  With
        ``with_labels`` the mixture component of every point is returned too
        (the same stream: labels do not change the points).
        """
        rng = np.random.default_rng(stream_seed)
        d = self.dim
        out_dtype = np.uint8 if self.kind == "u8" else np.float32
        out = np.empty((count, d), dtype=out_dtype)
        labels = np.empty(count, dtype=np.int32) if with_labels else None
        C = self.centres.shape[0]
        for lo in range(0, count, chunk):
            hi = min(count, lo + chunk)
            lab = rng.integers(0, C, size=hi - lo)
            if labels is not None:
                labels[lo:hi] = lab
            sig = self.sigma[lab]
            if self.basis is None:
                x = self.centres[lab] + rng.standard_normal((hi - lo, d)) * sig[:, None]
            else:
                r = self.basis.shape[2]
                z = rng.standard_normal((hi - lo, r))
                x = self.centres[lab] + rng.standard_normal((hi - lo, d)) * (self.noise * sig)[:, None]
                for j in range(r):
                    x += (sig * z[:, j])[:, None] * self.basis[lab, :, j]
            if self.dim_scale is not None:
                x = x * self.dim_scale[None, :]
            if self.kind == "u8":
                out[lo:hi] = np.clip(np.rint(x), 0, 255).astype(np.uint8)
            else:
                out[lo:hi] = x.astype(np.float32)
        if with_labels:
            return out, labels
        return out


def u8_mixture(seed: int, n_clusters: int, dim: int, sigma: float,
               centre_lo: float = 40.0, centre_hi: float = 215.0) -> GaussianMixture:
    """Isotropic mixture with centres ~ U[centre_lo, centre_hi]^dim and one
    common sigma; samples are rounded (half to even) and clipped to uint8."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(centre_lo, centre_hi, size=(n_clusters, dim))
    return GaussianMixture(centres=centres, sigma=np.full(n_clusters, float(sigma)), kind="u8")


def float_mixture(seed: int, n_clusters: int, dim: int, sigma_lo: float = 0.05,
                  sigma_hi: float = 0.3, lognormal_dim_scale: float | None = None) -> GaussianMixture:
    """Mixture with centres ~ N(0, 1)^dim and per-cluster sigma ~ U[lo, hi].

    With ``lognormal_dim_scale = s``, every coordinate j is further multiplied
    by a shared scale ~ LogNormal(0, s) (heavy-tailed per-dimension scales).
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_clusters, dim))
    sig = rng.uniform(sigma_lo, sigma_hi, size=n_clusters)
    scale = None
    if lognormal_dim_scale is not None:
        scale = rng.lognormal(0.0, lognormal_dim_scale, size=dim)
    return GaussianMixture(centres=centres, sigma=sig, kind="f32", dim_scale=scale)


def subspace_mixture(seed: int, n_clusters: int, dim: int, rank: int, sigma_lo: float = 0.05,
                     sigma_hi: float = 0.3, noise: float = 0.05) -> GaussianMixture:
    """Mixture with centres ~ N(0, 1)^dim whose components are ``rank``-dimensional
    Gaussians (standard deviation sigma ~ U[lo, hi] along ``rank`` random
    orthonormal directions per component) plus isotropic noise of standard
    deviation ``noise * sigma`` in every coordinate."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_clusters, dim))
    sig = rng.uniform(sigma_lo, sigma_hi, size=n_clusters)
    g = rng.standard_normal((n_clusters, dim, rank))
    basis, _ = np.linalg.qr(g)
    return GaussianMixture(centres=centres, sigma=sig, kind="f32", basis=basis, noise=float(noise))
