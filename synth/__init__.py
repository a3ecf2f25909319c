"""Seeded synthetic inputs for multilevel NMF: planted Gaussian-blob image columns.

This module only draws data. It contains none of the factorization arithmetic
(no update rule, no transfer operator, no objective); both the HIP path and the
FP64 oracle receive its FP32 arrays as plain inputs.

Data model (stands in for the face / astronomy image sets of the paper's
experiments, Section 5 Table 2, which are not available here):

* r atoms V*[:, k] = exp(-((y - cy)^2 + (x - cx)^2) / (2 sigma^2)) on an h x w
  pixel grid, pixel (y, x) stored at row y * w + x (row-major image, one image
  per column); centres uniform over the grid, sigma uniform in [sig_lo, sig_hi],
  peak value 1.
* column j mixes k_j ~ U{k_lo..k_hi} (capped at r) distinct atoms with
  amplitudes W*[k, j] ~ U[0, 1].
* M = V* W* + |N(0, noise_std^2)|, then rounded to FP32.
* V0 ~ U[0, 1] (m x r) and W0 ~ U[0, 1] (r x n), FP32, no rescaling.

Draw order is fixed: atoms, codes, noise, V0, W0.

Layouts handed to both sides: M is m x n column-major (each column one image,
contiguous), V is m x r column-major, W is r x n row-major.  In numpy terms we
return M and V as Fortran-ordered float32 arrays and W as a C-ordered one, so
``M[i, j]``, ``V[i, k]``, ``W[k, j]`` index naturally.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class BlobSpec:
    h: int
    w: int
    n: int
    r: int
    k_lo: int
    k_hi: int
    sig_lo: float
    sig_hi: float
    noise_std: float = 0.01

    @property
    def m(self) -> int:
        return self.h * self.w


@dataclasses.dataclass
class Instance:
    spec: BlobSpec
    seed: int
    M: np.ndarray          # (m, n) float32, Fortran order
    V0: np.ndarray         # (m, r) float32, Fortran order
    W0: np.ndarray         # (r, n) float32, C order
    eps_E: float           # ||M - V* W*||_F / ||M||_F, exact planted-noise level
    Vstar: np.ndarray      # (m, r) float64 planted atoms
    Wstar: np.ndarray      # (r, n) float64 planted codes


# Workload shapes (the configurations the benchmark and tests use).
# 16x16 images, n=500, r=10, 3-8 blobs, sigma 1-4 px.
CFG_SMALL = BlobSpec(h=16, w=16, n=500, r=10, k_lo=3, k_hi=8, sig_lo=1.0, sig_hi=4.0)
# ORL-shaped: 112x92 images, n=400, r=40, 5-15 blobs, sigma 2-10 px.
CFG_ORL = BlobSpec(h=112, w=92, n=400, r=40, k_lo=5, k_hi=15, sig_lo=2.0, sig_hi=10.0)
# Large: 256x256 images, n=2000, r=50, 10-30 blobs, sigma 2-20 px.
CFG_LARGE = BlobSpec(h=256, w=256, n=2000, r=50, k_lo=10, k_hi=30, sig_lo=2.0, sig_hi=20.0)


def _atoms(rng: np.random.Generator, spec: BlobSpec) -> np.ndarray:
    h, w, r = spec.h, spec.w, spec.r
    cy = rng.uniform(0.0, h, size=r)
    cx = rng.uniform(0.0, w, size=r)
    sig = rng.uniform(spec.sig_lo, spec.sig_hi, size=r)
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    yy = yy.reshape(-1)
    xx = xx.reshape(-1)
    V = np.empty((h * w, r), dtype=np.float64)
    for k in range(r):
        V[:, k] = np.exp(-((yy - cy[k]) ** 2 + (xx - cx[k]) ** 2) / (2.0 * sig[k] ** 2))
    return V


def _codes(rng: np.random.Generator, spec: BlobSpec) -> np.ndarray:
    r, n = spec.r, spec.n
    W = np.zeros((r, n), dtype=np.float64)
    lo = min(spec.k_lo, r)
    hi = min(spec.k_hi, r)
    counts = rng.integers(lo, hi + 1, size=n)
    for j in range(n):
        idx = rng.choice(r, size=int(counts[j]), replace=False)
        W[idx, j] = rng.uniform(0.0, 1.0, size=idx.size)
    return W


def make_instance(spec: BlobSpec, seed: int) -> Instance:
    """Draw one planted instance; deterministic for (spec, seed)."""
    rng = np.random.default_rng(seed)
    Vs = _atoms(rng, spec)
    Ws = _codes(rng, spec)
    clean = Vs @ Ws
    noise = np.abs(rng.normal(0.0, spec.noise_std, size=clean.shape))
    M32 = np.asfortranarray((clean + noise).astype(np.float32))
    V0 = np.asfortranarray(rng.uniform(0.0, 1.0, size=(spec.m, spec.r)).astype(np.float32))
    W0 = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(spec.r, spec.n)).astype(np.float32))
    M64 = M32.astype(np.float64)
    eps = float(np.linalg.norm(M64 - clean) / np.linalg.norm(M64))
    return Instance(spec=spec, seed=seed, M=M32, V0=V0, W0=W0, eps_E=eps, Vstar=Vs, Wstar=Ws)


@dataclasses.dataclass(frozen=True)
class SpectralSpec:
    """Hyperspectral-like data: r abundance maps (Gaussian blobs on an h x w
    grid, as in BlobSpec) times r smooth spectra over n ordered bands (each a
    sum of 1-3 Gaussian bumps of width bw_lo..bw_hi bands), so columns vary
    smoothly with the band index (the case Section 6.1 names for coarsening
    n as well)."""
    h: int
    w: int
    n: int
    r: int
    sig_lo: float
    sig_hi: float
    bw_lo: float
    bw_hi: float
    noise_std: float = 0.01

    @property
    def m(self) -> int:
        return self.h * self.w


# 64x64 pixels, 256 bands, 12 materials
CFG_SPECTRAL = SpectralSpec(h=64, w=64, n=256, r=12, sig_lo=3.0, sig_hi=12.0, bw_lo=6.0,
                            bw_hi=30.0)


def make_spectral_instance(spec: SpectralSpec, seed: int) -> Instance:
    """Draw one planted spectral instance (draw order: maps, spectra, noise,
    V0, W0); deterministic for (spec, seed)."""
    rng = np.random.default_rng(seed)
    blob = BlobSpec(h=spec.h, w=spec.w, n=spec.n, r=spec.r, k_lo=1, k_hi=1,
                    sig_lo=spec.sig_lo, sig_hi=spec.sig_hi, noise_std=spec.noise_std)
    Vs = _atoms(rng, blob)
    t = np.arange(spec.n, dtype=np.float64)
    Ws = np.zeros((spec.r, spec.n), dtype=np.float64)
    for k in range(spec.r):
        for _ in range(int(rng.integers(1, 4))):
            c = rng.uniform(0.0, spec.n)
            bw = rng.uniform(spec.bw_lo, spec.bw_hi)
            Ws[k] += rng.uniform(0.2, 1.0) * np.exp(-((t - c) ** 2) / (2.0 * bw ** 2))
    clean = Vs @ Ws
    noise = np.abs(rng.normal(0.0, spec.noise_std, size=clean.shape))
    M32 = np.asfortranarray((clean + noise).astype(np.float32))
    V0 = np.asfortranarray(rng.uniform(0.0, 1.0, size=(spec.m, spec.r)).astype(np.float32))
    W0 = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(spec.r, spec.n)).astype(np.float32))
    M64 = M32.astype(np.float64)
    eps = float(np.linalg.norm(M64 - clean) / np.linalg.norm(M64))
    return Instance(spec=blob, seed=seed, M=M32, V0=V0, W0=W0, eps_E=eps, Vstar=Vs, Wstar=Ws)


@dataclasses.dataclass(frozen=True)
class TensorSpec:
    """Video-like 3-way data for NTF: r blob images (as in BlobSpec, mode 1 the
    h x w pixels) times r nonnegative profiles over J and over K (uniform in
    [0, 1]), plus |N(0, noise_std^2)| noise."""
    h: int
    w: int
    J: int
    K: int
    r: int
    sig_lo: float
    sig_hi: float
    noise_std: float = 0.01

    @property
    def m(self) -> int:
        return self.h * self.w


# 56x46 pixels, 20 x 20 other modes, rank 12
CFG_TENSOR = TensorSpec(h=56, w=46, J=20, K=20, r=12, sig_lo=2.0, sig_hi=8.0)


@dataclasses.dataclass
class TensorInstance:
    spec: TensorSpec
    seed: int
    X1: np.ndarray        # (m, J K) float32 Fortran: the mode-1 unfolding, column j + J k
    A0: np.ndarray        # (m, r) float32 Fortran
    Bt0: np.ndarray       # (r, J) float32 C
    Ct0: np.ndarray       # (r, K) float32 C
    eps_E: float          # ||X - [[A*, B*, C*]]||_F / ||X||_F of the planted factors


def make_tensor_instance(spec: TensorSpec, seed: int) -> TensorInstance:
    """Draw one planted tensor (draw order: images, B*, C*, noise, A0, B0, C0);
    deterministic for (spec, seed)."""
    rng = np.random.default_rng(seed)
    blob = BlobSpec(h=spec.h, w=spec.w, n=1, r=spec.r, k_lo=1, k_hi=3, sig_lo=spec.sig_lo,
                    sig_hi=spec.sig_hi, noise_std=spec.noise_std)
    As = _atoms(rng, blob)
    Bs = rng.uniform(0.0, 1.0, size=(spec.J, spec.r))
    Cs = rng.uniform(0.0, 1.0, size=(spec.K, spec.r))
    # column j + J k of the unfolding: A* (C*[k] * B*[j])
    kr = (Cs[:, None, :] * Bs[None, :, :]).reshape(spec.K * spec.J, spec.r)
    clean = As @ kr.T
    noise = np.abs(rng.normal(0.0, spec.noise_std, size=clean.shape))
    X1 = np.asfortranarray((clean + noise).astype(np.float32))
    A0 = np.asfortranarray(rng.uniform(0.0, 1.0, size=(spec.m, spec.r)).astype(np.float32))
    Bt0 = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(spec.r, spec.J)).astype(np.float32))
    Ct0 = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(spec.r, spec.K)).astype(np.float32))
    X64 = X1.astype(np.float64)
    eps = float(np.linalg.norm(X64 - clean) / np.linalg.norm(X64))
    return TensorInstance(spec=spec, seed=seed, X1=X1, A0=A0, Bt0=Bt0, Ct0=Ct0, eps_E=eps)


def uniform_pair(m: int, n: int, r: int, seed: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Plain U[0,1] FP32 (M, V0, W0) of arbitrary shape: unstructured test data."""
    rng = np.random.default_rng(seed)
    M = np.asfortranarray(rng.uniform(0.0, 1.0, size=(m, n)).astype(np.float32))
    V0 = np.asfortranarray(rng.uniform(0.0, 1.0, size=(m, r)).astype(np.float32))
    W0 = np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(r, n)).astype(np.float32))
    return M, V0, W0


def batch_specs(count: int, seed: int = 1000) -> list:
    """Uneven batch: sides in {16,32,48,64}, n ~ U{100..2000}, r ~ U{5..40};
    3-8 blobs with sigma in [1,4] * side/16.  Instance i uses seed ``seed + i``
    for its data; the shape draw uses its own generator so shapes do not depend
    on the data draws."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(rng.choice([16, 32, 48, 64]))
        n = int(rng.integers(100, 2001))
        r = int(rng.integers(5, 41))
        s = side / 16.0
        out.append((BlobSpec(h=side, w=side, n=n, r=r, k_lo=3, k_hi=8,
                             sig_lo=1.0 * s, sig_hi=4.0 * s), seed + i))
    return out


def column_subset(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded sorted subset of column indices (used to sample large outputs)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def scaled_copy(inst: Instance, factor: Optional[float] = None) -> Instance:
    """Same instance with M multiplied by a power of two (exact in FP32)."""
    f = 2.0 if factor is None else factor
    return dataclasses.replace(inst, M=np.asfortranarray((inst.M * np.float32(f))))
