"""Seeded synthetic workloads for the SAQ encode path.

This module is the only code shared by the device path's tests/benchmark and
the FP64 oracle.  It draws random numbers and shapes data; it holds none of the
method's arithmetic (no projection, quantization, adjustment or plan search).

Every dataset is a deterministic function of its seed: rows are produced in
fixed blocks of ``BLOCK`` rows, block ``b`` from its own PCG64 stream
``SeedSequence([seed, b])``, so any row range can be regenerated on its own
and the result does not depend on how the caller chunks the request.

Workload shapes follow the embedding datasets the paper measures on
(Section 5, dataset table: 1M x 960 image features, 1M-10M x 1024-1536 text
embeddings).  Those datasets are not available here; these generators stand in
for them with the anisotropic spectra that PCA-projected embeddings show
(Section 4.1: long-tailed per-dimension variance after PCA).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BLOCK = 4096


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def haar_rotation(d: int, seed: int) -> np.ndarray:
    """Haar-distributed d x d orthogonal matrix (QR of a Gaussian matrix with
    the sign of R's diagonal folded into Q; Mezzadri, Notices AMS 2007)."""
    g = _rng(seed, 0x5EED).standard_normal((d, d))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


@dataclasses.dataclass
class Dataset:
    """A synthetic dataset of ``n`` rows of dimension ``d`` (float32).

    kind:
      "spectrum"  x = R diag(sqrt(lam)) z,  z ~ N(0, I)
      "clusters"  x = R (mu_k + diag(std) z), k uniform over the centers,
                  mu_k ~ N(0, I)
    """
    name: str
    n: int
    d: int
    kind: str
    seed: int
    rot_seed: int
    lam: Optional[np.ndarray] = None      # per-dim variance ("spectrum")
    std: Optional[np.ndarray] = None      # per-dim within-cluster std ("clusters")
    n_centers: int = 0
    center_seed: int = 0
    query_seed: int = 0
    _rot: Optional[np.ndarray] = dataclasses.field(default=None, repr=False)
    _centers: Optional[np.ndarray] = dataclasses.field(default=None, repr=False)

    @property
    def rotation(self) -> np.ndarray:
        if self._rot is None:
            self._rot = haar_rotation(self.d, self.rot_seed)
        return self._rot

    @property
    def centers(self) -> np.ndarray:
        if self._centers is None:
            self._centers = _rng(self.center_seed, 0xC3).standard_normal(
                (self.n_centers, self.d))
        return self._centers

    def _block(self, seed: int, b: int) -> np.ndarray:
        g = _rng(seed, b)
        if self.kind == "spectrum":
            z = g.standard_normal((BLOCK, self.d)) * np.sqrt(self.lam)[None, :]
        elif self.kind == "clusters":
            ids = g.integers(0, self.n_centers, size=BLOCK)
            z = self.centers[ids] + g.standard_normal((BLOCK, self.d)) * self.std[None, :]
        else:
            raise ValueError(self.kind)
        return (z @ self.rotation.T).astype(np.float32)

    def _rows(self, seed: int, start: int, stop: int) -> np.ndarray:
        out = np.empty((max(stop - start, 0), self.d), np.float32)
        if stop <= start:
            return out
        b0, b1 = start // BLOCK, (stop - 1) // BLOCK
        pos = 0
        for b in range(b0, b1 + 1):
            blk = self._block(seed, b)
            lo = max(start, b * BLOCK) - b * BLOCK
            hi = min(stop, (b + 1) * BLOCK) - b * BLOCK
            out[pos:pos + hi - lo] = blk[lo:hi]
            pos += hi - lo
        return out

    def rows(self, start: int = 0, stop: Optional[int] = None) -> np.ndarray:
        """Data rows [start, stop) as a C-contiguous float32 array."""
        stop = self.n if stop is None else min(stop, self.n)
        return self._rows(self.seed, start, stop)

    def take(self, idx: np.ndarray) -> np.ndarray:
        """Arbitrary data rows by index (regenerates only the blocks needed)."""
        idx = np.asarray(idx, np.int64)
        out = np.empty((idx.size, self.d), np.float32)
        for b in np.unique(idx // BLOCK):
            sel = np.nonzero(idx // BLOCK == b)[0]
            out[sel] = self._block(self.seed, int(b))[idx[sel] - b * BLOCK]
        return out

    def rows_torch(self, n: int, device, seed_offset: int = 0):
        """n rows generated on a torch device (for full-size GPU runs): the
        same distribution and structure (rotation, centers, spectrum) as
        ``rows``, drawn from a seeded torch generator on that device.  The
        scaling, centers and rotation are applied in FP64 and rounded to FP32
        once, so the rows do not depend on which library GEMM kernel runs
        (only on the device type and torch version, through the normal
        draws).  Callers that need the values on the host copy them back from
        the returned tensor."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed(self.seed * 1_000_003 + seed_offset)
        R = torch.from_numpy(self.rotation.astype(np.float64)).to(device)
        out = torch.empty((n, self.d), dtype=torch.float32, device=device)
        step = 65536
        if self.kind == "clusters":
            C = torch.from_numpy(self.centers.astype(np.float64)).to(device)
            sd = torch.from_numpy(self.std.astype(np.float64)).to(device)
        else:
            sd = torch.from_numpy(np.sqrt(self.lam).astype(np.float64)).to(device)
        for a in range(0, n, step):
            b = min(n, a + step)
            z = torch.randn((b - a, self.d), generator=g, device=device).double() * sd
            if self.kind == "clusters":
                ids = torch.randint(0, self.n_centers, (b - a,), generator=g, device=device)
                z = z + C[ids]
            out[a:b] = (z @ R.T).float()
        return out

    def queries(self, nq: int) -> np.ndarray:
        """Held-out query rows from the same distribution (own seed)."""
        return self._rows(self.query_seed, 0, nq)


def exp_spectrum(d: int, tau: float) -> np.ndarray:
    return np.exp(-np.arange(d) / tau)


def power_spectrum(d: int, alpha: float) -> np.ndarray:
    return (np.arange(d) + 1.0) ** (-alpha)


def cfg1(n: int = 10_000) -> Dataset:
    """10k x 128 Gaussian, variance exp(-i/24), Haar-rotated (seeds 11/12)."""
    return Dataset("gauss_exp24_d128", n, 128, "spectrum", seed=11, rot_seed=12,
                   lam=exp_spectrum(128, 24.0), query_seed=13)


def cfg2(n: int = 1_000_000) -> Dataset:
    """1M x 960 mixture of 1024 Gaussian clusters (centers N(0, I),
    within-cluster std (i+1)^-0.5), Haar-rotated (seeds 21/22/23).
    Shaped like the paper's 1M x 960 image-feature dataset."""
    return Dataset("clusters1024_d960", n, 960, "clusters", seed=21, rot_seed=22,
                   std=(np.arange(960) + 1.0) ** -0.5, n_centers=1024,
                   center_seed=23, query_seed=24)


def cfg3(i: int, n: int = 1_000_000) -> Dataset:
    """Dataset i (0..3) of the batched case: 1M x 3072, variance (i+1)^-1.2."""
    return Dataset(f"power1.2_d3072_{i}", n, 3072, "spectrum", seed=31 + 2 * i,
                   rot_seed=32 + 2 * i, lam=power_spectrum(3072, 1.2),
                   query_seed=131 + i)


def cfg4(n: int = 200_000) -> Dataset:
    """Served-ingestion dataset: D=768, variance exp(-i/96)."""
    return Dataset("gauss_exp96_d768", n, 768, "spectrum", seed=41, rot_seed=42,
                   lam=exp_spectrum(768, 96.0), query_seed=43)


CFG5_DIMS = (128, 128, 768, 768, 1536, 1536, 3072, 3072)


def cfg5(i: int, n: int = 1_000_000) -> Dataset:
    """Dataset i (0..7) of the multi-dataset mix; D from CFG5_DIMS and an
    exponential spectrum whose decay length is D/8."""
    d = CFG5_DIMS[i]
    return Dataset(f"mix{i}_d{d}", n, d, "spectrum", seed=51 + i, rot_seed=151 + i,
                   lam=exp_spectrum(d, d / 8.0), query_seed=251 + i)


def poisson_requests(rate: float, seconds: float, seed: int = 41,
                     median: float = 512.0, sigma: float = 1.5,
                     lo: int = 1, hi: int = 65_536,
                     budgets=(2.0, 4.0, 6.0)):
    """Arrival trace: Poisson arrivals (exponential gaps), lognormal sizes
    clipped to [lo, hi], budget uniform over ``budgets``.
    Returns (arrival_s float64[k], size int64[k], budget float64[k])."""
    g = _rng(seed, 0xA11)
    k_max = int(rate * seconds * 1.5 + 100)
    gaps = g.exponential(1.0 / rate, size=k_max)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    k = t.size
    size = np.clip(np.round(g.lognormal(math.log(median), sigma, size=k)), lo, hi)
    bud = np.asarray(budgets)[g.integers(0, len(budgets), size=k)]
    return t, size.astype(np.int64), bud.astype(np.float64)


def segment_vectors(n: int, w: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) rows of width w (already-projected segment inputs)."""
    return (_rng(seed, 0x5E6).standard_normal((n, w)) * scale)
