"""SAQ oracle (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously-correct CPU implementation of what the SAQ encode
path computes, used to check the device path.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product library
never does.  It shares no code with the device path: the quantization plan is
read as data (segment widths and bits, projection matrix M, reference c).

Paper: SAQ (arXiv 2509.12086).
  * encode / estimate: ``saq_oracle.c`` (FP64, literal Algorithm 1; see its
    header for the section of the paper each step follows);
  * PCA fit: Section 4.1 (mean, covariance, eigen-decomposition sorted by
    decreasing variance) through ``numpy.linalg.eigh``;
  * plan search: Section 4.2, Eq. (seg-err) and Algorithm 2 (quantization
    plan search), plus the "fewest segments within 0.1 % of the minimum"
    selection stated after it.

Parity pins for each function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "saq_oracle.c")
_LIB = os.path.join(_HERE, "_saq_oracle.so")
MAX_ROUNDS = 64


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = load(_LIB)
    return _lib


def load(path: str):
    """ctypes handle on a compiled oracle library at `path` (the oracle's own
    build, or a copy with a planted mistake that a test compiled to check
    that the pins catch it)."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    L.saqo_quantize.argtypes = [P, i64, i32, i32, P, P, i32, P, P, P, P, P, ctypes.c_int]
    L.saqo_project.argtypes = [P, i64, i32, P, i32, P, P, P, ctypes.c_int]
    L.saqo_encode.argtypes = [P, i64, i32, P, i32, P, i32, P, P, i32, P, P, P, P, P, P, P,
                              ctypes.c_int]
    L.saqo_pack.argtypes = [P, i64, i32, i32, P, P, P, i64]
    L.saqo_estimate.argtypes = [P, i32, i32, P, i32, P, i32, P, P, P, P, P, i64, i32, P,
                                ctypes.c_int]
    L.saqo_estimate_multistage.argtypes = [P, i32, i32, P, i32, P, i32, P, P, P, P, P, i64,
                                           P, P, ctypes.c_double, P, P, P, P, ctypes.c_int]
    for f in ("saqo_quantize", "saqo_project", "saqo_encode", "saqo_pack", "saqo_estimate",
              "saqo_estimate_multistage"):
        getattr(L, f).restype = ctypes.c_int
    return L


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Encode (Section 3.1, Algorithm 1) -- thin wrappers over the C oracle
# --------------------------------------------------------------------------

@dataclass
class Encoded:
    codes: np.ndarray              # [n, Dk] int32
    factors: np.ndarray            # [n, k]  f_s = ||o_s||^2 / <u_s, o_s>
    norm2: Optional[np.ndarray]    # [n]     ||x - c||^2
    O: Optional[np.ndarray] = None         # [n, Dk] FP64 projection
    seg_aux: Optional[np.ndarray] = None   # [n, k, 4] v, Delta, <o_a,o_s>, ||o_s||^2
    code_aux: Optional[np.ndarray] = None  # [n, Dk, 2] init margin, decision margin
    round_stats: Optional[np.ndarray] = None  # [n, k, MAX_ROUNDS+1]


def _kept(widths: Sequence[int], bits: Sequence[int]):
    w = np.ascontiguousarray([int(a) for a, b in zip(widths, bits) if int(b) > 0], np.int32)
    b = np.ascontiguousarray([int(b) for b in bits if int(b) > 0], np.int32)
    return w, b


def quantize(O: np.ndarray, widths: Sequence[int], bits: Sequence[int], rounds: int,
             instrument: bool = False, threads: int = 0, library=None) -> Encoded:
    """Quantize projected rows O [n, Dk] (float64) segment by segment.
    ``widths``/``bits`` list the kept segments (bits > 0) in plan order.
    ``library`` (from ``load``) replaces the oracle's own build."""
    O = np.ascontiguousarray(O, np.float64)
    n, dk = O.shape
    w, b = _kept(widths, bits)
    k = w.size
    codes = np.zeros((n, dk), np.int32)
    fac = np.zeros((n, k), np.float64)
    sa = np.zeros((n, k, 4)) if instrument else None
    ca = np.zeros((n, dk, 2)) if instrument else None
    rs = np.zeros((n, k, MAX_ROUNDS + 1), np.int32) if instrument else None
    rc = (library or lib()).saqo_quantize(_p(O), n, dk, k, _p(w), _p(b), rounds, _p(codes),
                                          _p(fac), _p(sa), _p(ca), _p(rs), threads)
    if rc:
        raise ValueError("oracle quantize: bad arguments")
    return Encoded(codes, fac, None, O, sa, ca, rs)


def project(X: np.ndarray, M: np.ndarray, c: np.ndarray, threads: int = 0):
    """o = M (x - c) in FP64 (Eq. rotate) and ||x - c||^2."""
    X = np.ascontiguousarray(X, np.float32)
    M = np.ascontiguousarray(M, np.float32)
    c = np.ascontiguousarray(c, np.float32)
    n, d = X.shape
    O = np.zeros((n, M.shape[0]), np.float64)
    nn = np.zeros(n, np.float64)
    if lib().saqo_project(_p(X), n, d, _p(M), M.shape[0], _p(c), _p(O), _p(nn), threads):
        raise ValueError("oracle project: bad arguments")
    return O, nn


def encode(X: np.ndarray, M: np.ndarray, c: np.ndarray, widths: Sequence[int],
           bits: Sequence[int], rounds: int, instrument: bool = False,
           threads: int = 0) -> Encoded:
    """Project (FP64) then quantize every kept segment."""
    O, nn = project(X, M, c, threads)
    e = quantize(O, widths, bits, rounds, instrument, threads)
    e.norm2 = nn
    return e


def pack(codes: np.ndarray, widths: Sequence[int], bits: Sequence[int]) -> np.ndarray:
    """Bit-plane code string per vector (MSB plane first; dim i of a plane at
    byte i//8, bit i%8; a plane is ceil(W/8) bytes)."""
    codes = np.ascontiguousarray(codes, np.int32)
    w, b = _kept(widths, bits)
    cb = int(sum(int(bb) * ((int(ww) + 7) // 8) for ww, bb in zip(w, b)))
    out = np.zeros((codes.shape[0], cb), np.uint8)
    if lib().saqo_pack(_p(codes), codes.shape[0], codes.shape[1], w.size, _p(w), _p(b),
                       _p(out), cb):
        raise ValueError("oracle pack: bad arguments")
    return out


def estimate(Q: np.ndarray, M: np.ndarray, c: np.ndarray, widths, bits, codes: np.ndarray,
             factors: np.ndarray, norm2: np.ndarray, threads: int = 0,
             prefix_bits: int = 0) -> np.ndarray:
    """Estimated squared distances [nq, n] (Section 3.2); prefix_bits > 0
    uses the progressive approximation from the first min(prefix_bits, B)
    bits of every code."""
    Q = np.ascontiguousarray(Q, np.float32)
    M = np.ascontiguousarray(M, np.float32)
    c = np.ascontiguousarray(c, np.float32)
    codes = np.ascontiguousarray(codes, np.int32)
    factors = np.ascontiguousarray(factors, np.float64)
    norm2 = np.ascontiguousarray(norm2, np.float64)
    w, b = _kept(widths, bits)
    nq, n = Q.shape[0], codes.shape[0]
    out = np.zeros((nq, n), np.float64)
    if lib().saqo_estimate(_p(Q), nq, Q.shape[1], _p(M), M.shape[0], _p(c), w.size, _p(w),
                           _p(b), _p(codes), _p(factors), _p(norm2), n, int(prefix_bits),
                           _p(out), threads):
        raise ValueError("oracle estimate: bad arguments")
    return out


def estimate_multistage(Q: np.ndarray, M: np.ndarray, c: np.ndarray, widths, bits,
                        codes: np.ndarray, factors: np.ndarray, norm2: np.ndarray,
                        P: np.ndarray, lam: np.ndarray, m: float, tau: np.ndarray,
                        threads: int = 0):
    """Multi-stage estimator of Section 4.3: returns (d2 [nq, n], stage [nq, n],
    sigma [nq, k]).  A pair pruned before reading segment t has stage t and
    d2 = the stage-t lower bound; stage k means the full estimate.  P [Dk, D]
    are the kept PCA axes (unrotated, plan order) and lam [Dk] their
    variances; sigma_s^2 = sum_{i in s} lam_i (P_i (q - c))^2."""
    Q = np.ascontiguousarray(Q, np.float32)
    M = np.ascontiguousarray(M, np.float32)
    c = np.ascontiguousarray(c, np.float32)
    codes = np.ascontiguousarray(codes, np.int32)
    factors = np.ascontiguousarray(factors, np.float64)
    norm2 = np.ascontiguousarray(norm2, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    lam = np.ascontiguousarray(lam, np.float64)
    tau = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, np.float64), (Q.shape[0],)))
    w, b = _kept(widths, bits)
    nq, n = Q.shape[0], codes.shape[0]
    if P.shape != (M.shape[0], Q.shape[1]) or lam.shape != (M.shape[0],):
        raise ValueError("P must be [Dk, D] and lam [Dk]")
    d2 = np.zeros((nq, n), np.float64)
    stage = np.zeros((nq, n), np.int32)
    sigma = np.zeros((nq, w.size), np.float64)
    if lib().saqo_estimate_multistage(_p(Q), nq, Q.shape[1], _p(M), M.shape[0], _p(c), w.size,
                                      _p(w), _p(b), _p(codes), _p(factors), _p(norm2), n,
                                      _p(P), _p(lam), float(m), _p(tau), _p(d2), _p(stage),
                                      _p(sigma), threads):
        raise ValueError("oracle multi-stage estimate: bad arguments")
    return d2, stage, sigma


def true_dist2(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Exact squared Euclidean distances [nq, n] in FP64."""
    Q = np.asarray(Q, np.float64)
    X = np.asarray(X, np.float64)
    out = np.empty((Q.shape[0], X.shape[0]))
    for i in range(Q.shape[0]):
        diff = X - Q[i][None, :]
        out[i] = np.einsum("ij,ij->i", diff, diff)
    return out


def relative_error(d2_est: np.ndarray, d2_true: np.ndarray) -> np.ndarray:
    """|d2_est - d2| / d2 (Section 5, performance metrics)."""
    return np.abs(d2_est - d2_true) / d2_true


# --------------------------------------------------------------------------
# PCA fit (Section 4.1)
# --------------------------------------------------------------------------

def pca(X: np.ndarray):
    """Mean, covariance (1/N), eigenvalues (descending) and eigenvectors
    (columns) of the rows of X, all FP64."""
    X = np.asarray(X, np.float64)
    c = X.mean(axis=0)
    Y = X - c
    cov = Y.T @ Y / X.shape[0]
    lam, V = np.linalg.eigh(cov)
    order = np.argsort(-lam, kind="stable")
    return c, cov, lam[order], V[:, order]


# --------------------------------------------------------------------------
# Plan search (Section 4.2)
# --------------------------------------------------------------------------

def seg_error(sig2_sum: float, B: int) -> float:
    """Eq. (seg-err) without the constant 1/pi (it does not move the argmin):
    ERROR(Seg, B) = 2^-B * sum_{i in Seg} sigma_i^2."""
    return sig2_sum * 2.0 ** (-B)


@dataclass
class Plan:
    widths: List[int]
    bits: List[int]
    error: float
    cost: int
    quota: int
    min_error: float = field(default=float("nan"))

    @property
    def nseg(self) -> int:
        return len(self.widths)


def _units(D: int, g: int):
    w = [g] * (D // g)
    if D % g:
        w.append(D % g)
    return np.asarray(w, np.int64)


def quota_bits(bits_per_dim: float, D: int) -> int:
    """Q_quota = floor(B * D) (tiny slack for decimal budgets such as 0.2)."""
    return int(math.floor(bits_per_dim * D + 1e-9))


def _layer(prev, S, uw, qg, nq, max_bits, max_w_units):
    """One DP layer: append one segment (d, d'] with b bits to every plan of
    the previous layer (Algorithm 2's inner loops; cost update Q + b*(d'-d))."""
    nu = len(uw)
    cur = np.full((nu + 1, nq), np.inf)
    back = np.full((nu + 1, nq, 2), -1, np.int64)
    pos = np.concatenate([[0], np.cumsum(uw)])
    for d2 in range(1, nu + 1):
        for d in range(0, d2):
            width = int(pos[d2] - pos[d])
            src = prev[d]
            if not np.isfinite(src).any():
                continue
            ssum = S[d2] - S[d]
            for b in range(0, max_bits + 1):
                if b > 0 and max_w_units is not None and d2 - d > max_w_units:
                    continue
                cq = b * width // qg
                if cq >= nq:
                    continue
                cand = src[: nq - cq] + seg_error(ssum, b)
                tgt = cur[d2, cq:]
                better = cand < tgt
                if better.any():
                    idx = np.nonzero(better)[0]
                    tgt[idx] = cand[idx]
                    back[d2, cq + idx, 0] = d
                    back[d2, cq + idx, 1] = b
    return cur, back


def alg2(sig2: np.ndarray, bits_per_dim: float, g: int = 16, max_bits: int = 9,
         max_width: int = 0):
    """Algorithm 2 as stated: p[d, Q] is the best plan over the first d units
    using exactly Q bits; every existing p[d, Q] is extended by one segment
    (d, d'] with b' bits (cost Q + b' * |seg|); the answer is the best p[D, Q]
    over Q <= Q_quota.  Returns (minimum error, (widths, bits))."""
    sig2 = np.asarray(sig2, np.float64)
    D = sig2.size
    uw = _units(D, g)
    nu = len(uw)
    qg = int(np.gcd.reduce(uw))
    quota = quota_bits(bits_per_dim, D)
    nq = quota // qg + 1
    pos = np.concatenate([[0], np.cumsum(uw)])
    S = np.concatenate([[0.0], np.cumsum(sig2)])[pos]
    mwu = max_width // g if max_width else None
    E = np.full((nu + 1, nq), np.inf)
    E[0, 0] = 0.0
    back = np.full((nu + 1, nq, 2), -1, np.int64)
    for d in range(nu):
        if not np.isfinite(E[d]).any():
            continue
        for d2 in range(d + 1, nu + 1):
            width = int(pos[d2] - pos[d])
            for b in range(0, max_bits + 1):
                if b > 0 and mwu is not None and d2 - d > mwu:
                    continue
                cq = b * width // qg
                if cq >= nq:
                    continue
                cand = E[d, : nq - cq] + seg_error(S[d2] - S[d], b)
                tgt = E[d2, cq:]
                better = cand < tgt
                idx = np.nonzero(better)[0]
                tgt[idx] = cand[idx]
                back[d2, cq + idx, 0] = d
                back[d2, cq + idx, 1] = b
    q = int(np.argmin(E[nu]))
    err = float(E[nu, q])
    widths, bits = [], []
    d2 = nu
    while d2 > 0 and np.isfinite(err):
        d, b = back[d2, q]
        widths.append(int(pos[d2] - pos[d]))
        bits.append(int(b))
        q -= int(b) * int(pos[d2] - pos[d]) // qg
        d2 = int(d)
    return err, (widths[::-1], bits[::-1])



def plan_search(sig2: np.ndarray, bits_per_dim: float, g: int = 16, max_bits: int = 9,
                max_width: int = 0, seg_eps: float = 1e-3) -> Plan:
    """Algorithm 2 over g-dim units, then the fewest-segments selection:
    among plans whose modelled error is within (1 + seg_eps) of the minimum,
    take one with the fewest segments (and the least error among those).
    Widths of segments with bits > 0 are capped at ``max_width`` (0 = none)."""
    sig2 = np.asarray(sig2, np.float64)
    D = sig2.size
    uw = _units(D, g)
    nu = len(uw)
    qg = int(np.gcd.reduce(uw))
    quota = quota_bits(bits_per_dim, D)
    nq = quota // qg + 1
    pos = np.concatenate([[0], np.cumsum(uw)])
    S = np.concatenate([[0.0], np.cumsum(sig2)])[pos]
    mwu = None
    if max_width:
        if max_width % g:
            raise ValueError("max_width must be a multiple of g")
        mwu = max_width // g

    min_err, _ = alg2(sig2, bits_per_dim, g, max_bits, max_width)
    if not np.isfinite(min_err):
        raise ValueError("no feasible plan")
    layers, backs = [], []
    prev = np.full((nu + 1, nq), np.inf)
    prev[0, 0] = 0.0
    kstar = None
    # layer k holds the best plans with exactly k+1 segments; stop at the
    # first layer that gets within (1 + seg_eps) of the overall minimum
    for k in range(nu):
        cur, back = _layer(prev, S, uw, qg, nq, max_bits, mwu)
        layers.append(cur)
        backs.append(back)
        if float(cur[nu].min()) <= (1.0 + seg_eps) * min_err:
            kstar = k
            break
        prev = cur
    assert kstar is not None
    cur = layers[kstar]
    q = int(np.argmin(cur[nu]))
    # trace back
    widths, bits = [], []
    d2 = nu
    for k in range(kstar, -1, -1):
        d, b = backs[k][d2, q]
        widths.append(int(pos[d2] - pos[d]))
        bits.append(int(b))
        q -= int(b) * int(pos[d2] - pos[d]) // qg
        d2 = int(d)
    assert d2 == 0 and q == 0
    widths.reverse(); bits.reverse()
    err = sum(seg_error(S_(sig2, widths, i), bits[i]) for i in range(len(widths)))
    cost = sum(w * b for w, b in zip(widths, bits))
    return Plan(widths, bits, err, cost, quota, min_err)


def S_(sig2, widths, i):
    a = int(sum(widths[:i]))
    return float(np.sum(sig2[a:a + widths[i]]))


def plan_error(sig2: np.ndarray, widths: Sequence[int], bits: Sequence[int]) -> float:
    """Modelled error of a plan: sum over segments of Eq. (seg-err)."""
    return float(sum(seg_error(S_(np.asarray(sig2, np.float64), list(widths), i), int(bits[i]))
                     for i in range(len(widths))))
