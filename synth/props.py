"""Counter-based synthetic quark propagators.

Every real number is a function of (seed, stream, flat element index) only, so
any slice can be regenerated independently, on the host here or on the GPU by
``libsynth.so`` (same definition, bit-identical results):

  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC 2011) with key (seed low word, seed high word) and
    counter (low word, high word of n, stream, 0), where n = 2*e + r for the
    flat complex element e and r = 0 (real part) or 1 (imaginary part);
  * the four output words w_i give u_i = (w_i + 1/2) 2^-32 and the value
    g = (u_0 + u_1 + u_2 + u_3 - 2) * sqrt(3): an Irwin-Hall approximation of
    a standard normal variate (mean 0, variance 1).  Every step before the
    final product is exact in binary64, so host and device agree bit for bit;
  * the stored propagator entry is g * decay[t] with decay[t] = exp(-m t)
    evaluated once on the host, then rounded to the storage precision.

Array layout: [problem][t][site][source][row][col] complex, row = 3*spin +
colour at the sink, col = 3*spin + colour at the source.
"""
from __future__ import annotations

import math

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
SQRT3 = math.sqrt(3.0)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on uint32 counter words (numpy arrays)."""
    c0 = np.asarray(c0, np.uint64) & _MASK
    c1 = np.asarray(c1, np.uint64) & _MASK
    c2 = np.asarray(c2, np.uint64) & _MASK
    c3 = np.asarray(c3, np.uint64) & _MASK
    k0 = np.uint64(k0) & _MASK
    k1 = np.uint64(k1) & _MASK
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def gaussian_like(seed: int, stream: int, n0: int, count: int) -> np.ndarray:
    """Values g for counters n = n0 .. n0+count-1 (float64)."""
    n = np.arange(n0, n0 + count, dtype=np.uint64)
    w = philox4x32_10(n & _MASK, n >> np.uint64(32), np.full(count, stream, np.uint64), 0,
                      seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    s = sum((wi.astype(np.float64) + 0.5) * 2.0**-32 for wi in w)
    return (s - 2.0) * SQRT3


def decay(T: int, m: float) -> np.ndarray:
    return np.exp(-m * np.arange(T, dtype=np.float64))


def props(seed: int, stream: int, n_prob: int, T: int, V: int, nsrc: int, m: float = 0.5,
          dtype=np.complex128, probs=None, ts=None) -> np.ndarray:
    """Propagators [len(probs)][len(ts)][V][nsrc][12][12] for the selected
    problems and timeslices of a dataset of shape (n_prob, T, V, nsrc)."""
    probs = range(n_prob) if probs is None else probs
    ts = range(T) if ts is None else ts
    per_t = V * nsrc * 144
    dec = decay(T, m)
    out = np.empty((len(probs), len(ts), V, nsrc, 12, 12), dtype)
    for i, p in enumerate(probs):
        for j, t in enumerate(ts):
            e0 = (p * T + t) * per_t
            g = gaussian_like(seed, stream, 2 * e0, 2 * per_t).reshape(per_t, 2)
            z = (g[:, 0] * dec[t]) + 1j * (g[:, 1] * dec[t])
            out[i, j] = z.astype(dtype).reshape(V, nsrc, 12, 12)
    return out


def momentum_phase(L: int, p3: int) -> np.ndarray:
    """Sink weights exp(i 2 pi p3 x_3 / L) over the sites of an L^3 lattice
    (site index x = x_1 + L x_2 + L^2 x_3)."""
    x3 = np.arange(L**3) // (L * L)
    ph = 2.0 * np.pi * p3 * x3 / L
    return np.cos(ph) + 1j * np.sin(ph)


def mix_problems(seed: int, n: int, n_types: int, Ls=(16, 24, 32), Ts=(32, 64, 96)):
    """An uneven batch of n problems drawn by seed: for problem p the first
    three Philox words of counter (p, 0, MIX_STREAM, 0) pick a type index
    (of n_types), a lattice size from Ls and a time extent from Ts.  Returns
    a list of (type, L, T)."""
    w = philox4x32_10(np.arange(n, dtype=np.uint64), 0, MIX_STREAM, 0, seed & 0xFFFFFFFF,
                      (seed >> 32) & 0xFFFFFFFF)
    return [(int(w[0][p] % n_types), int(Ls[int(w[1][p] % len(Ls))]), int(Ts[int(w[2][p] % len(Ts))]))
            for p in range(n)]


MIX_STREAM = 0x4D495800   # stream word of the mix draw (propagator streams are small integers)
