"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: it only draws integers.  The
same bytes feed the CPU oracle and the GPU library, so both sides see exactly
the same problem.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Output number ``i`` (0-based) of the stream
with seed ``s`` is ``mix(s + (i + 1) * GAMMA)`` with the published constants,
so any slice of the stream can be produced without producing the prefix.

Workloads (the paper benchmarks uniformly random square matrices over a prime
field; there is no public dataset to stand in for):

* ``uniform_residues``   entries uniform in [0, p), row-major draw order.
* ``centred_int8``       the same residues mapped to [-(p-1)/2, (p-1)/2] (p < 256).
* ``complex_residues``   F_{p^2} entries, real then imaginary part per element.
* ``batch_shapes``       n uniform in [32, 512], then k uniform in [n, 2n].
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: base seed; config c uses BASE_SEED + c
BASE_SEED = 2101010250


def config_seed(c: int) -> int:
    return BASE_SEED + int(c)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _draw_mod(seed: int, start: int, count: int, p: int, out: np.ndarray) -> None:
    chunk = 1 << 22
    pos = 0
    while pos < count:
        c = min(chunk, count - pos)
        out[pos:pos + c] = splitmix64(seed, start + pos, c) % np.uint64(p)
        pos += c


def uniform_residues(n: int, k: int, p: int, seed: int, start: int = 0,
                     dtype=np.int64) -> np.ndarray:
    """n x k row-major matrix of residues in [0, p) drawn from stream ``seed``."""
    flat = np.empty(n * k, dtype=dtype)
    _draw_mod(seed, start, n * k, p, flat)
    return flat.reshape(n, k)


def centred_int8(n: int, k: int, p: int, seed: int) -> np.ndarray:
    """Same draw as ``uniform_residues`` stored as int8 in [-(p-1)/2, (p-1)/2]."""
    if p >= 256:
        raise ValueError("centred int8 storage needs p < 256")
    r = uniform_residues(n, k, p, seed, dtype=np.int16)
    h = (p - 1) // 2
    r[r > h] -= p
    return r.astype(np.int8)


def to_centred(res: np.ndarray, p: int) -> np.ndarray:
    """Map canonical residues in [0,p) to the centred representative (storage change only)."""
    r = np.asarray(res).astype(np.int64)
    h = (p - 1) // 2
    return np.where(r > h, r - p, r)


def complex_residues(n: int, k: int, p: int, seed: int, dtype=np.int64):
    """F_{p^2} matrix: element (i,t) takes draws 2(ik+t) (real) and 2(ik+t)+1 (imaginary)."""
    flat = np.empty(2 * n * k, dtype=dtype)
    _draw_mod(seed, 0, 2 * n * k, p, flat)
    pairs = flat.reshape(n, k, 2)
    return np.ascontiguousarray(pairs[:, :, 0]), np.ascontiguousarray(pairs[:, :, 1])


def batch_shapes(count: int, seed: int, nmin: int = 32, nmax: int = 512):
    """Shapes of a batch: first all n_i = nmin + u mod (nmax-nmin+1), then k_i = n_i + u mod (n_i+1)."""
    u = splitmix64(seed, 0, count)
    ns = (np.uint64(nmin) + u % np.uint64(nmax - nmin + 1)).astype(np.int64)
    v = splitmix64(seed, count, count)
    ks = ns + (v % (ns.astype(np.uint64) + np.uint64(1))).astype(np.int64)
    return ns, ks


def batch_residues(ns, ks, p: int, seed: int, dtype=np.int64):
    """Entries of every problem of a batch, drawn after the 2*count shape draws, problem by problem."""
    out = []
    pos = 2 * len(ns)
    for n, k in zip(ns, ks):
        n, k = int(n), int(k)
        flat = np.empty(n * k, dtype=dtype)
        _draw_mod(seed, pos, n * k, p, flat)
        out.append(flat.reshape(n, k))
        pos += n * k
    return out
