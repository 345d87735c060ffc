"""Benchmark: equivalent n^2 k ops/s of Low(A A^T) mod p on one MI355X.

Default workload: n = k = 16384 over F_251, residues centred to [-125, 125]
as int8 (INT8 MFMA, exact int32 accumulation), output canonical uint8 —
the configuration the target "recursive INT8-MFMA beats the plain classical
GPU SYRK mod p at n = 16384" is stated on.  A step is one full call of the
library (conditioning if any, pre-additions, all products, post-additions) on
inputs already resident in HBM.  The same number of steps of the plain
classical modular SYRK (the same product kernel without recursion) is timed
beside it, and the CPU oracle on a bounded sample of the same workload.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0   # MI355X dense INT8 MFMA, tera-ops/s (2 ops per multiply-accumulate)
PEAK_F64_TFLOPS = 78.6    # MI355X FP64 matrix


WORKLOADS = {
    # name: (n, k, p, input, carrier description)
    # one level of Algorithm 1 at 16384^2 (the library's own choice there is now the classical
    # product, which this workload times beside it)
    "syrk_p251_int8": dict(n=16384, k=16384, p=251, dA="int8", carrier="int8 x1 limb", levels=1),
    "syrk_p251_int8_n32768": dict(n=32768, k=32768, p=251, dA="int8", carrier="int8 x1 limb"),
    "syrk_p65521_int8x2": dict(n=16384, k=16384, p=65521, dA="uint16", carrier="int8 x2 limbs"),
    "syrk_p65521_f64": dict(n=8192, k=8192, p=65521, dA="float64", carrier="fp64"),
    # the paper's two primes: 131071 = 3 mod 4 needs the 2x2-block Y, 131041 = 1 mod 4 a scalar Y
    "syrk_p131071_f64": dict(n=8192, k=8192, p=131071, dA="float64", carrier="fp64"),
    "syrk_p131041_f64": dict(n=8192, k=8192, p=131041, dA="float64", carrier="fp64"),
    "herk_p65519_int8x2": dict(n=4096, k=8192, p=65519, dA="uint16", carrier="int8 x2 limbs, complex"),
    # 4096 independent problems, n uniform in [32, 512], k uniform in [n, 2n]
    "batch4096_p65521": dict(count=4096, nmin=32, nmax=512, p=65521, dA="uint16",
                             carrier="autotuned"),
    # the small case: one recursion level over a classical base case, int64 storage; the
    # host figures are process CPU-seconds of the oracle and of the one-level model
    "syrk_p65521_n256_int64": dict(n=256, k=256, p=65521, dA="int64", carrier="int8 x2 limbs",
                                   levels=1, cpu_seconds=True),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="syrk_p251_int8", choices=sorted(WORKLOADS))
    ap.add_argument("--levels", type=int, default=-1, help="recursion depth (-1: library default)")
    ap.add_argument("--kernel", type=int, default=0,
                    help="INT8 product-kernel configuration + 1 for both plans (0: built-in choice)")
    ap.add_argument("--general", choices=["auto", "classical", "winograd"], default="auto",
                    help="general products P3, P4: one task, or one level of Strassen-Winograd")
    ap.add_argument("--wino-min", type=int, default=0,
                    help="Strassen-Winograd only on general products of at least this many rows "
                         "(0: the library's choice)")
    ap.add_argument("--herk-base", choices=["auto", "2m", "4m"], default="auto",
                    help="Hermitian base case: the 2M method or four real products")
    ap.add_argument("--streams", choices=["auto", "one", "two"], default="auto",
                    help="run the pre-additions and dependent products on a second stream")
    ap.add_argument("--no-classical", action="store_true", help="skip the classical comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB buffer three times (scale for FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size, profiled to scale the HBM byte counters."""
    import torch
    x = torch.empty(256 * 1024 * 1024, dtype=torch.uint8, device="cuda")
    x.fill_(3)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 256 * 1024 * 1024, "copies": 3}))


PROFILE_FILE = os.path.join(ROOT, "profiles", "gemm_i8_syrk_p251_n16384.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2101_01025_amd", "csrc", f)
                  for f in ("gemm_i8_kernel.h", "gemm_i8_configs.h", "device_common.h", "ffa_internal.h")]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, levels):
    """HBM bytes per product launch from the committed rocprofv3 counters, or None
    when the kernel sources changed since they were taken (or no record matches)."""
    import re
    try:
        text = open(PROFILE_FILE).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    if rec.get("workload") != workload or rec.get("levels") != levels:
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def make_input(w, torch):
    """Device inputs of the workload and their host copies (for the result check)."""
    import numpy as np

    import seeded_inputs as si
    n, k, p = w["n"], w["k"], w["p"]
    seed = si.config_seed(2)
    if w["dA"] == "int8":
        a = si.centred_int8(n, k, p, seed)
        return torch.from_numpy(a).to("cuda"), None, a, None
    if w["dA"] == "int64":
        a = si.uniform_residues(n, k, p, si.config_seed(0))
        return torch.from_numpy(a).to("cuda"), None, a, None
    if w["dA"] == "uint16":
        if w["name"].startswith("herk"):
            ar, ai = si.complex_residues(n, k, p, si.config_seed(4), dtype=np.int32)
            return (torch.from_numpy(ar).to("cuda").to(torch.uint16),
                    torch.from_numpy(ai).to("cuda").to(torch.uint16), ar, ai)
        a = si.uniform_residues(n, k, p, seed, dtype=np.int32)
        return torch.from_numpy(a).to("cuda").to(torch.uint16), None, a, None
    a = si.uniform_residues(n, k, p, si.config_seed(1), dtype=np.float64)
    return torch.from_numpy(a).to("cuda"), None, a, None


def timed_steps(ffa, torch, w, A, Ai, C, Ci, plans, steps, warmup, blocks=10):
    """Times each plan (recursive, then classical if given) three ways.

    (a) Exactly `steps` calls in one region bracketed by a device synchronisation
        and two HIP events on the current stream: ms per step = region time / steps
        (the headline figure).
    (b) The same number of calls in `blocks` blocks, each bracketed the same way,
        the plans alternating block by block: the median of the blocks' ms per call.
    (c) `steps` calls in one region with the library's HIP events around the product
        phase (the grouped product launch and its last-round sums) on the same
        stream: its ms per call, for the roofline, and the region's ms per step (the
        events themselves cost each call some microseconds, so (a) has none).
    Nothing is flushed between calls: the inputs and the workspace stay in HBM (and
    partly in the 256 MB MALL) from one call to the next, as in a loop of calls on
    resident data.
    Returns per plan: (ms per step (a), median ms per call (b), product-phase ms per
    call (c), ms per step of region (c)).
    """
    import statistics

    def one(opts):
        if Ai is None:
            ffa.syrk_modp(A, w["p"], C=C, opts=opts)
        else:
            ffa.herk_modp2(A, Ai, w["p"], C_re=C, C_im=Ci, opts=opts)

    def region(opts, n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            one(opts)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    for opts in plans:
        for _ in range(warmup):
            one(opts)
    torch.cuda.synchronize()
    headline = [region(opts, steps) / steps for opts in plans]
    blocks = max(1, min(blocks, steps))
    per_block = [steps // blocks + (1 if b < steps % blocks else 0) for b in range(blocks)]
    block_ms = [[] for _ in plans]
    for nb in per_block:
        for i, opts in enumerate(plans):
            block_ms[i].append(region(opts, nb) / nb)
    prod = []
    for opts in plans:
        ffa.profile_reset(0)
        ffa.profile_enable(0, True, phases=1 << ffa.PHASE_PRODUCTS)
        t = region(opts, steps)
        ffa.profile_enable(0, False)
        prod.append((ffa.profile_read(0, ffa.PHASE_PRODUCTS)[0] / steps, t / steps))
    # a product tile that waited in vain for the pre-additions beside it would have
    # made its call's result invalid: none did, or the benchmark stops here
    ffa.device_status(0)
    return [(headline[i], statistics.median(block_ms[i]), prod[i][0], prod[i][1]) for i in range(len(plans))]


def phase_breakdown(ffa, torch, w, A, Ai, C, Ci, opts, calls=5):
    """ms per call of each phase (HIP events around every phase) over `calls` calls
    outside the timed region."""
    names = ((ffa.PHASE_COND, "conditioning"), (ffa.PHASE_PRE, "preadd"),
             (ffa.PHASE_PRODUCTS, "products"), (ffa.PHASE_POST, "postadd"))
    torch.cuda.synchronize()
    ffa.profile_reset(0)
    ffa.profile_enable(0, True)
    for _ in range(calls):
        if Ai is None:
            ffa.syrk_modp(A, w["p"], C=C, opts=opts)
        else:
            ffa.herk_modp2(A, Ai, w["p"], C_re=C, C_im=Ci, opts=opts)
    torch.cuda.synchronize()
    ffa.profile_enable(0, False)
    out = {}
    for ph, name in names:
        ms, _ = ffa.profile_read(0, ph)
        out[name] = round(ms / calls, 4)
    return out


# ---------------------------------------------------------------- result checks
# After the timed region every plan runs once more into a C filled with a value
# that is not a residue, and the result is checked on the host from the
# definition itself (this is not the oracle): canonical residues everywhere in the
# lower triangle, the strict upper triangle untouched, sampled entries
# C_ij = sum_t A_it A_jt mod p, and Freivalds' test Sym(C) X = A (A^T X) mod p
# for four random vectors (a wrong C passes with probability at most p^-4).
# Every sum is formed in float64 from integers whose sums stay below 2^53, so
# the host arithmetic is exact.

VECTORS = 4
CHUNK = 2048


class VerifyError(RuntimeError):
    pass


def _f64(a):
    import numpy as np
    return np.asarray(a, dtype=np.float64)


def _modp(x, p):
    import numpy as np
    return np.mod(np.rint(x), p)


def _pairs(n, rng, count=2000):
    import numpy as np
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    i, j = np.maximum(i, j), np.minimum(i, j)
    edges = [0, 1, n - 2, n - 1]
    for q in (2, 4, 8):
        b = n // q
        edges += [b - 1, b, b + 1]
    e = np.unique(np.clip(np.array(edges), 0, n - 1))
    ei, ej = np.meshgrid(e, e)
    m = ei >= ej
    return np.concatenate([i, ei[m]]), np.concatenate([j, ej[m]])


def _sym_times(L, X, p):
    """Sym(L) X mod p for the lower triangle L (n x n, host) of a symmetric matrix."""
    import numpy as np
    n = L.shape[0]
    Y = np.zeros((n, X.shape[1]))
    for r0 in range(0, n, CHUNK):
        r1 = min(n, r0 + CHUNK)
        B = np.tril(_f64(L[r0:r1, :r1]), r0)          # rows r0..r1-1, columns j <= i
        Y[r0:r1] += B @ X[:r1]
        Bs = np.tril(B, r0 - 1)                        # j < i: the mirrored part
        Y[:r1] += Bs.T @ X[r0:r1]
    return _modp(Y, p)


def _herm_times(Lr, Li, Xr, Xi, p):
    """Herm(L) X mod p for the lower triangle L = Lr + i Li of a Hermitian matrix."""
    import numpy as np
    n = Lr.shape[0]
    Yr, Yi = np.zeros((n, Xr.shape[1])), np.zeros((n, Xr.shape[1]))
    for r0 in range(0, n, CHUNK):
        r1 = min(n, r0 + CHUNK)
        Br = np.tril(_f64(Lr[r0:r1, :r1]), r0)
        Bi = np.tril(_f64(Li[r0:r1, :r1]), r0)
        Yr[r0:r1] += Br @ Xr[:r1] - Bi @ Xi[:r1]
        Yi[r0:r1] += Br @ Xi[:r1] + Bi @ Xr[:r1]
        Sr, Si = np.tril(Br, r0 - 1), np.tril(Bi, r0 - 1)   # conj(L_ji) above the diagonal
        Yr[:r1] += Sr.T @ Xr[r0:r1] + Si.T @ Xi[r0:r1]
        Yi[:r1] += Sr.T @ Xi[r0:r1] - Si.T @ Xr[r0:r1]
    return _modp(Yr, p), _modp(Yi, p)


def _rows_times(A, X):
    """A X (A: n x k host residues, X: k x v float64), in row chunks."""
    import numpy as np
    out = np.zeros((A.shape[0], X.shape[1]))
    for r0 in range(0, A.shape[0], CHUNK):
        out[r0:r0 + CHUNK] = _f64(A[r0:r0 + CHUNK]) @ X
    return out


def _cols_times(A, X):
    """A^T X (A: n x k host residues, X: n x v float64), in row chunks."""
    import numpy as np
    out = np.zeros((A.shape[1], X.shape[1]))
    for r0 in range(0, A.shape[0], CHUNK):
        out += _f64(A[r0:r0 + CHUNK]).T @ X[r0:r0 + CHUNK]
    return out


def _lower_checks(Ch, p, sentinel, rng):
    import numpy as np
    n = Ch.shape[0]
    for r0 in range(0, n, CHUNK):
        blk = Ch[r0:r0 + CHUNK]
        rows = np.arange(r0, r0 + blk.shape[0])[:, None]
        cols = np.arange(n)[None, :]
        low = cols <= rows
        v = blk[low]
        if v.size and (v.min() < 0 or v.max() >= p):
            raise VerifyError(f"non-canonical entry in the lower triangle (rows {r0}..)")
        if not (blk[~low] == sentinel).all():
            raise VerifyError(f"strict upper triangle written (rows {r0}..)")


def verify_syrk(A_host, p, C_dev, sentinel, seed):
    """Checks the lower triangle of C = Low(A A^T) mod p computed on the device.
    A_host: n x k residues or centred residues (congruent mod p)."""
    import numpy as np
    n, k = A_host.shape
    amax = float(np.abs(A_host).max()) if A_host.size else 0.0
    if max(n, k) * amax * (p - 1) >= 2.0 ** 53 or k * amax * amax >= 2.0 ** 53:
        raise VerifyError("host check would not be exact in float64")
    rng = np.random.default_rng(seed)
    Ch = C_dev.cpu().numpy()
    if Ch.dtype == np.uint16:
        Ch = Ch.astype(np.int32)
    _lower_checks(Ch, p, sentinel, rng)
    ii, jj = _pairs(n, rng)
    got = Ch[ii, jj].astype(np.int64)
    exp = np.empty(len(ii), dtype=np.int64)
    for s0 in range(0, len(ii), 256):
        a = _f64(A_host[ii[s0:s0 + 256]])
        b = _f64(A_host[jj[s0:s0 + 256]])
        exp[s0:s0 + 256] = _modp((a * b).sum(1), p).astype(np.int64)
    if not np.array_equal(got, exp):
        bad = int(np.argmax(got != exp))
        raise VerifyError(f"entry ({ii[bad]}, {jj[bad]}) = {got[bad]}, expected {exp[bad]}")
    X = rng.integers(0, p, (n, VECTORS)).astype(np.float64)
    W = _modp(_cols_times(A_host, X), p)
    Ya = _modp(_rows_times(A_host, W), p)
    Yc = _sym_times(Ch, X, p)
    if not np.array_equal(Ya, Yc):
        raise VerifyError("Freivalds check failed")
    return {"entries": int(len(ii)), "freivalds_vectors": VECTORS}


def verify_herk(Ar, Ai, p, Cr_dev, Ci_dev, sentinel, seed):
    """Checks Low(A A^H) over F_p[i]/(i^2+1) (planar re/im) computed on the device."""
    import numpy as np
    n, k = Ar.shape
    if 2 * max(n, k) * float(p - 1) ** 2 >= 2.0 ** 53:
        raise VerifyError("host check would not be exact in float64")
    rng = np.random.default_rng(seed)
    Cr = Cr_dev.cpu().numpy().astype(np.int64)
    Ci = Ci_dev.cpu().numpy().astype(np.int64)
    _lower_checks(Cr, p, sentinel, rng)
    _lower_checks(Ci, p, sentinel, rng)
    if (np.diagonal(Ci) != 0).any():
        raise VerifyError("nonzero imaginary part on the diagonal")
    ii, jj = _pairs(n, rng)
    er = np.empty(len(ii), dtype=np.int64)
    ei = np.empty(len(ii), dtype=np.int64)
    for s0 in range(0, len(ii), 256):
        xr, xi = _f64(Ar[ii[s0:s0 + 256]]), _f64(Ai[ii[s0:s0 + 256]])
        yr, yi = _f64(Ar[jj[s0:s0 + 256]]), _f64(Ai[jj[s0:s0 + 256]])
        er[s0:s0 + 256] = _modp((xr * yr + xi * yi).sum(1), p)
        ei[s0:s0 + 256] = _modp((xi * yr - xr * yi).sum(1), p)
    if not (np.array_equal(Cr[ii, jj], er) and np.array_equal(Ci[ii, jj], ei)):
        raise VerifyError("sampled entries differ")
    Xr = rng.integers(0, p, (n, VECTORS)).astype(np.float64)
    Xi = rng.integers(0, p, (n, VECTORS)).astype(np.float64)
    # A (A^H X): W = A^H X = (Ar^T Xr + Ai^T Xi) + i (Ar^T Xi - Ai^T Xr)
    Wr = _modp(_cols_times(Ar, Xr) + _cols_times(Ai, Xi), p)
    Wi = _modp(_cols_times(Ar, Xi) - _cols_times(Ai, Xr), p)
    Yar = _modp(_rows_times(Ar, Wr) - _rows_times(Ai, Wi), p)
    Yai = _modp(_rows_times(Ar, Wi) + _rows_times(Ai, Wr), p)
    Ycr, Yci = _herm_times(Cr, Ci, Xr, Xi, p)
    if not (np.array_equal(Yar, Ycr) and np.array_equal(Yai, Yci)):
        raise VerifyError("Freivalds check failed")
    return {"entries": int(len(ii)), "freivalds_vectors": VECTORS}


def verify_batch(mats, c_off, ns, p, C_dev, sentinel, seed, whole=64):
    """Every problem of a batch: Freivalds with four vectors, canonical lower
    triangle, untouched upper triangle; `whole` of them compared entry by entry
    with the product formed on the host."""
    import numpy as np
    rng = np.random.default_rng(seed)
    Ch = C_dev.cpu().numpy().astype(np.int64)
    full = set(rng.choice(len(ns), min(whole, len(ns)), replace=False).tolist())
    for i, M in enumerate(mats):
        n = int(ns[i])
        if n == 0:
            continue
        G = Ch[c_off[i]:c_off[i] + n * n].reshape(n, n)
        low = np.tril(np.ones((n, n), dtype=bool))
        if G[low].min() < 0 or G[low].max() >= p or not (G[~low] == sentinel).all():
            raise VerifyError(f"problem {i}: non-canonical or upper triangle written")
        Mf = _f64(M)
        if i in full:
            if not np.array_equal(G[low], _modp(Mf @ Mf.T, p).astype(np.int64)[low]):
                raise VerifyError(f"problem {i} differs")
            continue
        X = rng.integers(0, p, (n, VECTORS)).astype(np.float64)
        Ya = _modp(Mf @ _modp(Mf.T @ X, p), p)
        if not np.array_equal(Ya, _sym_times(G, X, p)):
            raise VerifyError(f"problem {i}: Freivalds check failed")
    return {"problems": int(len(ns)), "compared_whole": len(full), "freivalds_vectors": VECTORS}


def run_batch(args, w, ffa, torch):
    """The batched workload: one plan for all problems, autotuned (carrier, product
    kernel, recursion cutoff) before the timed region, executed as one captured
    hipGraph per step.  Phase durations come from separate profiled blocks of the
    same plan (profiling launches the kernels directly, one HIP event pair per
    phase), interleaved with the graph blocks."""
    import numpy as np

    import seeded_inputs as si
    p = w["p"]
    seed = si.config_seed(3)
    ns, ks = si.batch_shapes(w["count"], seed, nmin=w["nmin"], nmax=w["nmax"])
    mats = si.batch_residues(ns, ks, p, seed, dtype=np.uint16)
    eq_ops = float((ns.astype(np.float64) ** 2 * ks).sum())
    B = ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16)
    Ap = B.pack(mats, np.uint16)
    A = torch.from_numpy(Ap.astype(np.int32)).to("cuda").to(torch.uint16)
    del Ap
    C = torch.zeros(B.c_total, dtype=torch.int32, device="cuda").to(torch.uint16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, tuned_ms = B.autotune(A, C, reps=3)
    tune_s = time.perf_counter() - t0
    plan = B.describe()
    Bc = None if args.no_classical else ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16,
                                                      algo=ffa.ALGO_CLASSICAL)
    runs = [B] + ([Bc] if Bc is not None else [])
    for b in runs:
        for _ in range(args.warmup):
            b.run(A, C)
    torch.cuda.synchronize()
    blocks = max(1, min(10, args.steps))
    per_block = [args.steps // blocks + (1 if i < args.steps % blocks else 0) for i in range(blocks)]
    total = [0.0] * len(runs)
    per_step = [[] for _ in runs]
    prof_ms, prof_calls = 0.0, 0
    phase_tot = {}
    names = ((ffa.PHASE_COND, "conditioning"), (ffa.PHASE_PRE, "preadd"),
             (ffa.PHASE_PRODUCTS, "products"), (ffa.PHASE_POST, "postadd"))
    for nb in per_block:
        if nb == 0:
            continue
        for i, b in enumerate(runs):
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record()
            for _ in range(nb):
                b.run(A, C)
            stop.record()
            torch.cuda.synchronize()
            total[i] += start.elapsed_time(stop)
            per_step[i].append(start.elapsed_time(stop) / nb)
        # profiled block of the tuned plan (direct launches, phase events)
        ffa.profile_reset(0)
        ffa.profile_enable(0, True)
        for _ in range(nb):
            B.run(A, C)
        torch.cuda.synchronize()
        ffa.profile_enable(0, False)
        for ph, name in names:
            ms_, calls = ffa.profile_read(0, ph)
            phase_tot[name] = phase_tot.get(name, 0.0) + ms_
        prof_calls += nb
    ms = total[0] / args.steps
    phases = {name: round(phase_tot[name] / prof_calls, 4) for _, name in names}
    # the result of each plan, checked on the host after the timed region
    import statistics
    checked = {}
    for name, b in (("tuned", B), ("classical", Bc)):
        if b is None:
            continue
        C.fill_(0xFFFF)
        b.run(A, C)
        torch.cuda.synchronize()
        checked[name] = verify_batch(mats, B.c_off, ns, p, C, 0xFFFF, 77)
    out = {
        "metric": "equivalent n^2k ops/s for A*A^T mod p (bit-exact)",
        "value": eq_ops / (ms * 1e-3),
        "unit": "n^2k/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_median": statistics.median(per_step[0]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if plan["carrier"] == "int8" else "f64",
        "data": "synthetic",
        "verified": checked,
        "config": {"workload": f"batch of {w['count']} syrk problems, n in [{w['nmin']},{w['nmax']}], "
                               f"k in [n,2n], p={p}, input=uint16, one hipGraph launch per step",
                   "count": w["count"], "p": p, "sum_n2k": eq_ops,
                   "levels_max": plan["levels"], "limbs": plan["limbs"],
                   "carrier": plan["carrier"], "parallelism": "single GPU"},
        "autotune": {"choice": best.as_dict(), "ms": tuned_ms, "seconds": round(tune_s, 2)},
        "phases_ms": phases,
    }
    ops = 2.0 * plan["macs"] * plan["limbs"] ** 2
    achieved = ops / (phases["products"] * 1e-3) / 1e12
    peak = PEAK_INT8_TOPS if plan["carrier"] == "int8" else PEAK_F64_TFLOPS
    out["roofline"] = {"bound": "mfma", "kernel": f"gemm_{'i8' if plan['carrier'] == 'int8' else 'f64'} "
                                                  "(grouped products, all problems in one launch)",
                       "achieved": achieved, "peak": peak,
                       "unit": "TOP/s" if plan["carrier"] == "int8" else "TFLOP/s",
                       "frac": achieved / peak, "traffic": None, "ops_per_step": ops}
    if Bc is not None:
        cms = total[1] / args.steps
        out["classical_gpu"] = {"value": eq_ops / (cms * 1e-3), "unit": "n^2k/s", "ms_per_step": cms,
                                "ms_median": statistics.median(per_step[1])}
        out["speedup_vs_classical"] = cms / ms
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(ns, ks, p, seed, args.cpu_seconds, eq_ops)
    B.close()
    if Bc is not None:
        Bc.close()
    return out


def cpu_baseline_batch(ns, ks, p, seed, seconds, eq_ops):
    """The oracle, unchanged, on the batch's problems in order until about
    `seconds` of CPU time; rate = their n^2 k over that time."""
    import oracle
    import seeded_inputs as si
    mats = si.batch_residues(ns[:512], ks[:512], p, seed)
    done, t = 0.0, 0.0
    count = 0
    for i, M in enumerate(mats):
        t0 = time.perf_counter()
        oracle.syrk_modp(M, p)
        t += time.perf_counter() - t0
        done += float(ns[i]) ** 2 * float(ks[i])
        count += 1
        if t > seconds:
            break
    return {"value": done / t, "unit": "n^2k/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the first {count} problems of the batch ({done / eq_ops:.3%} of its n^2k), "
                      f"{t:.2f} s"}


def cpu_baseline(w, seconds):
    """The oracle, unchanged, on the leading m x k rows (lower triangle of the
    leading m x m block of C): m(m+1)/2 * k of the n(n+1)/2 * k multiply-adds."""
    import numpy as np

    import oracle
    import seeded_inputs as si
    n, k, p = w["n"], w["k"], w["p"]
    herm = w["name"].startswith("herk")
    m = 256
    while True:
        if herm:
            ar, ai = si.complex_residues(m, k, p, si.config_seed(4))
            t0 = time.perf_counter()
            oracle.herk_modp2(ar, ai, p)
        else:
            a = si.uniform_residues(m, k, p, si.config_seed(2))
            t0 = time.perf_counter()
            oracle.syrk_modp(a, p)
        t = time.perf_counter() - t0
        # the timed sample itself is the baseline: keep growing it to about `seconds`
        if t > 0.6 * seconds or m >= n:
            break
        m = min(n, int(m * max(1.3, min(4.0, (seconds / max(t, 1e-3)) ** 0.5))))
    frac = (m * (m + 1) / 2) / (n * (n + 1) / 2)
    t_full = t / frac
    return {"value": n * n * k / t_full, "unit": "n^2k/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"lower triangle of the leading {m}x{m} block (rows 0..{m - 1}, full k={k}), "
                      f"{t:.2f} s, scaled by n(n+1)/(m(m+1))"}


def cpu_seconds_small(w, reps=5):
    """Process CPU-seconds (CLOCK_PROCESS_CPUTIME_ID, all threads) of the oracle and of
    the plain model of Algorithm 1 with one recursion level, on the workload itself
    (median of `reps` runs each)."""
    import statistics

    import oracle
    from oracle import alg1_model
    import seeded_inputs as si
    a = si.uniform_residues(w["n"], w["k"], w["p"], si.config_seed(0))

    def cpu(f):
        ts = []
        for _ in range(reps):
            t0 = time.process_time()
            f()
            ts.append(time.process_time() - t0)
        return statistics.median(ts)
    return {"oracle_cpu_s": cpu(lambda: oracle.syrk_modp(a, w["p"])),
            "alg1_one_level_model_cpu_s": cpu(lambda: alg1_model.syrk(a, w["p"], 1)),
            "oracle_threads": oracle.num_threads(), "reps": reps, "clock": "process CPU time"}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (use --gpus 1); "
                                   "the multi-GPU design is described, not built"}))
        sys.exit(2)
    import statistics

    import torch

    import paper_2101_01025_amd as ffa
    w = dict(WORKLOADS[args.workload])
    w["name"] = args.workload
    try:
        if args.workload.startswith("batch"):
            print(json.dumps(run_batch(args, w, ffa, torch)))
            return
        run_single(args, w, ffa, torch)
    except (VerifyError, ffa.FfaError) as e:
        print(json.dumps({"error": f"result check failed: {e}", "workload": args.workload}))
        sys.exit(1)


def run_single(args, w, ffa, torch):
    n, k, p = w["n"], w["k"], w["p"]
    herm = w["name"].startswith("herk")
    A, Ai, A_host, Ai_host = make_input(w, torch)
    od = ffa.default_out_dtype(p) if w["dA"] not in ("float64", "int64") else \
        (torch.float64 if w["dA"] == "float64" else torch.int64)
    C = torch.zeros((n, n), dtype=od, device="cuda")
    Ci = torch.zeros((n, n), dtype=od, device="cuda") if herm else None
    torch.cuda.synchronize()

    streams = {"auto": ffa.STREAMS_AUTO, "one": ffa.STREAMS_ONE, "two": ffa.STREAMS_TWO}[args.streams]
    hb = {"auto": ffa.HERK_AUTO, "2m": ffa.HERK_2M, "4m": ffa.HERK_4M}[args.herk_base]
    gen = {"auto": ffa.GENERAL_AUTO, "classical": ffa.GENERAL_CLASSICAL,
           "winograd": ffa.GENERAL_WINOGRAD}[args.general]
    levels = args.levels if args.levels >= 0 else w.get("levels", -1)
    opts = ffa.make_opts(levels=levels, streams=streams, herk_base=hb, kernel=args.kernel,
                         general=gen, wino_min=args.wino_min)
    dA_code = ffa._dtype_code(A)
    _, plan = ffa.plan_describe(n, k, p, hermitian=herm, dA=dA_code, dC=ffa._dtype_code(C, True),
                                opts=opts)
    # comparator: the plain classical product; over F_p[i] that is four real products per
    # complex product (the 2M base case is part of the method under test)
    classical = ffa.make_opts(algo=ffa.ALGO_CLASSICAL, herk_base=ffa.HERK_4M if herm else hb,
                              kernel=args.kernel)
    plans = [opts] if args.no_classical else [opts, classical]
    res = timed_steps(ffa, torch, w, A, Ai, C, Ci, plans, args.steps, args.warmup)
    ms, ms_med, prod_ms, ms_prof = res[0]
    value = n * n * k / (ms * 1e-3)
    phases = phase_breakdown(ffa, torch, w, A, Ai, C, Ci, opts)

    # the result of every timed plan, checked on the host after the timed region
    sentinel = {torch.uint8: 255, torch.int64: -7, torch.float64: -7.0}.get(od, 0xFFFF)
    checked = {}
    for name, o in zip(("recursive", "classical"), plans):
        C.fill_(sentinel)
        if herm:
            Ci.fill_(sentinel)
            ffa.herk_modp2(A, Ai, p, C_re=C, C_im=Ci, opts=o)
            torch.cuda.synchronize()
            checked[name] = verify_herk(A_host, Ai_host, p, C, Ci, sentinel, 91)
        else:
            ffa.syrk_modp(A, p, C=C, opts=o)
            torch.cuda.synchronize()
            checked[name] = verify_syrk(A_host, p, C, sentinel, 91)

    out = {
        "metric": "equivalent n^2k ops/s for A*A^T mod p (bit-exact)",
        "value": value,
        "unit": "n^2k/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_median": ms_med,
        "ms_per_step_profiled": ms_prof,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if plan["carrier"] == "int8" else "f64",
        "data": "synthetic",
        "verified": checked,
        "config": {"workload": f"{'herk' if herm else 'syrk'} n={n} k={k} p={p} input={w['dA']} "
                               f"carrier={w['carrier']}",
                   "n": n, "k": k, "p": p, "levels": plan["levels"], "limbs": plan["limbs"],
                   "parallelism": "single GPU"},
        "phases_ms": phases,
    }
    if herm:
        # value counts n^2 k operations of F_{p^2}; each is four products of F_p
        out["units"] = {"value": "n^2k/s of F_p^2 operations",
                        "fp_equivalent": 4.0 * n * n * k / (ms * 1e-3)}
    # roofline of the dominant kernel, the grouped product kernel: algorithmic ops of
    # one step's product phase over its duration in the timed region (HIP events)
    limb2 = plan["limbs"] ** 2  # macs counts real products (a complex one is four)
    ops = 2.0 * plan["macs"] * limb2
    if plan["carrier"] == "int8":
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_i8 (grouped products)",
                           "achieved": achieved, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                           "frac": achieved / PEAK_INT8_TOPS,
                           "traffic": measured_traffic(args.workload, plan["levels"]),
                           "ops_per_step": ops, "product_phase_ms": prod_ms}
    else:
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_f64 (grouped products)",
                           "achieved": achieved, "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_F64_TFLOPS, "traffic": None,
                           "ops_per_step": ops, "product_phase_ms": prod_ms}
    if not args.no_classical:
        cms, cmed, cprod, cprof = res[1]
        out["classical_gpu"] = {"value": n * n * k / (cms * 1e-3), "unit": "n^2k/s",
                                "ms_per_step": cms, "ms_median": cmed, "products_ms": cprod,
                                "ms_per_step_profiled": cprof}
        out["speedup_vs_classical"] = cms / ms
        out["speedup_vs_classical_median"] = cmed / ms_med
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        if w.get("cpu_seconds"):
            out["cpu_seconds"] = cpu_seconds_small(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
