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
    "syrk_p251_int8": dict(n=16384, k=16384, p=251, dA="int8", carrier="int8 x1 limb"),
    "syrk_p65521_int8x2": dict(n=16384, k=16384, p=65521, dA="uint16", carrier="int8 x2 limbs"),
    "syrk_p65521_f64": dict(n=8192, k=8192, p=65521, dA="float64", carrier="fp64"),
    # the paper's two primes: 131071 = 3 mod 4 needs the 2x2-block Y, 131041 = 1 mod 4 a scalar Y
    "syrk_p131071_f64": dict(n=8192, k=8192, p=131071, dA="float64", carrier="fp64"),
    "syrk_p131041_f64": dict(n=8192, k=8192, p=131041, dA="float64", carrier="fp64"),
    "herk_p65519_int8x2": dict(n=4096, k=8192, p=65519, dA="uint16", carrier="int8 x2 limbs, complex"),
    # 4096 independent problems, n uniform in [32, 512], k uniform in [n, 2n]
    "batch4096_p65521": dict(count=4096, nmin=32, nmax=512, p=65521, dA="uint16",
                             carrier="autotuned"),
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
                  for f in ("gemm_i8.hip", "device_common.h", "ffa_internal.h")]


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
    import numpy as np

    import seeded_inputs as si
    n, k, p = w["n"], w["k"], w["p"]
    seed = si.config_seed(2)
    if w["dA"] == "int8":
        return torch.from_numpy(si.centred_int8(n, k, p, seed)).to("cuda"), None
    if w["dA"] == "uint16":
        if w["name"].startswith("herk"):
            ar, ai = si.complex_residues(n, k, p, si.config_seed(4), dtype=np.int32)
            return (torch.from_numpy(ar).to("cuda").to(torch.uint16),
                    torch.from_numpy(ai).to("cuda").to(torch.uint16))
        a = si.uniform_residues(n, k, p, seed, dtype=np.int32)
        return torch.from_numpy(a).to("cuda").to(torch.uint16), None
    a = si.uniform_residues(n, k, p, si.config_seed(1), dtype=np.float64)
    return torch.from_numpy(a).to("cuda"), None


def timed_steps(ffa, torch, w, A, Ai, C, Ci, plans, steps, warmup, blocks=5):
    """Times `steps` calls of each plan (recursive, then classical if given).

    The plans run in alternating blocks so that clock and thermal drift during
    the run affects both alike.  Phase durations come from HIP events the
    library records around each phase on the same stream.
    Returns per plan: (ms per step, {phase: summed ms of its launches per call},
    {phase: launches per call}).
    """
    def one(opts):
        if Ai is None:
            ffa.syrk_modp(A, w["p"], C=C, opts=opts)
        else:
            ffa.herk_modp2(A, Ai, w["p"], C_re=C, C_im=Ci, opts=opts)
    for opts in plans:
        for _ in range(warmup):
            one(opts)
    torch.cuda.synchronize()
    total = [0.0] * len(plans)
    phase_ms = [dict() for _ in plans]
    phase_calls = [dict() for _ in plans]
    names = ((ffa.PHASE_COND, "conditioning"), (ffa.PHASE_PRE, "preadd"),
             (ffa.PHASE_PRODUCTS, "products"), (ffa.PHASE_POST, "postadd"))
    per_block = [steps // blocks + (1 if b < steps % blocks else 0) for b in range(blocks)]
    for nb in per_block:
        if nb == 0:
            continue
        for i, opts in enumerate(plans):
            ffa.profile_reset(0)
            ffa.profile_enable(0, True)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record()
            for _ in range(nb):
                one(opts)
            stop.record()
            torch.cuda.synchronize()
            ffa.profile_enable(0, False)
            total[i] += start.elapsed_time(stop)
            for ph, name in names:
                ms, calls = ffa.profile_read(0, ph)
                phase_ms[i][name] = phase_ms[i].get(name, 0.0) + ms
                phase_calls[i][name] = phase_calls[i].get(name, 0) + calls
    out = []
    for i in range(len(plans)):
        ph = {name: round(phase_ms[i][name] / steps, 4) for _, name in names}
        nl = {name: phase_calls[i][name] / steps for _, name in names}
        out.append((total[i] / steps, ph, nl))
    return out


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
    del mats
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
    blocks = 5
    per_block = [args.steps // blocks + (1 if i < args.steps % blocks else 0) for i in range(blocks)]
    total = [0.0] * len(runs)
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
    out = {
        "metric": "equivalent n^2k ops/s for A*A^T mod p (bit-exact)",
        "value": eq_ops / (ms * 1e-3),
        "unit": "n^2k/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if plan["carrier"] == "int8" else "f64",
        "data": "synthetic",
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
        out["classical_gpu"] = {"value": eq_ops / (cms * 1e-3), "unit": "n^2k/s", "ms_per_step": cms}
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


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (use --gpus 1); "
                                   "the multi-GPU design is described, not built"}))
        sys.exit(2)
    import torch

    import paper_2101_01025_amd as ffa
    w = dict(WORKLOADS[args.workload])
    w["name"] = args.workload
    if args.workload.startswith("batch"):
        print(json.dumps(run_batch(args, w, ffa, torch)))
        return
    n, k, p = w["n"], w["k"], w["p"]
    herm = w["name"].startswith("herk")
    A, Ai = make_input(w, torch)
    od = ffa.default_out_dtype(p) if w["dA"] != "float64" else torch.float64
    C = torch.zeros((n, n), dtype=od, device="cuda")
    Ci = torch.zeros((n, n), dtype=od, device="cuda") if herm else None
    torch.cuda.synchronize()

    streams = {"auto": ffa.STREAMS_AUTO, "one": ffa.STREAMS_ONE, "two": ffa.STREAMS_TWO}[args.streams]
    hb = {"auto": ffa.HERK_AUTO, "2m": ffa.HERK_2M, "4m": ffa.HERK_4M}[args.herk_base]
    gen = {"auto": ffa.GENERAL_AUTO, "classical": ffa.GENERAL_CLASSICAL,
           "winograd": ffa.GENERAL_WINOGRAD}[args.general]
    opts = ffa.make_opts(levels=args.levels, streams=streams, herk_base=hb, kernel=args.kernel,
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
    ms, phases, launches = res[0]
    value = n * n * k / (ms * 1e-3)

    out = {
        "metric": "equivalent n^2k ops/s for A*A^T mod p (bit-exact)",
        "value": value,
        "unit": "n^2k/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if plan["carrier"] == "int8" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{'herk' if herm else 'syrk'} n={n} k={k} p={p} input={w['dA']} "
                               f"carrier={w['carrier']}",
                   "n": n, "k": k, "p": p, "levels": plan["levels"], "limbs": plan["limbs"],
                   "parallelism": "single GPU"},
        "phases_ms": phases,
        "product_launches_per_step": launches["products"],
    }
    if herm:
        # value counts n^2 k operations of F_{p^2}; each is four products of F_p
        out["units"] = {"value": "n^2k/s of F_p^2 operations",
                        "fp_equivalent": 4.0 * n * n * k / (ms * 1e-3)}
    # roofline of the dominant kernel, the grouped product kernel: algorithmic ops of
    # its launches in one step over their summed durations (HIP events per launch)
    limb2 = plan["limbs"] ** 2  # macs counts real products (a complex one is four)
    ops = 2.0 * plan["macs"] * limb2
    prod_ms = phases["products"]
    if plan["carrier"] == "int8":
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_i8 (grouped products)",
                           "achieved": achieved, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                           "frac": achieved / PEAK_INT8_TOPS,
                           "traffic": measured_traffic(args.workload, plan["levels"]),
                           "ops_per_step": ops}
    else:
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_f64 (grouped products)",
                           "achieved": achieved, "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_F64_TFLOPS, "traffic": None,
                           "ops_per_step": ops}
    if not args.no_classical:
        cms, cph, _ = res[1]
        out["classical_gpu"] = {"value": n * n * k / (cms * 1e-3), "unit": "n^2k/s",
                                "ms_per_step": cms, "products_ms": cph["products"]}
        out["speedup_vs_classical"] = cms / ms
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
