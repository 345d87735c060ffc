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
    "herk_p65519_int8x2": dict(n=4096, k=8192, p=65519, dA="uint16", carrier="int8 x2 limbs, complex"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="syrk_p251_int8", choices=sorted(WORKLOADS))
    ap.add_argument("--levels", type=int, default=-1, help="recursion depth (-1: library default)")
    ap.add_argument("--no-classical", action="store_true", help="skip the classical comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


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


def run_steps(ffa, torch, w, A, Ai, C, Ci, opts, steps, warmup):
    def one():
        if Ai is None:
            ffa.syrk_modp(A, w["p"], C=C, opts=opts)
        else:
            ffa.herk_modp2(A, Ai, w["p"], C_re=C, C_im=Ci, opts=opts)
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ffa.profile_reset(0)
    ffa.profile_enable(0, True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        one()
    stop.record()
    torch.cuda.synchronize()
    ffa.profile_enable(0, False)
    total_ms = start.elapsed_time(stop)
    phases = {}
    for ph, name in ((ffa.PHASE_COND, "conditioning"), (ffa.PHASE_PRE, "preadd"),
                     (ffa.PHASE_PRODUCTS, "products"), (ffa.PHASE_POST, "postadd")):
        ms, calls = ffa.profile_read(0, ph)
        phases[name] = round(ms / calls, 4) if calls else 0.0
    return total_ms / steps, phases


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
        if t > seconds / 4 or m >= n:
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
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not "
                                   "part of this build (use --gpus 1)"}))
        sys.exit(2)
    import torch

    import paper_2101_01025_amd as ffa
    w = dict(WORKLOADS[args.workload])
    w["name"] = args.workload
    n, k, p = w["n"], w["k"], w["p"]
    herm = w["name"].startswith("herk")
    A, Ai = make_input(w, torch)
    od = ffa.default_out_dtype(p) if w["dA"] != "float64" else torch.float64
    C = torch.zeros((n, n), dtype=od, device="cuda")
    Ci = torch.zeros((n, n), dtype=od, device="cuda") if herm else None
    torch.cuda.synchronize()

    opts = ffa.make_opts(levels=args.levels) if args.levels >= 0 else ffa.make_opts()
    dA_code = ffa._dtype_code(A)
    _, plan = ffa.plan_describe(n, k, p, hermitian=herm, dA=dA_code, dC=ffa._dtype_code(C, True),
                                opts=opts)
    ms, phases = run_steps(ffa, torch, w, A, Ai, C, Ci, opts, args.steps, args.warmup)
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
    }
    # roofline of the dominant kernel: the grouped product launch
    limb2 = plan["limbs"] ** 2 * (4 if herm else 1)
    ops = 2.0 * plan["macs"] * limb2
    prod_ms = phases["products"]
    if plan["carrier"] == "int8":
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_i8 (grouped products)",
                           "achieved": achieved, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                           "frac": achieved / PEAK_INT8_TOPS, "traffic": None,
                           "ops_per_launch": ops}
    else:
        achieved = ops / (prod_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "gemm_f64 (grouped products)",
                           "achieved": achieved, "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_F64_TFLOPS, "traffic": None,
                           "ops_per_launch": ops}
    if not args.no_classical:
        copts = ffa.make_opts(algo=ffa.ALGO_CLASSICAL)
        cms, cph = run_steps(ffa, torch, w, A, Ai, C, Ci, copts, args.steps, args.warmup)
        out["classical_gpu"] = {"value": n * n * k / (cms * 1e-3), "unit": "n^2k/s",
                                "ms_per_step": cms, "products_ms": cph["products"]}
        out["speedup_vs_classical"] = cms / ms
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
