"""GPU tests of the batched path's launch modes and of the autotuner.

Every result is compared bit-exactly with the CPU oracle.  The graph tests
replay a captured launch sequence several times, with unrelated eager GPU
work and synchronisations between replays, and check every replay.
"""
import json

import numpy as np
import pytest

import oracle
import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ffa():
    import paper_2101_01025_amd as ffa
    return ffa


def _say(*a):
    print("[case]", *a, flush=True)


def _u16(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int32)).to("cuda").to(torch.uint16)


def _host(t):
    if t.dtype == torch.uint16:
        t = t.to(torch.int32)
    return t.cpu().numpy().astype(np.int64)


def _batch(count, seed, nmax=300, p=65521, **opts):
    ffa = _ffa()
    ns, ks = si.batch_shapes(count, seed, nmin=1, nmax=nmax)
    mats = si.batch_residues(ns, ks, p, seed)
    B = ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16, **opts)
    Ap = B.pack(mats, np.int64)
    B.ks_host = ks
    return B, ns, mats, _u16(Ap)


def _check_batch(B, ns, mats, Cp, p=65521, upper=None):
    Ch = _host(Cp)
    for i, M in enumerate(mats):
        n = int(ns[i])
        got = Ch[B.c_off[i]:B.c_off[i] + n * n].reshape(n, n)
        assert np.array_equal(np.tril(got), oracle.syrk_modp(M, p)), f"problem {i}"
        if upper is not None:
            assert np.all(got[np.triu_indices(n, 1)] == upper), f"upper triangle of problem {i}"


def _sentinel(total, v=0xBEEF):
    return torch.full((total,), v, dtype=torch.int32, device="cuda").to(torch.uint16)


def _busy_work():
    x = torch.randn(512, 512, device="cuda")
    y = (x @ x).sum()
    torch.cuda.synchronize()
    return float(y)


@pytest.mark.parametrize("levels", [0, 1])
def test_batch_graph_replays_and_buffer_changes(levels):
    """Default launch mode (captured hipGraph): repeated calls on one buffer pair,
    then on another pair (re-capture), then back; each result checked."""
    ffa = _ffa()
    _say("batch graph", levels)
    B, ns, mats, A = _batch(20, 301, levels=levels)
    C1, C2 = _sentinel(B.c_total), _sentinel(B.c_total)
    for C in (C1, C1, C2, C1, C2):
        B.run(A, C)
        torch.cuda.synchronize()
        _check_batch(B, ns, mats, C, upper=0xBEEF)
        _busy_work()
    B.close()


def test_batch_direct_and_graph_agree():
    ffa = _ffa()
    _say("batch direct vs graph")
    Bg, ns, mats, A = _batch(16, 302, levels=1)
    Bd = ffa.BatchSyrk(ns, Bg.ks_host, 65521, ffa.U16, ffa.U16, levels=1, launch=ffa.LAUNCH_DIRECT)
    Cg, Cd = _sentinel(Bg.c_total), _sentinel(Bd.c_total)
    Bg.run(A, Cg)
    Bd.run(A, Cd)
    torch.cuda.synchronize()
    assert torch.equal(Cg, Cd)
    _check_batch(Bg, ns, mats, Cg)
    Bg.close()
    Bd.close()


def test_batch_inside_torch_graph_capture():
    """The caller captures the batched call into its own graph: the kernels join
    that graph.  Replays are checked one by one, with C cleared eagerly between."""
    ffa = _ffa()
    _say("batch in torch graph")
    B, ns, mats, A = _batch(12, 303, levels=1)
    C = _sentinel(B.c_total)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.run(A, C)  # warm-up outside capture (first launches set kernel attributes)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    _check_batch(B, ns, mats, C)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.run(A, C)
    for rep in range(3):
        C.copy_(_sentinel(B.c_total, 0x0101 + rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_batch(B, ns, mats, C, upper=0x0101 + rep)
        _busy_work()
    del g
    B.close()


def test_batch_autotune_keeps_results_exact():
    ffa = _ffa()
    _say("batch autotune")
    B, ns, mats, A = _batch(24, 304)
    C = _sentinel(B.c_total)
    best, ms = B.autotune(A, C, reps=1)
    assert ms > 0
    assert best.carrier in (ffa.CARRIER_INT8, ffa.CARRIER_F64)
    torch.cuda.synchronize()
    _check_batch(B, ns, mats, C)
    C2 = _sentinel(B.c_total)
    B.run(A, C2)
    torch.cuda.synchronize()
    _check_batch(B, ns, mats, C2, upper=0xBEEF)
    B.close()


@pytest.mark.parametrize("p,n,k,dt", [(251, 1000, 700, "u8"), (65521, 600, 500, "u16")])
def test_autotune_syrk_and_tuned_default(p, n, k, dt):
    ffa = _ffa()
    _say("autotune", p, n, k)
    Ares = si.uniform_residues(n, k, p, 305)
    if dt == "u8":
        A = torch.from_numpy(Ares.astype(np.uint8)).to("cuda")
    else:
        A = _u16(Ares)
    exp = oracle.syrk_modp(Ares, p)
    best, ms = ffa.autotune_syrk(A, p, reps=1)
    assert ms > 0 and 0 <= best.levels <= 4
    # no options: the tuned choice for this shape
    C = ffa.syrk_modp(A, p)
    torch.cuda.synchronize()
    assert np.array_equal(np.tril(_host(C)), exp)
    rec = json.loads(ffa.tune_export())
    assert rec["arch"].startswith("gfx")
    mine = [r for r in rec["records"] if (r["n"], r["k"], r["p"]) == (n, k, p)]
    assert mine and mine[0]["levels"] == best.levels and mine[0]["kernel"] == best.kernel
    assert mine[0]["operands"] == best.operands and mine[0]["general"] == best.general
    assert ffa.tune_import(json.dumps(rec)) == len(rec["records"])
    # a shape of the same size class without a record of its own uses the class record
    A2 = A[: n - 3, : k - 5].contiguous()
    C2 = ffa.syrk_modp(A2, p)
    torch.cuda.synchronize()
    assert np.array_equal(np.tril(_host(C2)), oracle.syrk_modp(Ares[: n - 3, : k - 5], p))


@pytest.mark.parametrize("base", ["2m", "4m"])
@pytest.mark.parametrize("launch", ["graph", "direct"])
@pytest.mark.parametrize("p", [65519, 251])
def test_batch_herk(base, launch, p):
    """Batched Low(A_i A_i^H) over F_p[i] (two limbs at p = 65519, one at p = 251):
    every problem compared whole with the oracle; the graph mode is replayed on
    changed buffers (re-capture) and checked again."""
    ffa = _ffa()
    _say("batch herk", p, base, launch)
    ns, ks = si.batch_shapes(18, 306, nmin=1, nmax=300)
    dA = ffa.U16 if p > 255 else ffa.I64
    B = ffa.BatchHerk(ns, ks, p, dA, ffa.U16,
                      herk_base=ffa.HERK_2M if base == "2m" else ffa.HERK_4M,
                      launch=ffa.LAUNCH_GRAPH if launch == "graph" else ffa.LAUNCH_DIRECT,
                      cutoff=128)
    mats = [si.complex_residues(int(n), int(k), p, 700 + i) for i, (n, k) in enumerate(zip(ns, ks))]
    if p > 255:
        Ar = _u16(B.pack([m[0] for m in mats], np.int64))
        Ai = _u16(B.pack([m[1] for m in mats], np.int64))
    else:
        Ar = torch.from_numpy(B.pack([m[0] for m in mats], np.int64)).to("cuda")
        Ai = torch.from_numpy(B.pack([m[1] for m in mats], np.int64)).to("cuda")
    exp = [oracle.herk_modp2(m[0], m[1], p) for m in mats]

    def check(Cr, Ci):
        gr, gi = _host(Cr), _host(Ci)
        for i in range(len(ns)):
            n = int(ns[i])
            o = int(B.c_off[i])
            r = gr[o:o + n * n].reshape(n, n)
            m = gi[o:o + n * n].reshape(n, n)
            low = np.tril(np.ones((n, n), dtype=bool))
            assert np.array_equal(r[low], exp[i][0][low]), f"re of problem {i}"
            assert np.array_equal(m[low], exp[i][1][low]), f"im of problem {i}"
            assert (r[~low] == 0xBEEF).all() and (m[~low] == 0xBEEF).all(), f"upper of problem {i}"

    pairs = [(_sentinel(B.c_total), _sentinel(B.c_total)) for _ in range(2)]
    for j in (0, 0, 1):
        Cr, Ci = pairs[j]
        B.run(Ar, Ai, Cr, Ci)
        torch.cuda.synchronize()
        check(Cr, Ci)
        _busy_work()
    with pytest.raises(ffa.FfaError):
        B.autotune(Ar, Cr)
    B.close()


def test_tuned_record_applies_without_options():
    """A call with no options runs the context's tuned record for its shape: a record
    asking for one recursion level shows pre-additions in the phase profile, one
    asking for none does not; an explicit option overrides the record."""
    ffa = _ffa()
    p, n, k = 65521, 520, 600
    _say("tuned record without options")
    Ares = si.uniform_residues(n, k, p, 307)
    A = _u16(Ares)
    exp = oracle.syrk_modp(Ares, p)
    arch = json.loads(ffa.tune_export())["arch"]

    def record(levels):
        return json.dumps({"arch": arch, "records": [{
            "n": n, "k": k, "p": p, "herm": 0, "dA": ffa.U16, "dC": ffa.U16,
            "algo": ffa.ALGO_RECURSIVE if levels else ffa.ALGO_CLASSICAL, "levels": levels,
            "cutoff": 0, "carrier": ffa.CARRIER_INT8, "kernel": 0}]})

    def preadds(**kw):
        torch.cuda.synchronize()
        ffa.profile_reset(0)
        ffa.profile_enable(0, True)
        C = ffa.syrk_modp(A, p, **kw)
        torch.cuda.synchronize()
        _, calls = ffa.profile_read(0, ffa.PHASE_PRE)
        ffa.profile_enable(0, False)
        assert np.array_equal(np.tril(_host(C)), exp)
        return calls

    assert ffa.tune_import(record(1)) == 1
    assert preadds() > 0
    assert ffa.tune_import(record(0)) == 1
    assert preadds() == 0
    assert preadds(levels=1) > 0


@pytest.mark.parametrize("dc", ["u16", "i32"])
@pytest.mark.parametrize("general", ["classical", "winograd"])
def test_batch_p251_mixed_depths_and_formats(dc, general):
    """A batch at p = 251 whose workspace residues are bytes while C is wider, with
    problems deep enough to recurse next to ones that do not: every problem
    compared whole with the oracle."""
    ffa = _ffa()
    p = 251
    _say("batch p251", dc, general)
    ns, ks = si.batch_shapes(14, 308, nmin=1, nmax=400)
    mats = si.batch_residues(ns, ks, p, 308)
    dC, tdt = (ffa.U16, torch.uint16) if dc == "u16" else (ffa.I32, torch.int32)
    B = ffa.BatchSyrk(ns, ks, p, ffa.U8, dC, cutoff=128,
                      general=ffa.GENERAL_WINOGRAD if general == "winograd" else ffa.GENERAL_CLASSICAL)
    d = B.describe()
    assert d["levels"] >= 1 and (d["wino_tasks"] > 0) == (general == "winograd")
    A = torch.from_numpy(B.pack(mats, np.uint8)).to("cuda")
    C = torch.full((B.c_total,), 0x1234, dtype=torch.int32, device="cuda").to(tdt)
    B.run(A, C)
    torch.cuda.synchronize()
    Ch = _host(C)
    for i, M in enumerate(mats):
        n = int(ns[i])
        got = Ch[B.c_off[i]:B.c_off[i] + n * n].reshape(n, n)
        assert np.array_equal(np.tril(got), oracle.syrk_modp(M, p)), f"problem {i}"
        assert (got[np.triu_indices(n, 1)] == 0x1234).all(), f"upper of problem {i}"
    B.close()


def test_batch_input_range_check():
    """check_inputs on a batch: an entry outside [0, p) in one problem gives ERANGE and
    leaves C untouched; a clean batch runs."""
    ffa = _ffa()
    p = 65521
    _say("batch range check")
    ns, ks = si.batch_shapes(6, 309, nmin=1, nmax=200)
    mats = si.batch_residues(ns, ks, p, 309)
    B = ffa.BatchSyrk(ns, ks, p, ffa.I32, ffa.U16, check_inputs=True)
    packed = B.pack(mats, np.int32)
    C = _sentinel(B.c_total)
    B.run(torch.from_numpy(packed).to("cuda"), C)
    torch.cuda.synchronize()
    _check_batch(B, ns, mats, C)
    bad = packed.copy()
    i = 3
    bad[B.a_off[i] + int(B.lda[i]) * (int(ns[i]) // 2)] = p  # row n/2, column 0 of problem 3
    C2 = _sentinel(B.c_total)
    with pytest.raises(ffa.FfaError) as e:
        B.run(torch.from_numpy(bad).to("cuda"), C2)
    assert e.value.status == ffa.ERANGE
    torch.cuda.synchronize()
    assert (_host(C2) == 0xBEEF).all()
    B.close()
