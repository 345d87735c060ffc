"""GPU parity at the full sizes of the measured workloads.

The oracle cannot form these products whole in test time, so each case checks
(1) a sample of lower-triangle entries computed one by one by the oracle, with
the block edges of the recursion always included, (2) Freivalds random-vector
checks of the whole lower triangle, (3) that every entry is a canonical residue
and (4) that the strict upper triangle still holds its sentinel.  The small
256 x 256 workload is compared whole.
"""
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


def _host(t):
    if t.dtype == torch.uint16:
        t = t.to(torch.int32)
    return t.cpu().numpy().astype(np.int64)


def _u16(a):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int32)).to("cuda").to(torch.uint16)


def _pairs(n, rng, count=2000):
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    i, j = np.maximum(i, j), np.minimum(i, j)
    edges = [0, 1, n - 2, n - 1]
    for q in (2, 4, 8, 16):
        b = n // q
        edges += [b - 1, b, b + 1]
    edges = np.unique(np.clip(np.array(edges), 0, n - 1))
    ei, ej = np.meshgrid(edges, edges)
    m = ei >= ej
    return np.concatenate([i, ei[m]]), np.concatenate([j, ej[m]])


def _upper_untouched(C, sentinel, n, rows=64):
    """Strict upper triangle of a few whole rows (first, last, spread) still the sentinel."""
    idx = np.unique(np.linspace(0, n - 1, rows).astype(np.int64))
    for r in idx:
        row = _host(C[int(r), int(r) + 1:])
        assert (row == sentinel).all(), f"row {r}"


def _check_syrk_large(Ares, C, p, rng):
    n = Ares.shape[0]
    Ch = _host(C)
    low = np.tril_indices(n)
    assert Ch[low].min() >= 0 and Ch[low].max() < p
    ii, jj = _pairs(n, rng)
    assert np.array_equal(Ch[ii, jj], oracle.syrk_entries(Ares, p, ii, jj))
    Cl = np.tril(Ch)
    for _ in range(4):  # false-pass probability p^-4 at most
        x = rng.integers(0, p, n)
        yc, ya = oracle.freivalds_syrk(Ares, Cl, p, x)
        assert np.array_equal(yc, ya)


def test_small_256_int64_one_level():
    """256 x 256, p = 65521, int64 storage, one recursion level: compared whole."""
    ffa = _ffa()
    p = 65521
    _say("256 int64 p65521 levels=1")
    Ares = si.uniform_residues(256, 256, p, si.config_seed(0))
    C = torch.full((256, 256), -7, dtype=torch.int64, device="cuda")
    ffa.syrk_modp(torch.from_numpy(Ares).to("cuda"), p, C=C, levels=1)
    torch.cuda.synchronize()
    got = _host(C)
    low = np.tril(np.ones((256, 256), dtype=bool))
    assert np.array_equal(got[low], oracle.syrk_modp(Ares, p)[low])
    assert (got[~low] == -7).all()


@pytest.mark.parametrize("algo", ["recursive", "recursive_plain_general", "classical"])
def test_f64_8192_p65521(algo):
    """8192 x 8192, p = 65521, fp64 storage on the fp64 carrier, cutoff 512 (four levels);
    general products by Strassen-Winograd (the default here) or as single products."""
    ffa = _ffa()
    n = k = 8192
    p = 65521
    _say("f64", n, k, p, algo)
    Ares = si.uniform_residues(n, k, p, si.config_seed(1))
    A = torch.from_numpy(Ares.astype(np.float64)).to("cuda")
    C = torch.full((n, n), -7.0, dtype=torch.float64, device="cuda")
    kw = dict(algo=ffa.ALGO_CLASSICAL) if algo == "classical" else dict(cutoff=512)
    if algo == "recursive_plain_general":
        kw["general"] = ffa.GENERAL_CLASSICAL
    if algo != "classical":
        _, d = ffa.plan_describe(n, k, p, dA=ffa.F64, dC=ffa.F64,
                                 opts=ffa.make_opts(**{"cutoff": 512, **kw}))
        assert d["levels"] == 4 and d["carrier"] == "f64"
        assert d["general"] == ("winograd" if algo == "recursive" else "classical")
    ffa.syrk_modp(A, p, C=C, **kw)
    torch.cuda.synchronize()
    _upper_untouched(C, -7, n)
    _check_syrk_large(Ares, C, p, np.random.default_rng(11))


@pytest.mark.parametrize("algo", ["recursive", "classical", "winograd"])
def test_int8x2_16384_p65521(algo):
    """16384 x 16384, p = 65521, two balanced int8 limbs on INT8 MFMA."""
    ffa = _ffa()
    n = k = 16384
    p = 65521
    _say("int8x2", n, k, p, algo)
    Ares = si.uniform_residues(n, k, p, si.config_seed(2) + 1)
    A = _u16(Ares)
    C = torch.full((n, n), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    kw = dict(algo=ffa.ALGO_CLASSICAL) if algo == "classical" else dict()
    if algo == "winograd":
        kw = dict(general=ffa.GENERAL_WINOGRAD)
    ffa.syrk_modp(A, p, C=C, **kw)
    torch.cuda.synchronize()
    del A
    _upper_untouched(C, 0xBEEF, n)
    _check_syrk_large(Ares, C, p, np.random.default_rng(12))


@pytest.mark.parametrize("plan", ["default", "levels1-2m", "levels1-4m", "classical-4m"])
def test_herk_4096x8192_p65519(plan):
    """A 4096 x 8192 over F_p[i]/(i^2+1), p = 65519, planar uint16: the default plan (2M base
    case, no recursion), one level of Algorithm 1 over the 2M or the 4M base case, and the
    plain complex product (four real products)."""
    ffa = _ffa()
    n, k, p = 4096, 8192, 65519
    kw = {"default": {}, "levels1-2m": dict(levels=1, herk_base=ffa.HERK_2M),
          "levels1-4m": dict(levels=1, herk_base=ffa.HERK_4M),
          "classical-4m": dict(algo=ffa.ALGO_CLASSICAL, herk_base=ffa.HERK_4M)}[plan]
    if kw:
        st, d = ffa.plan_describe(n, k, p, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                                  opts=ffa.make_opts(**kw))
        assert st == 0 and d["levels"] == kw.get("levels", 0), d
    _say("herk", n, k, p, plan)
    Ar, Ai = si.complex_residues(n, k, p, si.config_seed(4))
    Cr = torch.full((n, n), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    Ci = torch.full((n, n), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    ffa.herk_modp2(_u16(Ar), _u16(Ai), p, C_re=Cr, C_im=Ci, **kw)
    torch.cuda.synchronize()
    _upper_untouched(Cr, 0xBEEF, n)
    _upper_untouched(Ci, 0xBEEF, n)
    gr, gi = _host(Cr), _host(Ci)
    low = np.tril_indices(n)
    assert gr[low].max() < p and gi[low].max() < p
    assert (np.diagonal(gi) == 0).all()
    rng = np.random.default_rng(13)
    ii, jj = _pairs(n, rng)
    er, ei = oracle.herk_entries(Ar, Ai, p, ii, jj)
    assert np.array_equal(gr[ii, jj], er) and np.array_equal(gi[ii, jj], ei)
    Lr, Li = np.tril(gr), np.tril(gi)
    for _ in range(4):  # false-pass probability p^-8 at most (two coordinates each)
        xr, xi = rng.integers(0, p, n), rng.integers(0, p, n)
        yc, ya = oracle.freivalds_herk(Ar, Ai, Lr, Li, p, xr, xi)
        assert np.array_equal(yc[0], ya[0]) and np.array_equal(yc[1], ya[1])


def test_batch_4096_p65521():
    """4096 problems, n in [32, 512], k in [n, 2n], p = 65521, uint16, default plan
    and launch mode.  Freivalds on every problem, whole comparison on 32 of them."""
    ffa = _ffa()
    p = 65521
    seed = si.config_seed(3)
    ns, ks = si.batch_shapes(4096, seed)
    _say("batch 4096", int((ns * ns * ks).sum()))
    mats = si.batch_residues(ns, ks, p, seed, dtype=np.int32)
    B = ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16)
    Ap = B.pack(mats, np.int32)
    A = _u16(Ap)
    del Ap
    C = torch.full((B.c_total,), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    B.run(A, C)
    torch.cuda.synchronize()
    Ch = C.to(torch.int32).cpu().numpy()
    rng = np.random.default_rng(14)
    whole = set(rng.choice(4096, 32, replace=False).tolist()) | {int(np.argmax(ns)), int(np.argmin(ns))}
    for i, M in enumerate(mats):
        n = int(ns[i])
        got = Ch[B.c_off[i]:B.c_off[i] + n * n].reshape(n, n).astype(np.int64)
        assert (got[np.triu_indices(n, 1)] == 0xBEEF).all(), f"upper of problem {i}"
        Cl = np.tril(got)
        assert Cl.max() < p
        if i in whole:
            assert np.array_equal(Cl, oracle.syrk_modp(M, p)), f"problem {i}"
        else:
            x = rng.integers(0, p, n)
            yc, ya = oracle.freivalds_syrk(M, Cl, p, x)
            assert np.array_equal(yc, ya), f"problem {i}"
    B.close()
