"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Integer results, so the bar is bit-exact.  Small and medium cases compare the
whole lower triangle (several tiles and a ragged tail) and check that the
strict upper triangle is untouched; the full-size cases compare sampled
entries computed one by one by the oracle plus a Freivalds check.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SENTINEL = {torch.uint8: 0xA5, torch.int64: -7, torch.int32: -7, torch.float64: -7.0}
if hasattr(torch, "uint16"):
    SENTINEL[torch.uint16] = 0xBEEF


def _ffa():
    import paper_2101_01025_amd as ffa
    return ffa


def _dev(a, dtype):
    if dtype == torch.uint16:
        return torch.from_numpy(a.astype(np.int32)).to("cuda").to(torch.uint16)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def _host(t):
    if t.dtype == torch.uint16:
        t = t.to(torch.int32)
    return t.cpu().numpy().astype(np.int64)


def _sentinel_c(n, dtype):
    return torch.full((n, n), SENTINEL[dtype], dtype=dtype, device="cuda")


def _say(*a):
    print("[case]", *a, flush=True)


def check_syrk(A_res, p, dA, dC, **kw):
    """A_res: canonical residues (int64 host).  Runs the GPU call, compares to the oracle."""
    ffa = _ffa()
    n, k = A_res.shape
    _say("syrk", n, k, p, dA, dC, kw)
    if dA == torch.int8:
        A = _dev(si.to_centred(A_res, p).astype(np.int8), torch.int8)
    else:
        A = _dev(A_res, dA)
    C = _sentinel_c(n, dC)
    ffa.syrk_modp(A, p, C=C, **kw)
    torch.cuda.synchronize()
    got = _host(C)
    exp = oracle.syrk_modp(A_res, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(got[low], exp[low]), f"lower triangle differs ({n}x{k}, p={p}, {kw})"
    if n > 1:
        up = _host(C)[~low]
        assert (up == np.int64(SENTINEL[dC])).all(), "strict upper triangle was written"
    return got


# ------------------------------------------------------------------ INT8, one limb (p < 256)

@pytest.mark.parametrize("levels", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(1, 1), (7, 13), (100, 64), (257, 300), (600, 520)])
def test_int8_p251_centred(levels, shape):
    n, k = shape
    A = si.uniform_residues(n, k, 251, 100 + n + k)
    check_syrk(A, 251, torch.int8, torch.uint8, levels=levels)


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("p,dt", [(251, torch.int8), (65521, torch.uint16), (65519, torch.uint16)])
def test_two_streams(levels, p, dt):
    """Pre-additions and the products that need them on the context's second stream."""
    ffa = _ffa()
    n, k = 300, 520
    A = si.uniform_residues(n, k, p, 700 + p + levels)
    if p == 65519:
        Ai = si.uniform_residues(n, k, p, 701 + p + levels)
        check_herk(A, Ai, p, dt, levels=levels, streams=ffa.STREAMS_TWO)
    else:
        check_syrk(A, p, dt, torch.uint8 if p < 256 else torch.uint16, levels=levels,
                   streams=ffa.STREAMS_TWO)


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("p,dt", [(251, torch.int8), (13, torch.int64), (65521, torch.uint16),
                                  (65521, torch.float64), (131071, torch.float64)])
@pytest.mark.parametrize("shape", [(300, 520), (257, 1000)])
def test_winograd_general_products(levels, p, dt, shape):
    """P3 and P4 of every node by one level of Strassen-Winograd (seven half-size products)."""
    ffa = _ffa()
    n, k = shape
    A = si.uniform_residues(n, k, p, 1200 + levels * 7 + p % 97 + n)
    kw = dict(levels=levels, general=ffa.GENERAL_WINOGRAD)
    if dt == torch.float64:
        kw["carrier"] = ffa.CARRIER_F64
    out = torch.uint8 if p < 256 else (torch.uint16 if p < 65536 else torch.int64)
    check_syrk(A, p, dt, out, **kw)


@pytest.mark.parametrize("p,dt", [(65521, torch.float64), (251, torch.int8)])
@pytest.mark.parametrize("wino_min", [100, 200])
def test_winograd_threshold_mixed_plans(p, dt, wino_min):
    """Strassen-Winograd on the general products of at least wino_min rows only: the
    upper levels go through it, the lower ones stay single products."""
    ffa = _ffa()
    n, k = 700, 650
    dA = ffa.F64 if dt == torch.float64 else ffa.I8_CENTRED
    st, d = ffa.plan_describe(n, k, p, dA=dA, dC=ffa.U16 if p > 255 else ffa.U8,
                              opts=ffa.make_opts(levels=3, general=ffa.GENERAL_WINOGRAD,
                                                 wino_min=wino_min))
    assert st == 0 and 0 < d["wino_tasks"] < 2 + 6 + 18
    A = si.uniform_residues(n, k, p, 1300 + wino_min)
    out = torch.uint8 if p < 256 else torch.uint16
    kw = dict(levels=3, general=ffa.GENERAL_WINOGRAD, wino_min=wino_min)
    if dt == torch.float64:
        kw["carrier"] = ffa.CARRIER_F64
    check_syrk(A, p, dt, out, **kw)


# (n, k, p, input, output, options): shapes whose launch leaves a partial last round of
# at most a quarter (a half) of each XCD, so that those tiles are computed as four (two)
# K-pieces and summed (one limb on 256-tiles, recursive and classical; two limbs on
# 128-tiles)
TAIL_CASES = [
    (2304, 2560, 251, "i8", "u8", dict(algo=1)),
    (4352, 1024, 251, "i8", "u8", dict(levels=1)),
    (2944, 1024, 65521, "u16", "u16", dict(algo=1)),
    (2944, 1024, 65521, "u16", "i64", dict(algo=1)),
    (3712, 1024, 65521, "u16", "u16", dict(algo=1)),  # halves only
]


@pytest.mark.parametrize("n,k,p,di,do,kw", TAIL_CASES)
def test_split_last_round_tiles(n, k, p, di, do, kw):
    ffa = _ffa()
    dA = ffa.I8_CENTRED if di == "i8" else ffa.U16
    dC = {"u8": ffa.U8, "u16": ffa.U16, "i64": ffa.I64}[do]
    st, d = ffa.plan_describe(n, k, p, dA=dA, dC=dC, opts=ffa.make_opts(**kw))
    assert st == 0 and d["tail_tiles"] > 0, d
    A = si.uniform_residues(n, k, p, 1500 + n + k)
    tdA = torch.int8 if di == "i8" else torch.uint16
    tdC = {"u8": torch.uint8, "u16": torch.uint16, "i64": torch.int64}[do]
    check_syrk(A, p, tdA, tdC, **kw)


@pytest.mark.parametrize("n,k", [(2304, 2560), (2304, 2816)])
def test_split_last_round_into_strided_unaligned_c(n, k):
    """The last-round pieces summed into a view of C whose rows are not 16-byte aligned
    (odd offset, odd row stride): the product kernel's element-wise edge stores and the
    scalar path of the piece sums; quarters (20 k-tiles) and halves (22 k-tiles)."""
    ffa = _ffa()
    p = 251
    st, d = ffa.plan_describe(n, k, p, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(algo=1))
    assert st == 0 and d["tail_tiles"] > 0, d
    A = si.uniform_residues(n, k, p, 1700 + k)
    big = torch.full((n + 2, n + 7), 0x5A, dtype=torch.uint8, device="cuda")
    C = big[1:1 + n, 3:3 + n]
    ffa.syrk_modp(_dev(si.to_centred(A, p).astype(np.int8), torch.int8), p, C=C, algo=1)
    torch.cuda.synchronize()
    g = big.cpu().numpy().astype(np.int64)
    exp = oracle.syrk_modp(A, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    view = g[1:1 + n, 3:3 + n]
    assert np.array_equal(view[low], exp[low])
    assert (view[~low] == 0x5A).all()
    outside = np.ones_like(g, dtype=bool)
    outside[1:1 + n, 3:3 + n] = False
    assert (g[outside] == 0x5A).all()


@pytest.mark.parametrize("p", [3, 5, 13, 241])
def test_int8_small_primes(p):
    # p = 3 and 251 use Y = [[a,b],[-b,a]] (x) I; p = 5, 13, 241 use Y = sqrt(-1) I
    A = si.uniform_residues(150, 190, p, p)
    for levels in (0, 1, 3):
        check_syrk(A, p, torch.uint8, torch.int64, levels=levels)


def test_int8_extremes():
    # all entries at the largest centred magnitude, at a large K: stresses int32 accumulation
    p, n, k = 251, 256, 65536
    for val in (125, 126):  # +125 and -125
        A = np.full((n, k), val, dtype=np.int64)
        check_syrk(A, p, torch.int8, torch.uint8, algo=1)
        check_syrk(A, p, torch.int8, torch.uint8, levels=2)


# ------------------------------------------------------------------ INT8, two limbs (p < 2^16)

@pytest.mark.parametrize("levels", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(130, 70), (300, 257), (513, 600)])
def test_int8x2_p65521(levels, shape):
    n, k = shape
    A = si.uniform_residues(n, k, 65521, 200 + n)
    check_syrk(A, 65521, torch.uint16, torch.uint16, levels=levels)


def test_int8x2_extreme_limbs():
    p = 65521
    n, k = 200, 30000
    # representatives with the largest limb magnitudes: -32881 (hi = -128) and 32639 (hi = 127)
    for v in (p - 32881, 32639, p - 1):
        A = np.full((n, k), v, dtype=np.int64)
        check_syrk(A, p, torch.uint16, torch.uint16, algo=1)
        check_syrk(A, p, torch.int32, torch.int64, levels=1)


# ------------------------------------------------------------------ at the exact-accumulation bound
# The planner admits a product while K * max|x| * max|y| stays below the carrier's exact
# range (int32 for INT8 MFMA, 2^53 for fp64).  These cases run at the largest K it admits,
# with the operand magnitudes that reach the bound, and compare the whole lower triangle.

def _pattern(n, k, hi, lo, kind):
    """Residues: all `hi`, all `lo`, or `hi` / `lo` alternating with the parity of
    row + column (so that rows of equal parity meet hi*hi + ... and rows of different
    parity hi*lo terms in every position)."""
    if kind == "hi":
        return np.full((n, k), hi, dtype=np.int64)
    if kind == "lo":
        return np.full((n, k), lo, dtype=np.int64)
    par = (np.arange(n)[:, None] + np.arange(k)[None, :]) & 1
    return np.where(par == 0, hi, lo).astype(np.int64)


def _check_planned(n, k, p, dA, dC, **kw):
    ffa = _ffa()
    st, d = ffa.plan_describe(n, k, p, dA=dA, dC=dC, opts=ffa.make_opts(**kw))
    assert st == 0, d
    return d


@pytest.mark.parametrize("kind", ["hi", "lo", "alt"])
@pytest.mark.parametrize("cfg", ["default", "cfg24", "cfg34", "cfg40", "cfg42"])
def test_int8_p251_at_bound(kind, cfg):
    """One limb, p = 251: K = 137344 (137344 * 125^2 = 2146000000, the last k-tile
    multiple below 2^31 - 2^17) with entries +125, -125, or both alternating."""
    ffa = _ffa()
    p, n, k = 251, 256, 137344
    kw = dict(algo=ffa.ALGO_CLASSICAL)
    if cfg != "default":
        kw["kernel"] = int(cfg[3:]) + 1  # 256-tiles with 32x32x32 or 16x16x64 MFMAs (40: deferred k-step)
    d = _check_planned(n, k, p, ffa.I8_CENTRED, ffa.U8, **kw)
    assert d["max_k"] == k and d["max_abs"] == 125
    assert ffa.plan_describe(n, k + 128, p, dA=ffa.I8_CENTRED, dC=ffa.U8,
                             opts=ffa.make_opts(**kw))[0] == ffa.EBOUND
    A = _pattern(n, k, 125, p - 125, kind)
    check_syrk(A, p, torch.int8, torch.uint8, **kw)
    if kind == "alt":
        check_syrk(A, p, torch.int8, torch.uint8, levels=1)


@pytest.mark.parametrize("vals", [(65521 - 32881, 65521 - 32881), (32639, 32639), (65520, 65520),
                                  (65521 - 32881, 32639)])
@pytest.mark.parametrize("operands", ["planes", "raw"])
def test_int8x2_p65521_at_bound(vals, operands):
    """Two limbs, p = 65521: K = 65408 (2 K 128^2 < 2^31 for the middle accumulator), with
    the representatives of largest limbs -32881 (hi = -128) and 32639 (hi = 127), p - 1
    (-1), and -32881 / 32639 alternating."""
    ffa = _ffa()
    p, n, k = 65521, 256, 65408
    kw = dict(algo=ffa.ALGO_CLASSICAL,
              operands=ffa.OPERANDS_RAW if operands == "raw" else ffa.OPERANDS_PLANES)
    d = _check_planned(n, k, p, ffa.U16, ffa.U16, **kw)
    assert d["max_k"] == k and d["src"] == ("raw_u16" if operands == "raw" else "carrier")
    assert ffa.plan_describe(n, k + 128, p, dA=ffa.U16, dC=ffa.U16,
                             opts=ffa.make_opts(**kw))[0] == ffa.EBOUND
    A = _pattern(n, k, vals[0], vals[1], "alt")
    check_syrk(A, p, torch.uint16, torch.uint16, **kw)


def test_f64_direct_at_bound():
    """fp64 carrier reading canonical doubles: K (p - 1)^2 < 2^53.  p = 131071 at the largest
    K the planner admits, K = 524304, every entry p - 1 in most rows: such a dot product is
    524304 * 131070^2 = 9007199248449600, 6291392 below 2^53."""
    ffa = _ffa()
    p, n, k = 131071, 64, 524304
    d = _check_planned(n, k, p, ffa.F64, ffa.F64, algo=ffa.ALGO_CLASSICAL)
    assert d["direct"] == 1 and d["max_k"] == k and d["max_abs"] == p - 1
    assert k * (p - 1) ** 2 < 2 ** 53 <= (k + 16) * (p - 1) ** 2
    assert ffa.plan_describe(n, k + 16, p, dA=ffa.F64, dC=ffa.F64,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == ffa.EBOUND
    A = np.full((n, k), p - 1, dtype=np.int64)
    A[::3, 1::2] = 1  # some rows with other values, so that not every entry is equal
    check_syrk(A.astype(np.float64), p, torch.float64, torch.float64, algo=ffa.ALGO_CLASSICAL)


def test_f64_recursive_near_bound():
    """fp64 carrier with recursion (centred values |x| <= 65535 held in fp32): one level,
    leaf and general products of K = kpad / 2 >= 1048608, so that K 65535^2 lies between
    2^52 and 2^53; entries +65535 / -65535 alternating."""
    ffa = _ffa()
    p, n, k = 131071, 64, 2097664
    d = _check_planned(n, k, p, ffa.F64, ffa.F64, levels=1)
    assert d["levels"] == 1 and d["st32"] == 1 and d["max_abs"] == 65535
    assert 2 ** 52 <= d["max_k"] * 65535 ** 2 < 2 ** 53, d
    A = _pattern(n, k, 65535, p - 65535, "alt")
    check_syrk(A.astype(np.float64), p, torch.float64, torch.float64, levels=1)


# ------------------------------------------------------------------ FP64 carrier

@pytest.mark.parametrize("levels", [0, 1, 2, 4])
def test_f64_p65521(levels):
    A = si.uniform_residues(300, 333, 65521, 300)
    check_syrk(A.astype(np.float64), 65521, torch.float64, torch.float64, levels=levels)


def test_f64_p131071_and_131041():
    # the paper's two primes (Section 7): Y blocks for 131071, Y = sqrt(-1) I for 131041
    for p in (131071, 131041):
        A = si.uniform_residues(200, 150, p, p)
        for levels in (0, 2):
            check_syrk(A, p, torch.int64, torch.int64, levels=levels, carrier=2)


# ------------------------------------------------------------------ Hermitian product over F_p[i]

def check_herk(Ar, Ai, p, dt, **kw):
    ffa = _ffa()
    n, k = Ar.shape
    _say("herk", n, k, p, dt, kw)
    Cr, Ci = _sentinel_c(n, dt), _sentinel_c(n, dt)
    ffa.herk_modp2(_dev(Ar, dt), _dev(Ai, dt), p, C_re=Cr, C_im=Ci, **kw)
    torch.cuda.synchronize()
    er, ei = oracle.herk_modp2(Ar, Ai, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    gr, gi = _host(Cr), _host(Ci)
    assert np.array_equal(gr[low], er[low]) and np.array_equal(gi[low], ei[low])
    if n > 1:
        assert (gr[~low] == np.int64(SENTINEL[dt])).all() and (gi[~low] == np.int64(SENTINEL[dt])).all()


@pytest.mark.parametrize("base", ["2m", "4m"])
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("shape", [(130, 70), (257, 200)])
def test_herk_p65519(levels, shape, base):
    """Base case by the 2M method (Algorithm 3, one real SYRK + one real GEMM) or by
    the four real products of the complex kernel."""
    ffa = _ffa()
    n, k = shape
    Ar, Ai = si.complex_residues(n, k, 65519, 400 + n)
    hb = ffa.HERK_2M if base == "2m" else ffa.HERK_4M
    check_herk(Ar, Ai, 65519, torch.uint16, levels=levels, herk_base=hb)


@pytest.mark.parametrize("base", ["2m", "4m"])
@pytest.mark.parametrize("p", [251, 7])
def test_herk_single_limb(p, base):
    ffa = _ffa()
    Ar, Ai = si.complex_residues(200, 130, p, 500 + p)
    hb = ffa.HERK_2M if base == "2m" else ffa.HERK_4M
    for levels in (0, 1, 2):
        check_herk(Ar, Ai, p, torch.int64, levels=levels, herk_base=hb)


# ------------------------------------------------------------------ degenerate cases, errors

def test_degenerate_shapes():
    ffa = _ffa()
    # n = 0: nothing to do
    A = torch.zeros((0, 5), dtype=torch.int64, device="cuda")
    C = ffa.syrk_modp(A, 251)
    assert C.shape == (0, 0)
    # k = 0: Low(C) = 0, upper untouched
    A = torch.zeros((6, 0), dtype=torch.int64, device="cuda")
    C = _sentinel_c(6, torch.int64)
    ffa.syrk_modp(A, 251, C=C)
    got = _host(C)
    low = np.tril(np.ones((6, 6), dtype=bool))
    assert (got[low] == 0).all() and (got[~low] == -7).all()
    # one row, one column
    check_syrk(np.array([[250]], dtype=np.int64), 251, torch.int64, torch.int64)
    check_syrk(np.arange(9, dtype=np.int64).reshape(9, 1), 251, torch.int64, torch.int64, levels=2)


def test_input_range_check_forced_from_host():
    ffa = _ffa()
    A = np.full((40, 40), 3, dtype=np.int64)
    A[17, 5] = 251  # outside [0, p)
    C = _sentinel_c(40, torch.int64)
    with pytest.raises(ffa.FfaError) as e:
        ffa.syrk_modp(_dev(A, torch.int64), 251, C=C, check_inputs=True)
    assert e.value.status == ffa.ERANGE
    assert (_host(C) == -7).all()  # nothing written


def test_deterministic_repeats():
    ffa = _ffa()
    A = _dev(si.centred_int8(700, 650, 251, 9), torch.int8)
    outs = []
    for _ in range(3):
        C = ffa.syrk_modp(A, 251, levels=2)
        torch.cuda.synchronize()
        outs.append(_host(C))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


# ------------------------------------------------------------------ SYRK update form, transpose

UPDATE_CASES = [
    # p, input dtype, output dtype, alpha, beta
    (251, torch.int8, torch.uint8, 1, 0),
    (251, torch.int8, torch.uint8, 250, 17),
    (251, torch.uint8, torch.int64, 0, 3),
    (65521, torch.uint16, torch.uint16, 40000, 65520),
    (65521, torch.float64, torch.float64, 12345, 54321),
    (131071, torch.float64, torch.int64, 131070, 2),
]


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(UPDATE_CASES)))
def test_syrk_update_and_trans(case, levels, trans):
    """C <- alpha Low(op(A) op(A)^T) + beta Low(C); op(A) = A^T with trans (A is k x n)."""
    ffa = _ffa()
    p, dA, dC, alpha, beta = UPDATE_CASES[case]
    n, k = 203, 330
    shape = (k, n) if trans else (n, k)
    A_res = si.uniform_residues(*shape, p, 800 + case * 7 + levels)
    C_res = si.uniform_residues(n, n, p, 900 + case)
    _say("update", p, dA, dC, alpha, beta, levels, trans)
    if dA == torch.int8:
        A = _dev(si.to_centred(A_res, p).astype(np.int8), torch.int8)
    else:
        A = _dev(A_res, dA)
    C = _dev(C_res, dC)
    kw = dict(algo=ffa.ALGO_CLASSICAL) if levels == 0 else dict(levels=levels)
    if dA == torch.float64 and p > 65535:
        kw["carrier"] = ffa.CARRIER_F64
    ffa.syrk_modp(A, p, C=C, alpha=alpha, beta=beta, trans=trans, **kw)
    torch.cuda.synchronize()
    exp = oracle.syrk_update(A_res, C_res, p, alpha=alpha, beta=beta, trans=trans)
    assert np.array_equal(_host(C), exp)


def test_syrk_update_degenerate():
    ffa = _ffa()
    p = 251
    # k = 0: C <- beta C on the lower triangle
    C_res = si.uniform_residues(7, 7, p, 950)
    C = _dev(C_res, torch.int64)
    ffa.syrk_modp(torch.zeros((7, 0), dtype=torch.int64, device="cuda"), p, C=C, alpha=5, beta=9)
    torch.cuda.synchronize()
    low = np.tril(np.ones((7, 7), dtype=bool))
    got = _host(C)
    assert np.array_equal(got[low], (9 * C_res[low]) % p) and np.array_equal(got[~low], C_res[~low])
    # beta = 0: C is not read (it may hold values outside [0, p))
    A_res = si.uniform_residues(6, 5, p, 951)
    C = torch.full((6, 6), -12345, dtype=torch.int64, device="cuda")
    ffa.syrk_modp(_dev(A_res, torch.int64), p, C=C, alpha=3, beta=0)
    torch.cuda.synchronize()
    got = _host(C)
    low = np.tril(np.ones((6, 6), dtype=bool))
    assert np.array_equal(got[low], (3 * oracle.syrk_modp(A_res, p)[low]) % p)
    assert (got[~low] == -12345).all()
    # alpha or beta outside [0, p) is refused
    with pytest.raises(ffa.FfaError):
        ffa.syrk_modp(_dev(A_res, torch.int64), p, C=C, alpha=p, beta=0)


# ------------------------------------------------------------------ raw uint16 operands

@pytest.mark.parametrize("n", [1, 5, 130, 257])
@pytest.mark.parametrize("k", [1, 7, 8, 9, 127, 128, 129, 300, 1000])
def test_raw_u16_products_ragged_k(n, k):
    """No recursion, uint16 input with 16-byte rows: the product kernel reads the
    caller's rows and splits them into limbs when k is a multiple of 8 (it reads whole
    16-byte chunks), else the limb planes are built.  The row padding holds nonzero
    residues, which must never reach the result."""
    ffa = _ffa()
    p = 65521
    lda = (k + 7) // 8 * 8 + 8
    _say("raw u16", n, k, lda)
    big = si.uniform_residues(n, lda, p, 900 + n * 7 + k)
    Ares = big[:, :k].copy()
    st, d = ffa.plan_describe(n, k, p, dA=ffa.U16, dC=ffa.U16, lda=lda,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, operands=ffa.OPERANDS_RAW))
    assert st == 0 and d["src"] == ("raw_u16" if k % 8 == 0 else "carrier")
    A = _dev(big, torch.uint16)[:, :k]
    C = _sentinel_c(n, torch.uint16)
    ffa.syrk_modp(A, p, C=C, algo=ffa.ALGO_CLASSICAL, operands=ffa.OPERANDS_RAW)
    torch.cuda.synchronize()
    got = _host(C)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(got[low], oracle.syrk_modp(Ares, p)[low])
    assert (got[~low] == 0xBEEF).all()


def test_raw_u16_extreme_residues():
    """Residues at the edges of the limb split (around 2^15 - 128 and p - 1)."""
    ffa = _ffa()
    p = 65521
    vals = np.array([0, 1, 127, 128, 255, 256, 32639, 32640, 32767, 32768, 65407, 65408, 65519, 65520])
    n, k = 70, 264
    A = np.resize(vals, n * k).reshape(n, k)
    A[::3] = 65520
    check_syrk(A.astype(np.int64), p, torch.uint16, torch.uint16, algo=ffa.ALGO_CLASSICAL,
               operands=ffa.OPERANDS_RAW)


# ------------------------------------------------------------------ batched

def test_batched_uneven_problems():
    ffa = _ffa()
    p = 65521
    ns, ks = si.batch_shapes(24, 77, nmin=1, nmax=300)
    mats = si.batch_residues(ns, ks, p, 77)
    _say("batch", len(ns))
    for opts in (dict(), dict(levels=1)):
        B = ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16, **opts)
        Ap = B.pack(mats, np.int64)
        Cp = torch.zeros(B.c_total, dtype=torch.int32, device="cuda").to(torch.uint16)
        B.run(_dev(Ap, torch.uint16), Cp)
        torch.cuda.synchronize()
        Ch = _host(Cp)
        for i, M in enumerate(mats):
            n = int(ns[i])
            got = Ch[B.c_off[i]:B.c_off[i] + n * n].reshape(n, n)
            exp = oracle.syrk_modp(M, p)
            assert np.array_equal(np.tril(got), exp), f"problem {i} ({n}x{ks[i]})"
        B.close()


def test_batch_plan_persistent_by_default():
    ffa = _ffa()
    ns, ks = np.array([40, 300, 7]), np.array([50, 310, 9])
    B = ffa.BatchSyrk(ns, ks, 65521, ffa.U16, ffa.U16)
    assert B.describe()["persist"] == 1
    B.close()
    B = ffa.BatchSyrk(ns, ks, 65521, ffa.U16, ffa.U16, persist=ffa.PERSIST_OFF)
    assert B.describe()["persist"] == 0
    B.close()
    with pytest.raises(ffa.FfaError):
        ffa.BatchSyrk(ns, ks, 65521, ffa.U16, ffa.U16, persist=5)


def test_batch_default_operands():
    """A batch of small two-limb problems reads the caller's uint16 rows with
    configuration 39 unless limb planes or a configuration are asked for; input that is
    not uint16, or a problem of 2048 rows or more, keeps limb planes."""
    ffa = _ffa()
    ns, ks = np.array([40, 300, 7]), np.array([50, 310, 9])
    for kw, dA, src, cfg in (({}, ffa.U16, "raw_u16", 39),
                             (dict(operands=ffa.OPERANDS_PLANES), ffa.U16, "carrier", 16),
                             (dict(kernel=17), ffa.U16, "carrier", 16),
                             ({}, ffa.I64, "carrier", 16)):
        B = ffa.BatchSyrk(ns, ks, 65521, dA, ffa.U16, **kw)
        d = B.describe()
        assert d["src"] == src and d["cfg"] == cfg, (kw, dA, d)
        B.close()
    B = ffa.BatchSyrk(np.array([40, 2048]), np.array([50, 64]), 65521, ffa.U16, ffa.U16)
    d = B.describe()
    assert d["src"] == "carrier" and d["cfg"] == 32, d
    B.close()


@pytest.mark.parametrize("persist", ["on", "off"])
@pytest.mark.parametrize("cfg", [16, 21, 39])
def test_batched_raw_rows_with_nonzero_padding(cfg, persist):
    """Raw uint16 operands over the packed layout with ragged k: the row's last
    16-byte chunk is read whole and its columns past k are zeroed in the kernel.  The
    packed rows' padding is filled with nonzero residues here, which must never
    reach the result."""
    ffa = _ffa()
    p = 65521
    ns, ks = si.batch_shapes(40, 91, nmin=1, nmax=200)
    ks = ks + (ks % 8 == 0)  # every k ragged
    mats = si.batch_residues(ns, ks, p, 91)
    _say("batch raw padding", cfg, len(ns))
    B = ffa.BatchSyrk(ns, ks, p, ffa.U16, ffa.U16, algo=ffa.ALGO_CLASSICAL,
                      operands=ffa.OPERANDS_RAW, kernel=cfg + 1,
                      persist=ffa.PERSIST_ON if persist == "on" else ffa.PERSIST_OFF)
    assert B.describe()["src"] == "raw_u16" and B.describe()["persist"] == (persist == "on")
    Ap = B.pack(mats, np.int64)
    rng = np.random.default_rng(91)
    for i in range(len(ns)):
        n, k, ld, o = int(ns[i]), int(ks[i]), int(B.lda[i]), int(B.a_off[i])
        if n:
            rows = Ap[o:o + n * ld].reshape(n, ld)
            rows[:, k:] = rng.integers(1, p, (n, ld - k))
    Cp = torch.zeros(B.c_total, dtype=torch.int32, device="cuda").to(torch.uint16)
    B.run(_dev(Ap, torch.uint16), Cp)
    torch.cuda.synchronize()
    Ch = _host(Cp)
    for i, M in enumerate(mats):
        n = int(ns[i])
        got = Ch[B.c_off[i]:B.c_off[i] + n * n].reshape(n, n)
        assert np.array_equal(np.tril(got), oracle.syrk_modp(M, p)), f"problem {i} ({n}x{ks[i]})"
    B.close()


@pytest.mark.parametrize("case", ["p251-default", "p251-cfg34", "p251-cfg40", "p65521-planes", "p65521-raw",
                                  "p65521-cfg32"])
def test_persistent_product_launch(case):
    """The product launch run persistent (workgroups taking tiles from a queue per XCD)
    against the oracle, on shapes of many ragged tiles, twice in a row (the queue
    counters are cleared before each launch)."""
    ffa = _ffa()
    p = 251 if case.startswith("p251") else 65521
    n, k = (1000, 777) if p == 251 else (700, 520)
    A = si.uniform_residues(n, k, p, 4242)
    kw = dict(algo=ffa.ALGO_CLASSICAL, persist=ffa.PERSIST_ON)
    if case.endswith("cfg34"):
        kw["kernel"] = 35
    if case.endswith("cfg40"):
        kw["kernel"] = 41
    if case.endswith("cfg32"):
        kw["kernel"] = 33
    if case.endswith("raw"):
        kw["operands"] = ffa.OPERANDS_RAW
    dA = torch.int8 if p == 251 else torch.uint16
    dC = torch.uint8 if p == 251 else torch.uint16
    d = _check_planned(n, k, p, ffa.I8_CENTRED if p == 251 else ffa.U16, ffa.U8 if p == 251 else ffa.U16,
                       **kw)
    assert d["persist"] == 1 and d["blocks"] > 8
    if case.endswith("raw"):
        assert d["src"] == "raw_u16"
    for _ in range(2):
        check_syrk(A, p, dA, dC, **kw)


# ------------------------------------------------------------------ full size, sampled

def _sample_pairs(n, rng, count=3000):
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    i, j = np.maximum(i, j), np.minimum(i, j)
    edges = np.array([0, 1, 255, 256, 257, n // 2 - 1, n // 2, n - 2, n - 1])
    ei, ej = np.meshgrid(edges, edges)
    m = ei >= ej
    return np.concatenate([i, ei[m]]), np.concatenate([j, ej[m]])


@pytest.mark.parametrize("algo", ["recursive", "classical"])
def test_full_size_p251_sampled_and_freivalds(algo):
    """n = k = 16384, p = 251, int8-centred input: the benchmark's configuration."""
    ffa = _ffa()
    n = k = 16384
    p = 251
    A8 = si.centred_int8(n, k, p, si.config_seed(2))
    _say("full", n, k, p, algo)
    dA = torch.from_numpy(A8).to("cuda")
    kw = dict(algo=1) if algo == "classical" else dict(levels=1)
    C = ffa.syrk_modp(dA, p, **kw)
    torch.cuda.synchronize()
    ffa.device_status(0)
    Ch = C.cpu().numpy().astype(np.int64)
    Ares = np.mod(A8.astype(np.int64), p)
    rng = np.random.default_rng(5)
    ii, jj = _sample_pairs(n, rng)
    exp = oracle.syrk_entries(Ares, p, ii, jj)
    assert np.array_equal(Ch[ii, jj], exp)
    Cl = np.tril(Ch)
    for _ in range(4):  # false-pass probability p^-4 at most
        x = rng.integers(0, p, n)
        yc, ya = oracle.freivalds_syrk(Ares, Cl, p, x)
        assert np.array_equal(yc, ya)


# ------------------------------------------------------------------ strided A and C

@pytest.mark.parametrize("case", ["p251-i8-0", "p251-i8-1", "p65521-u16-0", "p65521-u16-2",
                                  "p65521-f64-2w", "p65519-herk-0", "p65519-herk-1",
                                  "p65521-trans-1"])
def test_strided_a_and_c(case):
    """A and C as views into larger buffers (lda > k, ldc > n): the result lands in the
    view's lower triangle and nothing else of the buffer changes."""
    ffa = _ffa()
    p = int(case.split("-")[0][1:])
    kind, lv = case.split("-")[1], case.split("-")[2]
    levels = int(lv[0])
    n, k = 203, 331
    pad_a, pad_c = 13, 21
    _say("strided", case)
    kw = dict(levels=levels)
    if lv.endswith("w"):
        kw.update(general=ffa.GENERAL_WINOGRAD, carrier=ffa.CARRIER_F64)
    if kind == "herk":
        Ar, Ai = si.complex_residues(n, k + pad_a, p, 1400)
        er, ei = oracle.herk_modp2(Ar[:, :k].copy(), Ai[:, :k].copy(), p)
        Br = torch.full((n, n + pad_c), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
        Bi = torch.full((n, n + pad_c), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
        ffa.herk_modp2(_dev(Ar, torch.uint16)[:, :k], _dev(Ai, torch.uint16)[:, :k], p,
                       C_re=Br[:, :n], C_im=Bi[:, :n], **kw)
        torch.cuda.synchronize()
        low = np.tril(np.ones((n, n), dtype=bool))
        for buf, exp in ((Br, er), (Bi, ei)):
            g = _host(buf)
            assert np.array_equal(g[:, :n][low], exp[low])
            assert (g[:, :n][~low] == 0xBEEF).all() and (g[:, n:] == 0xBEEF).all()
        return
    trans = kind == "trans"
    rows, cols = (k, n) if trans else (n, k)
    big = si.uniform_residues(rows, cols + pad_a, p, 1401 + levels)
    Ares = big[:, :cols].copy()
    exp = oracle.syrk_modp(Ares.T.copy() if trans else Ares, p)
    if kind == "i8":
        A = _dev(si.to_centred(big, p).astype(np.int8), torch.int8)[:, :cols]
        dt, sent = torch.uint8, 0xA5
    elif kind == "f64":
        A = _dev(big.astype(np.float64), torch.float64)[:, :cols]
        dt, sent = torch.uint16, 0xBEEF
    else:
        A = _dev(big, torch.uint16)[:, :cols]
        dt, sent = torch.uint16, 0xBEEF
    Bc = torch.full((n, n + pad_c), sent, dtype=torch.int32, device="cuda").to(dt)
    ffa.syrk_modp(A, p, C=Bc[:, :n], trans=trans, **kw)
    torch.cuda.synchronize()
    g = _host(Bc)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(g[:, :n][low], exp[low])
    assert (g[:, :n][~low] == sent).all() and (g[:, n:] == sent).all()


# ------------------------------------------------------------------ pre-additions beside the products

@pytest.mark.parametrize("shape", [(1000, 900), (257, 300), (2048, 1536)])
@pytest.mark.parametrize("p", [251, 241])
def test_preadditions_beside_the_product_launch(shape, p):
    """One limb, one level, streams AUTO: the pre-addition kernel runs on the context's
    second stream beside the single product launch, whose tiles that read S1..S4 wait for
    it.  Same bits as the serial plan and as the oracle; no wait gave up."""
    ffa = _ffa()
    n, k = shape
    d = ffa.plan_describe(n, k, p, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(levels=1))[1]
    assert d["overlap_pre"] == 1 and d["levels"] == 1
    d1 = ffa.plan_describe(n, k, p, dA=ffa.I8_CENTRED, dC=ffa.U8,
                           opts=ffa.make_opts(levels=1, streams=ffa.STREAMS_ONE))[1]
    assert d1["overlap_pre"] == 0
    A = si.uniform_residues(n, k, p, 900 + n + p)
    for _ in range(3):  # repeated calls reuse the counter and the workspace
        got = check_syrk(A, p, torch.int8, torch.uint8, levels=1)
    serial = check_syrk(A, p, torch.int8, torch.uint8, levels=1, streams=ffa.STREAMS_ONE)
    assert np.array_equal(np.tril(got), np.tril(serial))
    ffa.device_status(0)
