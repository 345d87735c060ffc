"""Host-side tests of the C-ABI library: it loads, exports every declared
symbol, and its planner validates and plans calls without touching a GPU."""
import os
import re

import pytest

import oracle
import paper_2101_01025_amd as ffa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ffa.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(ffa_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = ffa.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(ffa.SYMBOLS) == names


def test_no_oracle_in_library_sources():
    csrc = os.path.join(ROOT, "paper_2101_01025_amd", "csrc")
    for f in os.listdir(csrc):
        if f.endswith((".hip", ".cpp", ".h")):
            txt = open(os.path.join(csrc, f)).read()
            assert "oracle" not in txt.lower(), f
    pkg = open(os.path.join(ROOT, "paper_2101_01025_amd", "__init__.py")).read()
    assert "import oracle" not in pkg


@pytest.mark.parametrize("p,herm", [(251, 0), (65521, 0), (65519, 1), (65519, 0), (3, 0), (7, 1),
                                    (131071, 0), (131041, 0)])
def test_skew_unitary_matches_independent_field_code(p, herm):
    a, b, kind = ffa.skew_unitary(p, herm)
    oa, ob, _ = oracle.sos(p, -1)
    assert (a, b) == (oa, ob)
    assert (a * a + b * b) % p == p - 1
    assert kind == (2 if herm else (0 if b == 0 else 1))


def test_skew_unitary_errors():
    with pytest.raises(ffa.FfaError):
        ffa.skew_unitary(9)
    with pytest.raises(ffa.FfaError):
        ffa.skew_unitary(65521, hermitian=True)


def test_plan_levels_padding_and_carriers():
    st, d = ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(levels=1))
    assert st == 0 and d["carrier"] == "int8" and d["limbs"] == 1 and d["direct"] == 1
    assert d["levels"] == 1 and d["npad"] == 16384 and d["kpad"] == 16384
    # built-in depth, one limb: classical at 16384, one level at 32768; two limbs: one at 16384
    assert ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8)[1]["levels"] == 0
    assert ffa.plan_describe(32768, 32768, 251, dA=ffa.I8_CENTRED, dC=ffa.U8)[1]["levels"] == 1
    assert ffa.plan_describe(16384, 16384, 65521, dA=ffa.U16, dC=ffa.U16)[1]["levels"] == 1
    assert d["ykind"] == 1 and (d["ya"], d["yb"]) == (80, 80)
    st, d = ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    # one task of 64 * 65 / 2 tiles; the 32 of its last partial round run as K-quarters
    assert d["levels"] == 0 and d["gemm_tasks"] == 1 + 4 * 32 and d["tiles"] == 64 * 65 // 2 + 3 * 32
    st, d = ffa.plan_describe(1000, 333, 65521, dA=ffa.U16, dC=ffa.U16, opts=ffa.make_opts(levels=3))
    assert st == 0 and d["limbs"] == 2 and d["levels"] == 3 and d["direct"] == 0
    assert d["npad"] % 8 == 0 and d["kpad"] % (64 * 8) == 0 and d["kpad"] >= 333
    assert d["preadd_tasks"] == [1, 3, 9] and d["postadd_tasks"] == [1, 3, 9]
    # 27 leaves and two general products per node, plus two or four K-pieces per split tile
    extra = d["gemm_tasks"] - (27 + 2 * (1 + 3 + 9))
    assert 2 * d["tail_tiles"] <= extra <= 4 * d["tail_tiles"], d
    # fp64 carrier: with recursion the blocks are conditioned into fp32 storage (exact
    # below 2^24; half the additions' traffic), without it the products read the doubles
    st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.F64)
    assert st == 0 and d["carrier"] == "f64" and d["levels"] == 4 and d["direct"] == 0
    assert d["conditioning"] == 1 and d["st32"] == 1
    st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.F64,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["direct"] == 1 and d["st32"] == 0
    st, d = ffa.plan_describe(4096, 8192, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["complex"] == 1 and d["ykind"] == 2


def test_plan_operand_source():
    # no recursion, uint16 rows on 16-byte boundaries: raw operands on request
    st, d = ffa.plan_describe(300, 200, 65521, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, operands=ffa.OPERANDS_RAW))
    assert st == 0 and d["src"] == "raw_u16" and d["conditioning"] == 0 and d["direct"] == 1
    st, d = ffa.plan_describe(300, 200, 65521, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["src"] == "carrier" and d["conditioning"] == 1
    # unaligned rows, recursion, another input format, one limb, complex: carriers
    for kw in (dict(k=201), dict(levels=1), dict(dA=ffa.I32), dict(p=251, dC=ffa.U8),
               dict(hermitian=True, p=65519)):
        args = dict(n=300, k=200, p=65521, dA=ffa.U16, dC=ffa.U16)
        levels = kw.pop("levels", 0)
        herm = kw.pop("hermitian", False)
        args.update(kw)
        o = ffa.make_opts(levels=1, operands=ffa.OPERANDS_RAW) if levels else \
            ffa.make_opts(algo=ffa.ALGO_CLASSICAL, operands=ffa.OPERANDS_RAW)
        st, d = ffa.plan_describe(args["n"], args["k"], args["p"], hermitian=herm, dA=args["dA"],
                                  dC=args["dC"], opts=o)
        assert st == 0 and d["src"] == "carrier", (kw, d)
    # raw operands are split into limbs between registers and LDS: a product kernel that
    # loads straight into LDS (two-limb configurations 25 and 26) reads carrier planes
    for cfg, src in ((16, "raw_u16"), (25, "carrier"), (26, "carrier")):
        st, d = ffa.plan_describe(300, 200, 65521, dA=ffa.U16, dC=ffa.U16,
                                  opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, operands=ffa.OPERANDS_RAW,
                                                     kernel=cfg + 1))
        assert st == 0 and d["cfg"] == cfg and d["src"] == src, (cfg, d)


def test_default_product_configurations():
    # one limb: 128-tiles below 2048 rows per leaf, else 8 waves of 128x64 on 256-tiles with
    # direct loads and 16x16x64 MFMAs; two limbs: 128-tiles, direct loads into two buffers
    # from 2048 rows, else a register ring
    for n, cfg in ((1024, 2), (2048, 34), (16384, 34)):
        st, d = ffa.plan_describe(n, n, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                                  opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
        assert st == 0 and d["cfg"] == cfg and d["tile"] == (128 if cfg == 2 else 256), (n, d)
    st, d = ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(levels=1))
    # centred int8 input is read in place by the pre-additions and products; recursive
    # plans take the same kernel with the thread index's range restated (configuration 42)
    assert st == 0 and d["levels"] == 1 and d["cfg"] == 42 and d["direct"] == 1 and d["conditioning"] == 0
    st, d = ffa.plan_describe(16384, 16384, 65521, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["cfg"] == 32
    st, d = ffa.plan_describe(1024, 1024, 65521, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["cfg"] == 16


def test_plan_product_groups_and_streams():
    # one level: P1, P2 read only A (group 1), P3, P4, P5 need the pre-additions
    st, d = ffa.plan_describe(4096, 4096, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(levels=1, streams=ffa.STREAMS_TWO))
    assert st == 0 and d["streams"] == 2
    assert ffa.plan_describe(4096, 4096, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                             opts=ffa.make_opts(levels=1))[1]["streams"] == 1
    st1, d1 = ffa.plan_describe(4096, 4096, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                                opts=ffa.make_opts(levels=1, streams=ffa.STREAMS_ONE))
    assert st1 == 0 and d1["streams"] == 1 and d1["blocks_a_only"] == d1["blocks"]
    assert 0 < d["blocks_a_only"] < d["blocks"] and d["tiles"] == d1["tiles"]
    # no recursion: one group, one stream
    st, d = ffa.plan_describe(4096, 4096, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert d["streams"] == 1 and d["blocks_a_only"] == d["blocks"]
    assert ffa.plan_describe(10, 10, 251, opts=ffa.make_opts(streams=3))[0] == ffa.EINVAL
    assert ffa.plan_describe(10, 10, 251, opts=ffa.make_opts(operands=3))[0] == ffa.EINVAL


def test_plan_persistent_product_launch():
    # single calls: persistent on request only, never beside the pre-additions or split
    # over two streams (batches, planned with a device context, in the GPU tests)
    kw = dict(dA=ffa.I8_CENTRED, dC=ffa.U8)
    assert ffa.plan_describe(2048, 2048, 251, opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL), **kw)[1]["persist"] == 0
    st, d = ffa.plan_describe(2048, 2048, 251, opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL,
                                                                  persist=ffa.PERSIST_ON), **kw)
    st0, d0 = ffa.plan_describe(2048, 2048, 251, opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL), **kw)
    assert st == 0 and d["persist"] == 1 and d["ws_bytes"] == d0["ws_bytes"] + 256  # the queue counters
    st, d = ffa.plan_describe(4096, 4096, 251, opts=ffa.make_opts(levels=1, persist=ffa.PERSIST_ON), **kw)
    assert st == 0 and d["overlap_pre"] == 1 and d["persist"] == 0
    st, d = ffa.plan_describe(4096, 4096, 251, opts=ffa.make_opts(levels=1, streams=ffa.STREAMS_TWO,
                                                                  persist=ffa.PERSIST_ON), **kw)
    assert st == 0 and d["streams"] == 2 and d["persist"] == 0
    for bad in (-1, 3):
        assert ffa.plan_describe(10, 10, 251, opts=ffa.make_opts(persist=bad))[0] == ffa.EINVAL


def test_plan_herk_base_case_2m():
    # no recursion: 2M = one real SYRK (n(n+1)/2 k) + one real GEMM (n^2 k); 4M = four
    # real products on the lower triangle
    n, k = 512, 384
    st, d = ffa.plan_describe(n, k, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["herk_base"] == "2m" and d["real_tasks"] == 2 and d["gemm_tasks"] == 0
    assert d["macs"] == n * (n + 1) // 2 * k + n * n * k
    st, d = ffa.plan_describe(n, k, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, herk_base=ffa.HERK_4M))
    assert st == 0 and d["herk_base"] == "4m" and d["real_tasks"] == 0
    assert d["macs"] == 4 * n * (n + 1) // 2 * k
    # one level: three 2M leaves, the general products P3, P4 stay complex
    st, d = ffa.plan_describe(n, k, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(levels=1))
    assert st == 0 and d["real_tasks"] == 6 and d["gemm_tasks"] == 2
    assert ffa.plan_describe(n, k, 65519, hermitian=True, opts=ffa.make_opts(herk_base=3))[0] == ffa.EINVAL
    # a long H = Xr Xi^T goes in two halves over K (three real products per leaf, same MACs)
    st, d = ffa.plan_describe(4096, 8192, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["real_tasks"] == 3
    assert d["macs"] == 4096 * 4097 // 2 * 8192 + 4096 * 4096 * 8192
    st, d = ffa.plan_describe(200, 130, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["real_tasks"] == 2
    # the kernel option: a real two-limb configuration selects the 2M real products'
    st, d0 = ffa.plan_describe(n, k, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d0["cfg_real"] >= 0
    st, d1 = ffa.plan_describe(n, k, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                               opts=ffa.make_opts(kernel=14))   # configuration 13: 64-tiles
    assert st == 0 and d1["cfg_real"] == 13 and d1["cfg"] == d0["cfg"]


def test_plan_winograd_general_products():
    # one level of Algorithm 1, P3 and P4 each by Strassen-Winograd: 3 leaves + 2 x 7 products
    n = k = 4096
    st, d = ffa.plan_describe(n, k, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(levels=1, general=ffa.GENERAL_WINOGRAD))
    # (plus two or four K-pieces per tile of the launch's split last round)
    extra = d["gemm_tasks"] - 17
    assert st == 0 and d["general"] == "winograd" and d["wino_tasks"] == 2
    assert 2 * d["tail_tiles"] <= extra <= 4 * d["tail_tiles"], d
    h, w = n // 2, k // 2
    assert d["macs"] == 3 * (h * (h + 1) // 2) * w + 2 * 7 * (h // 2) ** 2 * (w // 2)
    # rows and columns are padded one halving deeper
    st, d = ffa.plan_describe(1000, 333, 65521, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(levels=2, general=ffa.GENERAL_WINOGRAD))
    assert st == 0 and d["npad"] % 8 == 0 and d["kpad"] % (128 << 3) == 0
    # no recursion: no general products, nothing changes
    st, d = ffa.plan_describe(n, k, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, general=ffa.GENERAL_WINOGRAD))
    assert st == 0 and d["general"] == "classical"
    assert ffa.plan_describe(10, 10, 251, opts=ffa.make_opts(general=3))[0] == ffa.EINVAL
    # default: Winograd on the fp64 carrier only, on general products of 2048 rows and more
    st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.F64)
    assert st == 0 and d["levels"] == 4 and d["general"] == "winograd" and d["wino_min"] == 2048
    assert d["wino_tasks"] == 2 + 2 * 3          # levels 0 and 1 (4096 and 2048 rows)
    h = [8192 >> (i + 1) for i in range(4)]
    macs = 81 * h[3] * (h[3] + 1) // 2 * h[3]          # the leaves: 512 x 512 SYRKs
    for i in range(4):
        m = h[i]
        if m >= 2048:
            macs += 2 * 3 ** i * 7 * (m // 2) ** 3
        else:
            macs += 2 * 3 ** i * m ** 3
    assert d["macs"] == macs
    # an explicit threshold, and every general product under the Winograd option
    for wmin, tasks in ((4096, 2), (1, 2 + 6 + 18 + 54)):
        st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.F64,
                                  opts=ffa.make_opts(wino_min=wmin))
        assert st == 0 and d["wino_tasks"] == tasks
    st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.F64,
                              opts=ffa.make_opts(general=ffa.GENERAL_WINOGRAD))
    assert st == 0 and d["wino_tasks"] == 80 and d["wino_min"] == 0
    assert ffa.plan_describe(10, 10, 251, opts=ffa.make_opts(wino_min=-1))[0] == ffa.EINVAL
    assert ffa.plan_describe(8192, 8192, 65521, dA=ffa.U16, dC=ffa.U16,
                             opts=ffa.make_opts(levels=1))[1]["general"] == "classical"


def test_plan_macs_follow_recursion():
    # products MACs = 3^l leaf SYRKs + 2 * 3^i general products of level i
    for L in range(0, 4):
        n = k = 4096
        st, d = ffa.plan_describe(n, k, 251, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(levels=L))
        nl, kl = n >> L, k >> L
        exp = 3 ** L * nl * (nl + 1) // 2 * kl + sum(2 * 3 ** i * (n >> (i + 1)) ** 2 * (k >> (i + 1))
                                                   for i in range(L))
        assert d["macs"] == exp


def test_plan_errors():
    assert ffa.plan_describe(10, 10, 9)[0] == ffa.EPRIME            # not prime
    assert ffa.plan_describe(10, 10, 2)[0] == ffa.EPRIME            # even
    assert ffa.plan_describe(10, 10, 65521, hermitian=True)[0] == ffa.EUNSUPPORTED
    assert ffa.plan_describe(10, 10, 251, lda=5)[0] == ffa.EINVAL   # lda < k
    assert ffa.plan_describe(10, 10, 251, ldc=5)[0] == ffa.EINVAL   # ldc < n
    assert ffa.plan_describe(-1, 10, 251)[0] == ffa.EINVAL
    assert ffa.plan_describe(10, 10, 65521, dA=ffa.U8, dC=ffa.U16)[0] == ffa.EINVAL  # p > 255 in u8
    assert ffa.plan_describe(10, 10, 65521, dA=ffa.U16, dC=ffa.U8)[0] == ffa.EINVAL
    assert ffa.plan_describe(10, 10, 65521, dA=ffa.I8_CENTRED, dC=ffa.U16)[0] == ffa.EINVAL
    assert ffa.plan_describe(10, 10, 131071, dA=ffa.I64, dC=ffa.I64,
                             opts=ffa.make_opts(carrier=ffa.CARRIER_INT8))[0] == ffa.EPRIME
    assert ffa.plan_describe(10, 10, 65519, hermitian=True, dA=ffa.F64, dC=ffa.F64)[0] == 0
    assert ffa.plan_describe(10, 10, 65519, hermitian=True, dA=ffa.F64, dC=ffa.F64,
                             opts=ffa.make_opts(carrier=ffa.CARRIER_F64))[0] == ffa.EUNSUPPORTED
    # exact-accumulation bounds (k a multiple of the k-tile): one limb p=251: k 125^2 < 2^31 - 2^17
    assert ffa.plan_describe(4, 137344, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == 0
    assert ffa.plan_describe(4, 137472, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == ffa.EBOUND
    # two limbs: 2 * k * 128^2 < 2^31
    assert ffa.plan_describe(4, 65408, 65521, dA=ffa.U16, dC=ffa.U16,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == 0
    assert ffa.plan_describe(4, 65536, 65521, dA=ffa.U16, dC=ffa.U16,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == ffa.EBOUND
    # fp64: k (p-1)^2 < 2^53 for canonical direct input
    assert ffa.plan_describe(4, 2098176, 65521, dA=ffa.F64, dC=ffa.F64,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == 0
    assert ffa.plan_describe(4, 2098192, 65521, dA=ffa.F64, dC=ffa.F64,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == ffa.EBOUND


def test_degenerate_plans():
    st, d = ffa.plan_describe(0, 10, 251)
    assert st == 0 and d["gemm_tasks"] == 0
    st, d = ffa.plan_describe(5, 0, 251)
    assert st == 0 and d["levels"] == 0 and d["gemm_tasks"] == 1
    st, d = ffa.plan_describe(1, 7, 251, opts=ffa.make_opts(levels=3))
    assert st == 0 and d["levels"] == 0


def test_plan_refuses_operands_beyond_32bit_offsets():
    # two-limb carrier: two planes of n*k bytes must stay addressable with 32-bit offsets
    assert ffa.plan_describe(16384, 16384, 65521, dA=ffa.U16, dC=ffa.U16)[0] == 0
    assert ffa.plan_describe(50000, 50000, 65521, dA=ffa.I32, dC=ffa.U16,
                             opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))[0] == ffa.EUNSUPPORTED
    # raw uint16 operands have no limb planes: only a tile of rows must be addressable
    st, d = ffa.plan_describe(50000, 50000, 65521, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["src"] == "raw_u16"


def test_plans_keep_every_task_inside_the_workspace():
    """Every plan checks on the host that the bytes its product and addition tasks
    touch lie inside its workspace (status EINVAL otherwise): a sweep of ragged
    shapes, depths and options must plan cleanly."""
    import itertools
    cases = [
        (251, ffa.I8_CENTRED, ffa.U8, False, {}),
        (251, ffa.U8, ffa.U8, False, dict(general=ffa.GENERAL_WINOGRAD)),
        (65521, ffa.U16, ffa.U16, False, {}),
        (65521, ffa.U16, ffa.U16, False, dict(general=ffa.GENERAL_WINOGRAD)),
        (65521, ffa.F64, ffa.F64, False, dict(carrier=ffa.CARRIER_F64)),
        (131071, ffa.I64, ffa.I32, False, dict(carrier=ffa.CARRIER_F64)),
        (65519, ffa.U16, ffa.U16, True, dict(herk_base=ffa.HERK_2M)),
        (65519, ffa.U16, ffa.U16, True, dict(herk_base=ffa.HERK_4M)),
        (251, ffa.I64, ffa.I64, True, {}),
    ]
    for (p, dA, dC, herm, kw), (n, k), levels in itertools.product(
            cases, [(1, 1), (7, 300), (129, 130), (300, 520), (1000, 333), (2049, 700)], range(4)):
        st, d = ffa.plan_describe(n, k, p, hermitian=herm, dA=dA, dC=dC,
                                  opts=ffa.make_opts(levels=levels, **kw))
        assert st == 0, (p, herm, kw, n, k, levels, st)


def test_last_round_split():
    # one level at 16384^2, p = 251: 3632 tiles of 256 on 8 XCDs of 32 CUs leave 6 tiles
    # past 14 full rounds on each XCD; they run as four K-quarters each
    st, d = ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(levels=1))
    assert st == 0 and d["tail_tiles"] == 48 and d["tiles"] == 3632 + 3 * 48, d
    # the classical product: 2080 tiles, 4 past 8 full rounds per XCD
    st, d = ffa.plan_describe(16384, 16384, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["tail_tiles"] == 32 and d["tiles"] == 2080 + 3 * 32, d
    # two limbs, one level: 14432 tiles of 128 leave 12 per XCD, too many for quarters: halves
    st, d = ffa.plan_describe(16384, 16384, 65521, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["tail_tiles"] == 96 and d["tiles"] == 14432 + 96, d
    st, d = ffa.plan_describe(3712, 1024, 65521, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["tail_tiles"] == 15 and d["gemm_tasks"] == 1 + 2 * 15, d
    # not split: a last round fuller than a half, K not a multiple of four (two) k-tiles,
    # two streams, the fp64 carrier, F_p[i]
    for args, kw in (((4096, 4096, 251), dict(algo=ffa.ALGO_CLASSICAL)),
                     ((2304, 2560 - 128, 251), dict(algo=ffa.ALGO_CLASSICAL)),
                     ((16384, 16384, 251), dict(levels=1, streams=ffa.STREAMS_TWO))):
        st, d = ffa.plan_describe(*args, dA=ffa.I8_CENTRED, dC=ffa.U8, opts=ffa.make_opts(**kw))
        assert st == 0 and d["tail_tiles"] == 0, (args, kw, d)
    st, d = ffa.plan_describe(8192, 8192, 65521, dA=ffa.F64, dC=ffa.U16)
    assert st == 0 and d["tail_tiles"] == 0
    st, d = ffa.plan_describe(4096, 8192, 65519, hermitian=True, dA=ffa.U16, dC=ffa.U16)
    assert st == 0 and d["tail_tiles"] == 0
    # quarters that do not divide K (22 k-tiles of 128 bytes): halves instead
    st, d = ffa.plan_describe(2304, 2816, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL))
    assert st == 0 and d["tail_tiles"] > 0 and d["gemm_tasks"] == 1 + 2 * d["tail_tiles"], d
    # a configuration whose LDS lets two workgroups share a CU (128-tiles, 64 KiB): its
    # rounds are not 32 tiles per XCD, so nothing is split
    st, d = ffa.plan_describe(4352, 1024, 251, dA=ffa.I8_CENTRED, dC=ffa.U8,
                              opts=ffa.make_opts(algo=ffa.ALGO_CLASSICAL, kernel=3))
    assert st == 0 and d["cfg"] == 2 and d["tail_tiles"] == 0, d


def test_sizes_beyond_the_limits_are_refused_quickly():
    # n above FFA_N_MAX (its C would not fit one GPU) is refused before any table is built
    # (a plan of 2^24 rows used to try to build a schedule of 2^31 tiles on the host)
    assert ffa.plan_describe(1 << 19, 16, 251, dA=ffa.I8_CENTRED, dC=ffa.U8)[0] == ffa.OK
    for n in ((1 << 19) + 1, 1 << 24, 1 << 40):
        assert ffa.plan_describe(n, 16, 251, dA=ffa.I8_CENTRED, dC=ffa.U8)[0] == ffa.EINVAL
    assert ffa.plan_describe(16, 1 << 31, 251, dA=ffa.I8_CENTRED, dC=ffa.U8)[0] == ffa.EINVAL


_ENOMEM_PROBE = r"""
import ctypes, resource, sys
sys.path.insert(0, {root!r})
import paper_2101_01025_amd as ffa
L = ffa.lib()
vm = [int(l.split()[1]) * 1024 for l in open('/proc/self/status') if l.startswith('VmSize')][0]
# 256 MiB of address space beyond what is mapped now: the schedule of this plan
# (2^19 rows in 64-row tiles, 2^25 tiles) needs more
resource.setrlimit(resource.RLIMIT_AS, (vm + (256 << 20), resource.RLIM_INFINITY))
o = ffa.make_opts(kernel=15)
buf = ctypes.create_string_buffer(256)
st = L.ffa_plan_describe(1 << 19, 4096, 251, 0, ffa.I8_CENTRED, ffa.U8, 4096, 1 << 19,
                         ctypes.byref(o), buf, 256)
print("status", st)
"""


def test_host_allocation_failure_returns_enomem():
    # A failing host allocation inside an entry point becomes FFA_ENOMEM instead of an
    # exception crossing the C interface (which would terminate the caller's process).
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", _ENOMEM_PROBE.format(root=ROOT)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "status %d" % ffa.ENOMEM in r.stdout, r.stdout


def test_binding_refuses_outputs_it_cannot_write():
    import torch
    dev = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="tensor on"):
        ffa._out(torch.zeros((4, 4), dtype=torch.uint8), 4, dev, torch.uint8)


class _FakeTensor:
    """Stands in for a device tensor in the binding's argument checks (no GPU here)."""

    def __init__(self, dtype, numel, cuda=True, index=0, contiguous=True):
        import torch
        self.dtype, self._numel, self.is_cuda = dtype, numel, cuda
        self.device = torch.device("cuda", index) if cuda else torch.device("cpu")
        self._contiguous = contiguous

    def numel(self):
        return self._numel

    def is_contiguous(self):
        return self._contiguous


def test_batch_run_checks_its_packed_buffers():
    import torch
    b = ffa.BatchSyrk.__new__(ffa.BatchSyrk)
    b.handle, b.device_index, b.dA, b.dC, b.a_total, b.c_total = 1, 0, ffa.U16, ffa.U16, 100, 50
    ok_a, ok_c = _FakeTensor(torch.uint16, 100), _FakeTensor(torch.uint16, 50)
    b._packed(ok_a, b.dA, b.a_total, "A_packed", False)
    b._packed(ok_c, b.dC, b.c_total, "C_packed", True)
    bad = [(_FakeTensor(torch.uint16, 100, cuda=False), "tensor on"),
           (_FakeTensor(torch.uint16, 100, index=1), "tensor on"),
           (_FakeTensor(torch.int32, 100), "dtype"),
           (_FakeTensor(torch.uint16, 100, contiguous=False), "contiguous"),
           (_FakeTensor(torch.uint16, 99), "elements")]
    for t, msg in bad:
        with pytest.raises(ValueError, match=msg):
            b._packed(t, b.dA, b.a_total, "A_packed", False)
    b.handle = None
    with pytest.raises(ValueError, match="closed"):
        b._packed(ok_a, b.dA, b.a_total, "A_packed", False)


def test_short_centred_reduction_is_exact_for_every_small_prime():
    # The kernels' reduction of short sums (|v| <= 3 (p-1)/2) for p < 2^8:
    # q = (v * round(2^20 / p) + 2^19) >> 20 (arithmetic shift), v - q p, must give the
    # centred residue for every odd prime p < 256 and every v in range.
    import numpy as np
    for p in range(3, 256, 2):
        if not oracle.is_prime(p):
            continue
        half = (p - 1) // 2
        r20 = ((1 << 20) + p // 2) // p
        v = np.arange(-3 * half, 3 * half + 1, dtype=np.int64)
        q = (v * r20 + (1 << 19)) >> 20
        got = v - q * p
        want = np.mod(v + half, p) - half
        assert np.array_equal(got, want), p
        assert (np.abs(v * r20) < 2 ** 31).all() and r20 < 2 ** 23


def _fast_mod_emulated(x, p):
    """The product kernel's six-operation reduction, emulated exactly on the host:
    t = fp32 fma(fp32(x), fp32(1/p), 1.5 * 2^23) (the product of two fp32 values and the
    sum are exact in fp64, then rounded once to fp32), q = bits(t) - bits(1.5 * 2^23),
    r = x - q p, canonical = min(r, r + p) as unsigned 32-bit values."""
    import numpy as np
    xf = x.astype(np.float32).astype(np.float64)
    inv = np.float64(np.float32(1.0 / p))
    t = (xf * inv + 12582912.0).astype(np.float32)
    q = t.view(np.int32).astype(np.int64) - int(np.float32(12582912.0).view(np.int32))
    r = x - q * p
    ru = np.mod(r, 2 ** 32)
    rp = np.mod(r + p, 2 ** 32)
    return np.minimum(ru, rp)


def test_fast_epilogue_reduction_is_exact_below_its_bound():
    # the kernel takes it when K ((p-1)/2)^2 < 2^22 p, i.e. every accumulator |x| < 2^22 p
    import numpy as np
    rng = np.random.default_rng(0)
    for p in [3, 5, 7, 11, 13, 61, 127, 131, 241, 251]:
        lim = (1 << 22) * p - 1
        x = np.concatenate([rng.integers(-lim, lim + 1, 200000),
                            np.array([-lim, lim, 0, 1, -1, p, -p, p - 1, -(p - 1)])])
        mult = rng.integers(-(lim // p), lim // p + 1, 100000) * p
        x = np.concatenate([x, mult - 1, mult, mult + 1]).astype(np.int64)
        x = x[np.abs(x) <= lim]
        assert np.array_equal(_fast_mod_emulated(x, p), np.mod(x, p)), p
