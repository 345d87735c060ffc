"""GPU parity of every INT8 product-kernel configuration.

The planner and the autotuner may pick any configuration, so each one is run
on shapes that span several of its tiles with ragged edges in both dimensions
and in K, with and without one recursion level, and compared bit-exactly with
the CPU oracle.  Two-limb real configurations are also run on raw uint16
operands.  Complex configurations run the Hermitian product.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_CFG = 48


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


def _cfg_of(n, k, p, herm, dA, dC, **opts):
    ffa = _ffa()
    st, d = ffa.plan_describe(n, k, p, hermitian=herm, dA=dA, dC=dC, opts=ffa.make_opts(**opts))
    return d["cfg"] if st == 0 else None


# (p, input, output, limbs) of the real cases
REAL = [(251, "i8", "u8", 1), (65521, "u16", "u16", 2)]
CPLX = [(251, 1), (65519, 2)]


def _real_configs():
    ffa = _ffa()
    out = []
    for cfg in range(MAX_CFG):
        for p, di, do, nl in REAL:
            dA = ffa.I8_CENTRED if di == "i8" else ffa.U16
            dC = ffa.U8 if do == "u8" else ffa.U16
            if _cfg_of(300, 520, p, False, dA, dC, kernel=cfg + 1, levels=0) == cfg:
                out.append((cfg, p))
    return out


def _cplx_configs():
    ffa = _ffa()
    out = []
    for cfg in range(MAX_CFG):
        for p, nl in CPLX:
            if _cfg_of(200, 130, p, True, ffa.I64, ffa.I64, kernel=cfg + 1, levels=0,
                       herk_base=ffa.HERK_4M) == cfg:
                out.append((cfg, p))
    return out


def _ids(cases):
    return [f"cfg{c}-p{p}" for c, p in cases]


try:
    _REAL_CASES = _real_configs()
    _CPLX_CASES = _cplx_configs()
except Exception:  # the library is not built: the tests below report it
    _REAL_CASES = [(0, 251)]
    _CPLX_CASES = [(0, 251)]


@pytest.mark.parametrize("cfg,p", _REAL_CASES, ids=_ids(_REAL_CASES))
def test_real_config(cfg, p):
    ffa = _ffa()
    n, k = 300, 520
    Ares = si.uniform_residues(n, k, p, 900 + cfg)
    exp = oracle.syrk_modp(Ares, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    if p < 256:
        A = torch.from_numpy(si.to_centred(Ares, p).astype(np.int8)).to("cuda")
        sent, dt = 0xA5, torch.uint8
    else:
        A = _u16(Ares)
        sent, dt = 0xBEEF, torch.uint16
    runs = [dict(levels=0), dict(levels=1)]
    if p >= 256:
        runs.append(dict(levels=0, operands=ffa.OPERANDS_RAW))
    for kw in runs:
        _say("config", cfg, "p", p, kw)
        C = torch.full((n, n), sent, dtype=torch.int32, device="cuda").to(dt)
        ffa.syrk_modp(A, p, C=C, kernel=cfg + 1, **kw)
        torch.cuda.synchronize()
        got = _host(C)
        assert np.array_equal(got[low], exp[low]), (cfg, kw)
        assert (got[~low] == sent).all(), (cfg, kw)


@pytest.mark.parametrize("cfg,p", _CPLX_CASES, ids=_ids(_CPLX_CASES))
def test_complex_config(cfg, p):
    ffa = _ffa()
    n, k = 200, 130
    Ar, Ai = si.complex_residues(n, k, p, 950 + cfg)
    er, ei = oracle.herk_modp2(Ar, Ai, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    for levels in (0, 1):
        _say("complex config", cfg, "p", p, "levels", levels)
        Cr = torch.full((n, n), -7, dtype=torch.int64, device="cuda")
        Ci = torch.full((n, n), -7, dtype=torch.int64, device="cuda")
        ffa.herk_modp2(torch.from_numpy(Ar).to("cuda"), torch.from_numpy(Ai).to("cuda"), p,
                       C_re=Cr, C_im=Ci, kernel=cfg + 1, levels=levels, herk_base=ffa.HERK_4M)
        torch.cuda.synchronize()
        gr, gi = _host(Cr), _host(Ci)
        assert np.array_equal(gr[low], er[low]) and np.array_equal(gi[low], ei[low]), (cfg, levels)
        assert (gr[~low] == -7).all() and (gi[~low] == -7).all()


_R2 = [c for c in _REAL_CASES if c[1] == 65521]


@pytest.mark.parametrize("cfg,p", _R2, ids=_ids(_R2))
def test_herk_2m_real_config(cfg, p):
    """The 2M base case over F_p[i] (p = 65519) with its real products on this two-limb
    configuration."""
    ffa = _ffa()
    p = 65519
    n, k = 230, 300
    Ar, Ai = si.complex_residues(n, k, p, 970 + cfg)
    er, ei = oracle.herk_modp2(Ar, Ai, p)
    low = np.tril(np.ones((n, n), dtype=bool))
    st, d = ffa.plan_describe(n, k, p, hermitian=True, dA=ffa.U16, dC=ffa.U16,
                              opts=ffa.make_opts(kernel=cfg + 1, herk_base=ffa.HERK_2M))
    assert st == 0 and d["cfg_real"] == cfg
    _say("2M real config", cfg)
    Cr = torch.full((n, n), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    Ci = torch.full((n, n), 0xBEEF, dtype=torch.int32, device="cuda").to(torch.uint16)
    ffa.herk_modp2(_u16(Ar), _u16(Ai), p, C_re=Cr, C_im=Ci, kernel=cfg + 1, herk_base=ffa.HERK_2M)
    torch.cuda.synchronize()
    gr, gi = _host(Cr), _host(Ci)
    assert np.array_equal(gr[low], er[low]) and np.array_equal(gi[low], ei[low]), cfg
    assert (gr[~low] == 0xBEEF).all() and (gi[~low] == 0xBEEF).all()
