"""ffa_syrk_modp_noalloc (the entry point that allocates no device memory) against
ffa_syrk_modp, through the C ABI: two calls in a row, the second on a smaller input,
each compared with ffa_syrk_modp's result on the same input and with the oracle; a
call that needs more than the fixed scratch is refused without writing C."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ffa():
    import paper_2101_01025_amd as ffa
    return ffa


def _host(t):
    if t.dtype == torch.uint16:
        t = t.to(torch.int32)
    return t.cpu().numpy().astype(np.int64)


def _case(n, k, p, seed):
    A = si.uniform_residues(n, k, p, seed)
    if p < 256:
        dev = torch.from_numpy(si.to_centred(A, p).astype(np.int8)).to("cuda")
        dt, sent = torch.uint8, 0xA5
    else:
        dev = torch.from_numpy(A.astype(np.int32)).to("cuda").to(torch.uint16)
        dt, sent = torch.uint16, 0xBEEF
    return A, dev, dt, sent


@pytest.mark.parametrize("order", ["large-then-small", "twice"])
def test_noalloc_matches_syrk_modp(order):
    ffa = _ffa()
    cases = [(1000, 900, 251, 2, 61), (300, 260, 65521, 2, 62)]
    if order == "twice":
        cases = [(700, 700, 65521, 1, 63), (260, 300, 251, 0, 64)]
    for n, k, p, levels, seed in cases:
        print("[case] noalloc", n, k, p, levels, flush=True)
        A, dA, dt, sent = _case(n, k, p, seed)
        st, d = ffa.plan_describe(n, k, p, dA=ffa._dtype_code(dA), dC=ffa._dtype_code(
            torch.empty(0, dtype=dt), True), opts=ffa.make_opts(levels=levels))
        assert st == 0 and d["levels"] == levels
        C_ref = torch.full((n, n), sent, dtype=torch.int32, device="cuda").to(dt)
        C_fix = torch.full((n, n), sent, dtype=torch.int32, device="cuda").to(dt)
        ffa.syrk_modp(dA, p, C=C_ref, levels=levels)
        ffa.syrk_modp_noalloc(dA, p, C_fix, levels=levels)
        torch.cuda.synchronize()
        ref, fix = _host(C_ref), _host(C_fix)
        assert np.array_equal(ref, fix), f"noalloc differs from syrk_modp ({n}x{k}, p={p})"
        low = np.tril(np.ones((n, n), dtype=bool))
        assert np.array_equal(fix[low], oracle.syrk_modp(A, p)[low])
        assert (fix[~low] == sent).all()


def test_noalloc_refuses_beyond_its_scratch():
    ffa = _ffa()
    n = k = 4096
    p = 65521
    # one level at 4096^2 with two limbs: limb planes, S blocks and P slots above 64 MiB
    st, d = ffa.plan_describe(n, k, p, dA=ffa.U16, dC=ffa.U16, opts=ffa.make_opts(levels=1))
    assert st == 0 and d["ws_bytes"] > ffa.SCRATCH_BYTES
    A, dA, dt, sent = _case(n, k, p, 65)
    C = torch.full((n, n), sent, dtype=torch.int32, device="cuda").to(dt)
    with pytest.raises(ffa.FfaError) as e:
        ffa.syrk_modp_noalloc(dA, p, C, levels=1)
    assert e.value.status == ffa.ESCRATCH
    torch.cuda.synchronize()
    assert (_host(C) == sent).all()
