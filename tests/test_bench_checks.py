"""The benchmark's result checks (host side): they accept the oracle's products
and reject a single wrong entry, an unwritten entry and a written upper triangle."""
import numpy as np
import pytest

import bench
import oracle
import seeded_inputs as si

torch = pytest.importorskip("torch")


def _c(low, sentinel, dtype):
    n = low.shape[0]
    C = np.where(np.tril(np.ones((n, n), dtype=bool)), low, sentinel)
    return torch.from_numpy(C.astype(dtype))


@pytest.mark.parametrize("p,centred", [(251, True), (65521, False)])
def test_verify_syrk(p, centred):
    n, k = 300, 170
    A = si.uniform_residues(n, k, p, 5)
    Ah = si.to_centred(A, p).astype(np.int8) if centred else A
    dt = np.uint8 if p < 256 else np.uint16
    sent = 255 if p < 256 else 0xFFFF
    exp = oracle.syrk_modp(A, p)
    info = bench.verify_syrk(Ah, p, _c(exp, sent, dt), sent, 1)
    assert info["freivalds_vectors"] == 4
    for i, j, v in ((257, 3, None), (0, 0, None), (299, 299, None)):
        bad = exp.copy()
        bad[i, j] = (bad[i, j] + 1) % p
        with pytest.raises(bench.VerifyError):
            bench.verify_syrk(Ah, p, _c(bad, sent, dt), sent, 1)
    # an entry left unwritten (still the sentinel), and a written upper entry
    C = _c(exp, sent, dt)
    C[120, 7] = sent
    with pytest.raises(bench.VerifyError):
        bench.verify_syrk(Ah, p, C, sent, 1)
    C = _c(exp, sent, dt)
    C[7, 120] = 3
    with pytest.raises(bench.VerifyError):
        bench.verify_syrk(Ah, p, C, sent, 1)


def test_verify_herk():
    n, k, p = 260, 90, 65519
    Ar, Ai = si.complex_residues(n, k, p, 6)
    er, ei = oracle.herk_modp2(Ar, Ai, p)
    sent = 0xFFFF
    bench.verify_herk(Ar, Ai, p, _c(er, sent, np.int32), _c(ei, sent, np.int32), sent, 2)
    bad = ei.copy()
    bad[200, 100] = (bad[200, 100] + 5) % p
    with pytest.raises(bench.VerifyError):
        bench.verify_herk(Ar, Ai, p, _c(er, sent, np.int32), _c(bad, sent, np.int32), sent, 2)


def test_verify_batch():
    p = 65521
    ns, ks = si.batch_shapes(12, 9, nmin=8, nmax=40)
    mats = si.batch_residues(ns, ks, p, 9)
    offs, total = [], 0
    for n in ns:
        offs.append(total)
        total += int(n) * int(n)
    C = np.full(total, 0xFFFF, dtype=np.int64)
    for i, M in enumerate(mats):
        n = int(ns[i])
        g = np.where(np.tril(np.ones((n, n), dtype=bool)), oracle.syrk_modp(M, p), 0xFFFF)
        C[offs[i]:offs[i] + n * n] = g.ravel()
    info = bench.verify_batch(mats, offs, ns, p, torch.from_numpy(C), 0xFFFF, 3, whole=4)
    assert info["problems"] == 12
    i = int(np.argmax(ns))
    C[offs[i] + int(ns[i]) + 1] = (C[offs[i] + int(ns[i]) + 1] + 1) % p   # entry (1, 1) of it
    with pytest.raises(bench.VerifyError):
        bench.verify_batch(mats, offs, ns, p, torch.from_numpy(C), 0xFFFF, 3, whole=0)
