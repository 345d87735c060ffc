"""Pins of the CPU oracle and of the plain model of Algorithm 1 (no GPU).

The oracle is checked against things other than itself: an arbitrary-precision
brute force by a different expansion, closed forms, invariants (symmetry,
Hermitian symmetry, Freivalds), exhaustive agreement with Algorithm 1 on all
inputs of two tiny fields, and the identities of the paper's correctness proof.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import alg1_model as model
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SMALL_PRIMES = [p for p in range(3, 2000) if all(p % d for d in range(2, int(p ** 0.5) + 1))]
CONFIG_PRIMES = [251, 65519, 65521, 131041, 131071]


# ---------------------------------------------------------------- field helpers

def test_is_prime_matches_sieve():
    sieve = [True] * 2000
    sieve[0] = sieve[1] = False
    for i in range(2, 2000):
        if sieve[i]:
            for j in range(i * i, 2000, i):
                sieve[j] = False
    assert [oracle.is_prime(x) for x in range(2000)] == sieve


@pytest.mark.parametrize("p", SMALL_PRIMES[:120])
def test_legendre_matches_enumerated_squares(p):
    squares = {(x * x) % p for x in range(1, p)}
    for a in range(p):
        expect = 0 if a == 0 else (1 if a in squares else -1)
        assert oracle.legendre(a, p) == expect


@pytest.mark.parametrize("p", SMALL_PRIMES + CONFIG_PRIMES)
def test_sqrt_and_sos(p):
    # Tonelli-Shanks roots square back, smaller root returned
    for a in range(1, min(p, 60)):
        r = oracle.sqrt_mod(a, p)
        if oracle.legendre(a, p) == 1:
            assert (r * r) % p == a and r <= p - r
        else:
            assert r == -1
    # Algorithm 2 with k = -1
    a, b, s = oracle.sos(p, -1)
    assert (a * a + b * b) % p == p - 1
    if p % 4 == 1:  # Proposition lemsqrt: -1 is a square, Y = sqrt(-1) I
        assert b == 0 and s == 0
    else:           # s is the least quadratic non-residue
        assert s >= 2 and oracle.legendre(s, p) == -1
        assert all(oracle.legendre(t, p) == 1 for t in range(2, s))


def test_paper_lemmas_on_primes():
    for p in SMALL_PRIMES:
        if p % 8 == 3:   # Lemma minustwo
            assert oracle.legendre(-2, p) == 1
        if p % 4 == 1:   # Proposition lemsqrt
            assert oracle.legendre(-1, p) == 1
        if p % 4 == 3:   # -1 is not a square: F_p[i]/(i^2+1) is a field
            assert oracle.legendre(-1, p) == -1


def test_sos_golden_constants():
    g = json.load(open(os.path.join(GOLDEN, "small_cases.json")))["sos_minus_one"]
    for p, v in g.items():
        assert oracle.sos(int(p), -1) == (v["a"], v["b"], v["s"])
    # p = 251 = 3 mod 8: s = 2, a = b = sqrt(125) = 80
    assert oracle.sos(251, -1) == (80, 80, 2)
    assert oracle.sos(65521, -1)[:2] == (24297, 0)


@pytest.mark.parametrize("p,herm", [(3, False), (5, False), (7, False), (251, False), (65521, False),
                                    (7, True), (65519, True), (131071, False)])
@pytest.mark.parametrize("orientation", ["halves", "pairs"])
def test_y_is_skew_unitary(p, herm, orientation):
    F = model.GaussField(p) if herm else model.PrimeField(p)
    kind, a, b = model.y_parameters(p, herm)
    for d in (2, 4, 6):
        Y = model.skew_unitary(F, d, kind, a, b, orientation)
        prod = F.mul(Y, F.phi(Y))
        minus_i = F.neg(F.eye_times(d, 1 if not herm else (1, 0)))
        assert F.equal(prod, minus_i)


# ---------------------------------------------------------------- oracle vs brute force

@pytest.mark.parametrize("p", [3, 5, 7, 251, 65519, 65521, 2147483647])
def test_syrk_vs_bigint_brute_force(p):
    rng = np.random.default_rng(p)
    for n in range(0, 7):
        for k in (0, 1, 2, 5, 8):
            A = rng.integers(0, p, size=(n, k), dtype=np.int64)
            got = oracle.syrk_modp(A, p)
            exp = brute.lower(brute.syrk_full(A.tolist(), p)) if n else []
            assert got.tolist() == exp
            full = oracle.syrk_modp(A, p, full=True)
            assert full.tolist() == (brute.syrk_full(A.tolist(), p) if n else [])


@pytest.mark.parametrize("p", [3, 7, 65519])
def test_herk_vs_bigint_brute_force(p):
    rng = np.random.default_rng(p + 1)
    for n in range(0, 6):
        for k in (0, 1, 3, 7):
            Ar = rng.integers(0, p, size=(n, k), dtype=np.int64)
            Ai = rng.integers(0, p, size=(n, k), dtype=np.int64)
            Cr, Ci = oracle.herk_modp2(Ar, Ai, p, full=True)
            if n == 0:
                continue
            er, ei = brute.herk_full(Ar.tolist(), Ai.tolist(), p)
            assert Cr.tolist() == er and Ci.tolist() == ei


def test_golden_small_cases():
    g = json.load(open(os.path.join(GOLDEN, "small_cases.json")))
    for c in g["syrk"]:
        A = si.uniform_residues(c["n"], c["k"], c["p"], c["seed"])
        assert oracle.syrk_modp(A, c["p"]).tolist() == c["C"]
    for c in g["herk"]:
        Ar, Ai = si.complex_residues(c["n"], c["k"], c["p"], c["seed"])
        Cr, Ci = oracle.herk_modp2(Ar, Ai, c["p"])
        assert Cr.tolist() == c["Cre"] and Ci.tolist() == c["Cim"]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("p", [251, 65521])
def test_special_cases(p):
    n, k = 9, 13
    assert not oracle.syrk_modp(np.zeros((n, k), np.int64), p).any()              # A = 0
    assert np.array_equal(oracle.syrk_modp(np.eye(n, dtype=np.int64), p), np.eye(n, dtype=np.int64))
    C = oracle.syrk_modp(np.full((n, k), p - 1, np.int64), p)                      # all p-1
    assert np.array_equal(C, np.tril(np.full((n, n), k % p)))
    rng = np.random.default_rng(1)
    u = rng.integers(0, p, n)
    A = np.zeros((n, k), np.int64)
    A[:, 4] = u                                                                    # one column
    assert np.array_equal(oracle.syrk_modp(A, p), np.tril(np.outer(u, u) % p))
    v = rng.integers(0, p, (n, 1))                                                 # k = 1
    assert np.array_equal(oracle.syrk_modp(v, p), np.tril((v @ v.T) % p))
    r = rng.integers(0, p, (1, 50))                                                # one row
    assert oracle.syrk_modp(r, p)[0, 0] == int(sum(int(x) ** 2 for x in r[0])) % p


def test_linearity_and_permutation():
    p = 65521
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, (11, 6))
    B = rng.integers(0, p, (11, 9))
    full = lambda X: oracle.syrk_modp(X, p, full=True)
    # column concatenation adds
    assert np.array_equal(full(np.hstack([A, B])), (full(A) + full(B)) % p)
    # scaling by alpha scales by alpha^2
    assert np.array_equal(full((7 * A) % p), (49 * full(A)) % p)
    # row permutation conjugates
    perm = rng.permutation(11)
    assert np.array_equal(full(A[perm]), full(A)[np.ix_(perm, perm)])
    # symmetry of the full product
    F = full(A)
    assert np.array_equal(F, F.T)


def test_hermitian_invariants():
    p = 65519
    rng = np.random.default_rng(4)
    Ar = rng.integers(0, p, (8, 5))
    Ai = rng.integers(0, p, (8, 5))
    Cr, Ci = oracle.herk_modp2(Ar, Ai, p, full=True)
    assert np.array_equal(Cr, Cr.T)                    # C = C^H
    assert np.array_equal(Ci, (-Ci.T) % p)
    assert not np.diag(Ci).any()                       # Im(C_ii) = 0
    # real input: Hermitian product = transpose product
    Z = np.zeros_like(Ar)
    Rr, Ri = oracle.herk_modp2(Ar, Z, p)
    assert np.array_equal(Rr, oracle.syrk_modp(Ar, p)) and not Ri.any()
    # purely imaginary input iB: (iB)(iB)^H = B B^T
    Rr, Ri = oracle.herk_modp2(Z, Ai, p)
    assert np.array_equal(Rr, oracle.syrk_modp(Ai, p)) and not Ri.any()
    # multiplying A by i leaves A A^H unchanged: i(Ar + i Ai) = -Ai + i Ar
    Sr, Si = oracle.herk_modp2((-Ai) % p, Ar, p, full=True)
    assert np.array_equal(Sr, Cr) and np.array_equal(Si, Ci)


def test_freivalds_accepts_correct_and_rejects_planted_error():
    p = 251
    A = si.uniform_residues(40, 33, p, 7)
    C = oracle.syrk_modp(A, p)
    rng = np.random.default_rng(5)
    for _ in range(4):
        x = rng.integers(0, p, 40)
        yc, ya = oracle.freivalds_syrk(A, C, p, x)
        assert np.array_equal(yc, ya)
    Cbad = C.copy()
    Cbad[17, 3] = (Cbad[17, 3] + 1) % p
    caught = 0
    for _ in range(4):
        x = rng.integers(0, p, 40)
        yc, ya = oracle.freivalds_syrk(A, Cbad, p, x)
        caught += not np.array_equal(yc, ya)
    assert caught >= 1


def test_hermitian_freivalds_accepts_and_rejects():
    p = 65519
    Ar, Ai = si.complex_residues(30, 17, p, 8)
    Cr, Ci = oracle.herk_modp2(Ar, Ai, p)
    rng = np.random.default_rng(6)
    for _ in range(3):
        xr, xi = rng.integers(0, p, 30), rng.integers(0, p, 30)
        yc, ya = oracle.freivalds_herk(Ar, Ai, Cr, Ci, p, xr, xi)
        assert np.array_equal(yc[0], ya[0]) and np.array_equal(yc[1], ya[1])
    Bad = Ci.copy()
    Bad[20, 7] = (Bad[20, 7] + 1) % p
    xr, xi = rng.integers(0, p, 30), rng.integers(0, p, 30)
    yc, ya = oracle.freivalds_herk(Ar, Ai, Cr, Bad, p, xr, xi)
    assert not (np.array_equal(yc[0], ya[0]) and np.array_equal(yc[1], ya[1]))


def test_entries_match_full():
    p = 65521
    A = si.uniform_residues(30, 21, p, 9)
    F = oracle.syrk_modp(A, p, full=True)
    rows = np.array([0, 29, 5, 3, 29])
    cols = np.array([0, 0, 17, 29, 29])
    assert np.array_equal(oracle.syrk_entries(A, p, rows, cols), F[rows, cols])
    Ar, Ai = si.complex_residues(12, 5, 65519, 3)
    Cr, Ci = oracle.herk_modp2(Ar, Ai, 65519, full=True)
    r, c = np.array([0, 11, 4]), np.array([3, 2, 4])
    er, ei = oracle.herk_entries(Ar, Ai, 65519, r, c)
    assert np.array_equal(er, Cr[r, c]) and np.array_equal(ei, Ci[r, c])


def test_error_codes():
    with pytest.raises(oracle.OracleError):
        oracle.syrk_modp(np.zeros((2, 2), np.int64), 9)      # not prime
    with pytest.raises(oracle.OracleError):
        oracle.syrk_modp(np.full((2, 2), 300), 251)          # out of range
    with pytest.raises(oracle.OracleError):
        oracle.herk_modp2(np.zeros((2, 2)), np.zeros((2, 2)), 65521)  # p = 1 mod 4


# ---------------------------------------------------------------- Algorithm 1 vs the oracle

def test_exhaustive_f3_2x4():
    """Every A in F_3^{2x4} (Y = [[1,1],[-1,1]], one level) agrees with the definition."""
    p = 3
    for vals in itertools.product(range(p), repeat=8):
        A = np.array(vals, dtype=np.int64).reshape(2, 4)
        assert np.array_equal(model.syrk(A, p, 1), oracle.syrk_modp(A, p))


def test_exhaustive_f5_2x2():
    """Every A in F_5^{2x2} (Y = 2 I since 2^2 = -1 mod 5, one level)."""
    p = 5
    for vals in itertools.product(range(p), repeat=4):
        A = np.array(vals, dtype=np.int64).reshape(2, 2)
        assert np.array_equal(model.syrk(A, p, 1), oracle.syrk_modp(A, p))


@pytest.mark.parametrize("p", [3, 7, 13, 251, 65521, 131071])
@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_model_matches_oracle_random_shapes(p, levels):
    rng = np.random.default_rng(p * 10 + levels)
    for (n, k) in [(1, 1), (2, 3), (7, 5), (16, 16), (17, 31), (24, 9), (33, 40)]:
        A = rng.integers(0, p, (n, k))
        assert np.array_equal(model.syrk(A, p, levels), oracle.syrk_modp(A, p)), (n, k)


@pytest.mark.parametrize("p", [7, 11, 65519])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_model_herk_matches_oracle(p, levels):
    rng = np.random.default_rng(p + levels)
    for (n, k) in [(2, 2), (9, 7), (16, 12)]:
        Ar = rng.integers(0, p, (n, k))
        Ai = rng.integers(0, p, (n, k))
        got = model.herk(Ar, Ai, p, levels)
        exp = oracle.herk_modp2(Ar, Ai, p)
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1])


def test_result_independent_of_y_choice():
    p = 251  # = 3 mod 8: besides Algorithm 2's (80, 80), (1, sqrt(-2)) also works (Lemma minustwo)
    r2 = oracle.sqrt_mod(p - 2, p)
    A = si.uniform_residues(20, 24, p, 5)
    ref = oracle.syrk_modp(A, p)
    for (a, b) in [(80, 80), (1, r2), (171, 80), (80, 171)]:
        assert (a * a + b * b) % p == p - 1
        for orient in ("halves", "pairs"):
            got = model.syrk(A, p, 2, ykind="blocks", ya=a, yb=b, orientation=orient)
            assert np.array_equal(got, ref)
    p = 65521  # both square roots of -1
    A = si.uniform_residues(12, 10, p, 6)
    for a in (24297, p - 24297):
        assert np.array_equal(model.syrk(A, p, 2, ykind="scalar", ya=a, yb=0), oracle.syrk_modp(A, p))


@pytest.mark.parametrize("p,herm", [(251, False), (65521, False), (65519, True)])
def test_correctness_proof_identities(p, herm):
    """The identities of the proof of Theorem complexitybound, on one level."""
    F = model.GaussField(p) if herm else model.PrimeField(p)
    rng = np.random.default_rng(7)
    shp = (10, 12)
    A = (rng.integers(0, p, shp), rng.integers(0, p, shp)) if herm else rng.integers(0, p, shp)
    A = F.red(A)
    d = {}
    C = model.low_a_phi_a(F, A, 1, dump=d)
    A11, A12, A21, A22, Y = d["A11"], d["A12"], d["A21"], d["A22"], d["Y"]
    mul, add, sub, phi, low = F.mul, F.add, F.sub, F.phi, F.low
    S2 = d["S2"]
    # eq. prf:u3
    assert F.equal(d["U3"], low(add(mul(A11, phi(A11)), mul(A12, phi(A12)))))
    # eq. prf:r1: R1 = A11 Y phi(S2) = A11 (Y phi(A22) + phi(A21))
    R1 = mul(A11, mul(Y, phi(S2)))
    assert F.equal(R1, mul(A11, add(mul(Y, phi(A22)), phi(A21))))
    # eq. prf:u1: U1 = S2 phi(S2) + R1 + phi(R1)
    assert F.equal(d["U1"], add(add(mul(S2, phi(S2)), R1), phi(R1)))
    # eq. prf:s2s2T
    R2 = mul(A21, mul(Y, phi(A22)))
    rhs = sub(sub(sub(mul(A22, phi(A22)), mul(A21, phi(A21))), R2), phi(R2))
    assert F.equal(mul(S2, phi(S2)), rhs)
    # eq. prf:r1p4
    assert F.equal(add(R1, d["P4"]), add(R2, mul(A21, phi(A21))))
    # eq. prf:u5 (full U5 = U1 + P4 + phi(P4))
    U5full = add(add(d["U1"], d["P4"]), phi(d["P4"]))
    assert F.equal(U5full, add(mul(A22, phi(A22)), mul(A21, phi(A21))))
    # P3 = phi(R2) - phi(R1) + A21 phi(A11) + A22 phi(A12) - A22 phi(A22).  The proof's
    # displayed expansion of P3 omits the last two terms; the printed U4 only follows with them.
    P3exp = add(sub(phi(R2), phi(R1)), mul(A21, phi(A11)))
    P3exp = sub(add(P3exp, mul(A22, phi(A12))), mul(A22, phi(A22)))
    assert F.equal(d["P3"], P3exp)
    assert not F.equal(d["P3"], add(sub(phi(R2), phi(R1)), mul(A21, phi(A11))))
    # eq. prf2:u4
    assert F.equal(d["U4"], add(mul(A22, phi(A12)), mul(A21, phi(A11))))
    # P1, P5 are phi-invariant: the full products equal their adjoints
    for X in (A11, d["S3"]):
        P = mul(X, phi(X))
        assert F.equal(P, phi(P))
    # the result
    if herm:
        exp = oracle.herk_modp2(A[0], A[1], p)
        assert F.equal(C, exp)
    else:
        assert F.equal(C, oracle.syrk_modp(A, p))


def test_operation_counts_against_paper():
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    # additions per level: 15/2 b^2 + 1.5 b for b x b blocks (Remark rq:7.5)
    for b in (4, 8, 16):
        st = {}
        model.syrk(np.zeros((2 * b, 2 * b), np.int64), 65521, 1, stats=st)
        c = consts["scalar_additions_per_level"]
        assert st["adds"] == c["square_coeff"] * b * b + c["linear_coeff"] * b
    # multiplications: 3 recursive + 2 general per level, leaves are lower-triangle products
    for levels in range(0, 5):
        n = k = 16 * 2 ** levels
        st = {}
        model.syrk(np.zeros((n, k), np.int64), 65521, levels, stats=st)
        nl, kl = n >> levels, k >> levels
        closed = 3 ** levels * (nl * (nl + 1) // 2) * kl + sum(
            2 * 3 ** i * (n >> (i + 1)) ** 2 * (k >> (i + 1)) for i in range(levels))
        assert st["macs"] == closed
    # leading constant: ops = 2 * MACs -> 0.8 n^3 as the depth grows (Table tab:ffcomplex)
    target = consts["aat_leading_ops_classical"]["value"]
    f = lambda l: 0.4 + 0.1 * (3 / 8) ** l   # MACs per n^2 k at depth l (Master theorem lemma)
    for levels in (1, 3, 6, 10):
        n = 2 ** 22
        macs = 3 ** levels * (n >> levels) ** 3 / 2 + sum(2 * 3 ** i * (n >> (i + 1)) ** 3
                                                          for i in range(levels))
        assert abs(macs / n ** 3 - f(levels)) < 1e-9
    assert abs(2 * f(60) - target) < 1e-12
    # depth 0 is the classical SYRK: n^3/2 MACs = n^3 operations, the prior row of the table
    assert abs(2 * f(0) - consts["aat_leading_ops_prior"]["value"]) < 1e-12


# ------------------------------------------------------------------ SYRK update form

def test_syrk_update_special_cases():
    p = 251
    A = si.uniform_residues(9, 7, p, 41)
    C = si.uniform_residues(9, 9, p, 42)
    full = oracle.syrk_modp(A, p)
    low = np.tril(np.ones((9, 9), dtype=bool))
    # alpha = 1, beta = 0: the plain product; the strict upper triangle is C's
    U = oracle.syrk_update(A, C, p)
    assert np.array_equal(U[low], full[low]) and np.array_equal(U[~low], C[~low])
    # alpha = 0: beta Low(C)
    U = oracle.syrk_update(A, C, p, alpha=0, beta=7)
    assert np.array_equal(U[low], (7 * C[low]) % p)
    # alpha = c^2: the product of cA (a square alpha scales A)
    c = 11
    U = oracle.syrk_update(A, C, p, alpha=c * c % p, beta=0)
    assert np.array_equal(U[low], oracle.syrk_modp((c * A) % p, p)[low])


def test_syrk_update_trans_and_brute_force():
    p = 13
    A = si.uniform_residues(5, 4, p, 43)          # k x n with trans: C = A^T A (4 x 4)
    C = si.uniform_residues(4, 4, p, 44)
    U = oracle.syrk_update(A, C, p, alpha=3, beta=5, trans=True)
    for i in range(4):
        for j in range(4):
            if j <= i:
                s = sum(int(A[t, i]) * int(A[t, j]) for t in range(5))
                assert U[i, j] == (3 * s + 5 * int(C[i, j])) % p
            else:
                assert U[i, j] == C[i, j]
