"""Plain CPU model of Algorithm 1 (Section 3), kept for tests — TEST INFRASTRUCTURE ONLY.

It follows the algorithm's steps in the paper's order and notation: split A
into 2x2 blocks, S1..S4 with two right-multiplications by the skew-unitary Y,
the products P1, P2, P5 (recursive) and P3, P4 (general), then U1..U5, and
returns Low(A*phi(A)).  Every intermediate of the top level can be returned
so that the identities of the correctness proof can be checked.

Y is built as an explicit matrix (Section 4) and applied with a plain matrix
product, so that nothing here depends on a structured fast path:

* transpose, p = 1 mod 4: Y = sqrt(-1) * I          (Proposition "lemsqrt")
* transpose, p = 3 mod 4: Y = [[a, b], [-b, a]] (x) I  (Proposition "pigeonhole"),
  (a, b) from Algorithm 2 with k = -1
* conjugate transpose over F_p[i]/(i^2+1), p = 3 mod 4: Y = (a + i b) * I
  (Section 4.4), (a, b) from Algorithm 2 in F_p

Odd dimensions are zero-padded (Section 3 allows padding; Section 4.3 pads the
inner dimension so that the block-structured Y has even order).

Matrices over F_p are int64 arrays of canonical residues; over F_p[i] they are
pairs (re, im) of such arrays.  Every product is exact in int64 for the sizes
used in tests (k * p^2 < 2^63).
"""
from __future__ import annotations

import numpy as np

from . import sos


# ----------------------------------------------------------------------------
# scalar algebras: F_p with transpose, F_p[i]/(i^2+1) with conjugate transpose
# ----------------------------------------------------------------------------

class PrimeField:
    """Matrices over F_p; phi = transpose."""
    hermitian = False

    def __init__(self, p: int):
        self.p = int(p)

    def red(self, X):
        return np.mod(X, self.p)

    def zeros(self, r, c):
        return np.zeros((r, c), dtype=np.int64)

    def shape(self, X):
        return X.shape

    def add(self, X, Z):
        return self.red(X + Z)

    def sub(self, X, Z):
        return self.red(X - Z)

    def mul(self, X, Z):
        return self.red(X @ Z)

    def phi(self, X):
        return np.ascontiguousarray(X.T)

    def low(self, X):
        return np.tril(X)

    def block(self, X, r0, r1, c0, c1):
        return X[r0:r1, c0:c1]

    def pad(self, X, r, c):
        out = self.zeros(r, c)
        out[:X.shape[0], :X.shape[1]] = X
        return out

    def assemble(self, C11, C21, C22):
        h = C11.shape[0]
        out = self.zeros(2 * h, 2 * h)
        out[:h, :h] = C11
        out[h:, :h] = C21
        out[h:, h:] = C22
        return out

    def eye_times(self, d, s):
        return self.red(np.eye(d, dtype=np.int64) * s)

    def equal(self, X, Z):
        return np.array_equal(self.red(X), self.red(Z))

    def neg(self, X):
        return self.red(-X)


class GaussField:
    """Matrices over F_p[i]/(i^2+1), p = 3 mod 4, as (re, im) pairs; phi = conjugate transpose."""
    hermitian = True

    def __init__(self, p: int):
        if p % 4 != 3:
            raise ValueError("i^2+1 is reducible unless p = 3 mod 4")
        self.p = int(p)

    def red(self, X):
        return (np.mod(X[0], self.p), np.mod(X[1], self.p))

    def zeros(self, r, c):
        return (np.zeros((r, c), dtype=np.int64), np.zeros((r, c), dtype=np.int64))

    def shape(self, X):
        return X[0].shape

    def add(self, X, Z):
        return self.red((X[0] + Z[0], X[1] + Z[1]))

    def sub(self, X, Z):
        return self.red((X[0] - Z[0], X[1] - Z[1]))

    def mul(self, X, Z):
        xr, xi = X
        zr, zi = Z
        return self.red((xr @ zr - xi @ zi, xr @ zi + xi @ zr))

    def phi(self, X):
        return self.red((np.ascontiguousarray(X[0].T), np.ascontiguousarray(-X[1].T)))

    def low(self, X):
        return (np.tril(X[0]), np.tril(X[1]))

    def block(self, X, r0, r1, c0, c1):
        return (X[0][r0:r1, c0:c1], X[1][r0:r1, c0:c1])

    def pad(self, X, r, c):
        out = self.zeros(r, c)
        out[0][:X[0].shape[0], :X[0].shape[1]] = X[0]
        out[1][:X[1].shape[0], :X[1].shape[1]] = X[1]
        return out

    def assemble(self, C11, C21, C22):
        h = C11[0].shape[0]
        out = self.zeros(2 * h, 2 * h)
        for c in range(2):
            out[c][:h, :h] = C11[c]
            out[c][h:, :h] = C21[c]
            out[c][h:, h:] = C22[c]
        return out

    def eye_times(self, d, s):
        re, im = s
        e = np.eye(d, dtype=np.int64)
        return self.red((e * re, e * im))

    def equal(self, X, Z):
        X, Z = self.red(X), self.red(Z)
        return np.array_equal(X[0], Z[0]) and np.array_equal(X[1], Z[1])

    def neg(self, X):
        return self.red((-X[0], -X[1]))


# ----------------------------------------------------------------------------
# skew-unitary matrices (Section 4)
# ----------------------------------------------------------------------------

def y_parameters(p: int, hermitian: bool):
    """(kind, a, b) of the Y used by default.

    kind 'scalar': Y = a*I (a^2 = -1 in F_p);  kind 'blocks': Y = [[a,b],[-b,a]] (x) I;
    kind 'gauss':  Y = (a + i b)*I over F_p[i] with a^2 + b^2 = -1 in F_p.
    """
    a, b, _ = sos(p, -1)
    if hermitian:
        return "gauss", a, b
    if b == 0:
        return "scalar", a, 0
    return "blocks", a, b


def skew_unitary(F, d: int, kind: str, a: int, b: int, orientation: str = "halves"):
    """Explicit d x d skew-unitary matrix of the given kind.

    'halves' is the paper's [[aI, bI], [-bI, aI]]; 'pairs' is the equally valid
    I (x) [[a, b], [-b, a]] (adjacent columns paired).
    """
    p = F.p
    if kind == "scalar":
        return F.eye_times(d, a)
    if kind == "gauss":
        return F.eye_times(d, (a, b))
    if d % 2:
        raise ValueError("block skew-unitary matrix needs even order")
    Y = np.zeros((d, d), dtype=np.int64)
    h = d // 2
    for j in range(h):
        if orientation == "halves":
            r0, r1 = j, j + h
        else:
            r0, r1 = 2 * j, 2 * j + 1
        Y[r0, r0] = a % p
        Y[r0, r1] = b % p
        Y[r1, r0] = (-b) % p
        Y[r1, r1] = a % p
    return Y


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

def _round_up(x, m):
    return ((x + m - 1) // m) * m


def low_a_phi_a(F, A, levels: int, ykind=None, ya=None, yb=None, orientation="halves",
                dump=None, stats=None):
    """Low(A * phi(A)) by ``levels`` recursive applications of Algorithm 1.

    ``dump``: optional dict that receives the top-level intermediates
    (A11..A22, Y, S1..S4, P1..P5, U1..U5) after padding.
    ``stats``: optional dict; ``stats['macs']`` accumulates the multiplications
    of the five products (a base case m x n counts m(m+1)/2 * n, the lower
    triangle a SYRK computes; a general product h x w by w x h counts h*h*w);
    ``stats['adds']`` accumulates the scalar additions of the nine block
    additions (full blocks count every entry, half additions their lower
    triangle), not counting the multiplications by Y.
    """
    if ykind is None:
        ykind, ya, yb = y_parameters(F.p, F.hermitian)
    m, n = F.shape(A)
    if levels <= 0 or m < 2 or n < 1:
        # base case: the general product restricted to its lower triangle
        if stats is not None:
            stats["macs"] = stats.get("macs", 0) + m * (m + 1) // 2 * n
        return F.low(F.mul(A, F.phi(A)))
    # Padding (Section 3 for odd sizes; Section 4.3 for the inner dimension of
    # the block-structured Y, whose order n/2 must be even).
    mp = _round_up(m, 2)
    npad = _round_up(n, 4 if ykind == "blocks" else 2)
    Ap = F.pad(A, mp, npad)
    h, w = mp // 2, npad // 2
    A11 = F.block(Ap, 0, h, 0, w)
    A12 = F.block(Ap, 0, h, w, npad)
    A21 = F.block(Ap, h, mp, 0, w)
    A22 = F.block(Ap, h, mp, w, npad)
    Y = skew_unitary(F, w, ykind, ya, yb, orientation)
    # four additions and two multiplications by Y
    S1 = F.mul(F.sub(A21, A11), Y)
    S2 = F.sub(A22, F.mul(A21, Y))
    S3 = F.sub(S1, A22)
    S4 = F.add(S3, A12)
    if stats is not None:
        stats["adds"] = stats.get("adds", 0) + 4 * h * w + 2 * h * h + 3 * (h * (h + 1) // 2)
    # three recursive and two general products
    rec = lambda X: low_a_phi_a(F, X, levels - 1, ykind, ya, yb, orientation, stats=stats)
    P1 = rec(A11)
    P2 = rec(A12)
    P3 = F.mul(A22, F.phi(S4))
    P4 = F.mul(S1, F.phi(S2))
    P5 = rec(S3)
    if stats is not None:
        stats["macs"] = stats.get("macs", 0) + 2 * h * h * w
    # three half additions and two complete additions
    U1low = F.add(F.low(P1), F.low(P5))
    U3low = F.add(F.low(P1), F.low(P2))
    # Up(U1) = phi(Low(U1)): the full U1 takes the strict upper part from
    # phi(Low(U1)) and keeps the computed diagonal.
    up = F.phi(U1low)
    strict_up = _strict_upper(F, up)
    U1 = F.add(U1low, strict_up)
    U2 = F.add(U1, P4)
    U4 = F.add(U2, P3)
    U5low = F.add(F.low(U2), F.low(F.phi(P4)))
    C = F.assemble(U3low, U4, U5low)
    if dump is not None:
        dump.update(dict(A11=A11, A12=A12, A21=A21, A22=A22, Y=Y, S1=S1, S2=S2, S3=S3, S4=S4,
                         P1=P1, P2=P2, P3=P3, P4=P4, P5=P5, U1=U1, U2=U2, U3=U3low, U4=U4,
                         U5=U5low))
    return F.block(C, 0, m, 0, m)


def _strict_upper(F, X):
    if isinstance(X, tuple):
        return (np.triu(X[0], 1), np.triu(X[1], 1))
    return np.triu(X, 1)


def syrk(A, p, levels, **kw):
    """Low(A A^T) mod p by the model (int64 canonical residues in, out)."""
    F = PrimeField(p)
    return low_a_phi_a(F, np.mod(np.asarray(A, dtype=np.int64), p), levels, **kw)


def herk(Ar, Ai, p, levels, **kw):
    """Low(A A^H) over F_p[i]/(i^2+1) by the model; returns (re, im)."""
    F = GaussField(p)
    A = F.red((np.asarray(Ar, dtype=np.int64), np.asarray(Ai, dtype=np.int64)))
    return low_a_phi_a(F, A, levels, **kw)
