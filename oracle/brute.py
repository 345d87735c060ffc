"""Arbitrary-precision brute force for tiny inputs — TEST INFRASTRUCTURE ONLY.

A deliberately different route from the oracle's row-by-row dot products:
the full product over the integers is accumulated as a sum of outer products
of the columns of A (A*phi(A) = sum_t a_t phi(a_t), column expansion of the
matrix product), with Python integers (no overflow), and is reduced mod p only
at the end.  The Hermitian case works over the Gaussian integers Z[i]
((x + iy) * conj(u + iv) = (xu + yv) + i(yu - xv)) before reducing to
F_p[i]/(i^2+1).
"""
from __future__ import annotations


def syrk_full(A, p):
    n = len(A)
    k = len(A[0]) if n else 0
    M = [[0] * n for _ in range(n)]
    for t in range(k):
        col = [int(A[i][t]) for i in range(n)]
        for i in range(n):
            for j in range(n):
                M[i][j] += col[i] * col[j]
    return [[M[i][j] % p for j in range(n)] for i in range(n)]


def herk_full(Ar, Ai, p):
    n = len(Ar)
    k = len(Ar[0]) if n else 0
    Re = [[0] * n for _ in range(n)]
    Im = [[0] * n for _ in range(n)]
    for t in range(k):
        xr = [int(Ar[i][t]) for i in range(n)]
        xi = [int(Ai[i][t]) for i in range(n)]
        for i in range(n):
            for j in range(n):
                Re[i][j] += xr[i] * xr[j] + xi[i] * xi[j]
                Im[i][j] += xi[i] * xr[j] - xr[i] * xi[j]
    return ([[Re[i][j] % p for j in range(n)] for i in range(n)],
            [[Im[i][j] % p for j in range(n)] for i in range(n)])


def lower(M):
    n = len(M)
    return [[M[i][j] if j <= i else 0 for j in range(n)] for i in range(n)]
