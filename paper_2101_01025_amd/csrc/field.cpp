// Host-side prime-field helpers: primality, Legendre symbol, square roots,
// and the skew-unitary parameters of Section 4.
//
//  * p = 1 mod 4: -1 is a square (Proposition lemsqrt), Y = sqrt(-1) I.
//  * p = 3 mod 4: Algorithm 2 ("SoS") gives a^2 + b^2 = -1 with b != 0 and
//    Y = [[a, b], [-b, a]] (x) I (Proposition pigeonhole).
//  * Hermitian product over F_p[i]/(i^2+1), p = 3 mod 4: Y = (a + i b) I
//    with the same (a, b) (Section 4.4): (a+ib)(a-ib) = a^2 + b^2 = -1.
// Every square root returned is the smaller of the two roots.
#include "field.h"

namespace ffa {

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p)
{
    return (uint64_t)((unsigned __int128)a * b % p);
}

uint64_t powmod(uint64_t b, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    b %= p;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, b, p);
        b = mulmod(b, b, p);
    }
    return r;
}

bool is_odd_prime(uint64_t p)
{
    if (p < 3 || (p & 1) == 0) return false;
    for (uint64_t d = 3; d * d <= p; d += 2)
        if (p % d == 0) return false;
    return true;
}

int legendre(uint64_t a, uint64_t p)
{
    a %= p;
    if (a == 0) return 0;
    return powmod(a, (p - 1) / 2, p) == 1 ? 1 : -1;
}

// Tonelli-Shanks; returns the smaller root, or UINT64_MAX for a non-residue.
uint64_t sqrt_mod(uint64_t a, uint64_t p)
{
    a %= p;
    if (a == 0) return 0;
    if (legendre(a, p) != 1) return UINT64_MAX;
    uint64_t q = p - 1;
    int s = 0;
    while ((q & 1) == 0) {
        q >>= 1;
        ++s;
    }
    uint64_t z = 2;
    while (legendre(z, p) != -1) ++z;
    uint64_t c = powmod(z, q, p), t = powmod(a, q, p), r = powmod(a, (q + 1) / 2, p);
    int m = s;
    while (t != 1) {
        int i = 0;
        for (uint64_t u = t; u != 1; u = mulmod(u, u, p)) ++i;
        uint64_t b = c;
        for (int j = 0; j < m - i - 1; ++j) b = mulmod(b, b, p);
        m = i;
        c = mulmod(b, b, p);
        t = mulmod(t, c, p);
        r = mulmod(r, b, p);
    }
    return (r <= p - r) ? r : p - r;
}

int sum_of_squares(uint64_t p, uint64_t k, uint64_t* a, uint64_t* b)
{
    if (!is_odd_prime(p)) return -1;
    k %= p;
    if (legendre(k, p) >= 0) {
        *a = sqrt_mod(k, p);
        *b = 0;
        return 0;
    }
    uint64_t s = 2;
    while (legendre(s, p) == 1) ++s;          // least quadratic non-residue
    uint64_t c = sqrt_mod(s - 1, p);          // s - 1 is a square
    uint64_t r = mulmod(k, powmod(s, p - 2, p), p);
    uint64_t x = sqrt_mod(r, p);              // k = x^2 s = x^2 (1 + c^2)
    *a = x;
    *b = mulmod(x, c, p);
    return 0;
}

int skew_unitary_params(uint64_t p, bool hermitian, int* kind, uint64_t* a, uint64_t* b)
{
    uint64_t x, y;
    if (sum_of_squares(p, p - 1, &x, &y)) return -1;
    *a = x;
    *b = y;
    if (hermitian) *kind = Y_GAUSS;
    else *kind = (y == 0) ? Y_SCALAR : Y_BLOCKS;
    return 0;
}

}  // namespace ffa
