// Host-side prime-field helpers used by the planner (Section 4 of the paper).
#pragma once
#include <stdint.h>

#include "ffa_internal.h"

namespace ffa {

uint64_t powmod(uint64_t b, uint64_t e, uint64_t p);
bool is_odd_prime(uint64_t p);
int legendre(uint64_t a, uint64_t p);
uint64_t sqrt_mod(uint64_t a, uint64_t p);
// Algorithm 2: a^2 + b^2 = k mod p (returns 0 on success).
int sum_of_squares(uint64_t p, uint64_t k, uint64_t* a, uint64_t* b);
// Y used for p: kind (YKind) and coefficients; hermitian selects Section 4.4.
int skew_unitary_params(uint64_t p, bool hermitian, int* kind, uint64_t* a, uint64_t* b);

}  // namespace ffa
