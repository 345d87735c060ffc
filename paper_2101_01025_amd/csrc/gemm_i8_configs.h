// Configurations of the INT8 product kernel: id -> (limbs, complex, tile edge,
// wave grid, k-tile bytes, prefetch depth, MFMA block edge, options; depth 0 =
// direct global-to-LDS loads into two buffers).  Options: bits 0-3 = waves per
// SIMD that the register allocation must allow (0: the compiler's choice); bit 4 =
// each k-tile's last k-step multiplied after the k-tile's barrier (depth 0);
// bit 5 = the thread index's range not restated to the compiler.
// Accumulator registers per lane: NROLE * NACC * (BT/WGM/32) * (BT/WGN/32) * 16.
// Configurations whose accumulators do not fit the register file without
// spilling are left out (configuration 40 spills 44 bytes per lane around its
// k-loop, not inside it); ids are not renumbered.
// Each list holds the configurations that one translation unit instantiates, so
// that the units compile in parallel.
#pragma once

#define FFA_I8_CONFIGS_A(X)               \
    X(24, 1, 0, 256, 2, 4, 128, 0, 32, 0)   \
    X(2, 1, 0, 128, 2, 2, 128, 2, 32, 0)    \
    X(1, 1, 0, 256, 2, 4, 64, 2, 32, 0)     \
    X(14, 1, 0, 64, 2, 2, 128, 2, 32, 0)    \
    X(39, 2, 0, 64, 2, 2, 64, 2, 32, 4)

#define FFA_I8_CONFIGS_B(X)               \
    X(16, 2, 0, 128, 2, 4, 128, 2, 32, 32)  \
    X(15, 2, 0, 128, 2, 4, 128, 1, 32, 0)   \
    X(26, 2, 0, 128, 2, 4, 128, 0, 32, 0)   \
    X(9, 2, 0, 128, 2, 2, 128, 1, 32, 0)

#define FFA_I8_CONFIGS_C(X)               \
    X(10, 1, 0, 256, 2, 4, 128, 2, 32, 32)  \
    X(11, 1, 0, 256, 2, 4, 64, 3, 32, 0)    \
    X(12, 1, 0, 256, 4, 2, 64, 2, 32, 0)    \
    X(25, 2, 0, 128, 2, 2, 128, 0, 32, 0)   \
    X(13, 2, 0, 64, 2, 2, 128, 2, 32, 0)

#define FFA_I8_CONFIGS_D(X)               \
    X(4, 1, 1, 128, 2, 2, 128, 2, 32, 0)    \
    X(8, 2, 1, 64, 2, 2, 128, 2, 32, 0)     \
    X(17, 2, 0, 64, 2, 2, 64, 2, 32, 0)     \
    X(18, 2, 0, 128, 2, 4, 64, 4, 32, 0)    \
    X(21, 2, 0, 64, 2, 2, 64, 4, 32, 0)

// depth -NBUF: direct loads into NBUF buffers, issued between the k-steps
#define FFA_I8_CONFIGS_E(X)               \
    X(29, 1, 0, 256, 2, 4, 128, -2, 32, 0)  \
    X(32, 2, 0, 128, 2, 4, 128, -2, 32, 0)  \
    X(34, 1, 0, 256, 2, 4, 128, 0, 16, 32)  \
    X(35, 1, 0, 256, 2, 4, 128, -2, 16, 0)  \
    X(36, 2, 0, 128, 2, 4, 128, -2, 16, 0)  \
    X(37, 1, 0, 256, 4, 2, 128, 0, 16, 0)   \
    X(38, 1, 0, 128, 2, 2, 128, 0, 16, 0)   \
    X(40, 1, 0, 256, 2, 4, 128, 0, 16, 48)  \
    X(41, 2, 0, 128, 2, 4, 128, 0, 32, 16)  \
    X(42, 1, 0, 256, 2, 4, 128, 0, 16, 0)

#define FFA_I8_CONFIGS(X) \
    FFA_I8_CONFIGS_A(X)   \
    FFA_I8_CONFIGS_B(X)   \
    FFA_I8_CONFIGS_C(X)   \
    FFA_I8_CONFIGS_D(X)   \
    FFA_I8_CONFIGS_E(X)

// Returned by a unit's entry points for a configuration that the unit does not hold.
#define FFA_I8_NOT_HERE (-100000)
