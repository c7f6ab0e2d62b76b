// Counter-based draws of an instance, device side.
//
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11, section 3 and Table 2): ten rounds; a round
// multiplies word 0 by M0 and word 2 by M1, splits both products into high
// and low halves and forms (hi1^w1^k0, lo1, hi0^w3^k1, lo0); the key is
// advanced by the Weyl constants between rounds.
//
// Everything the generator draws (bijections pi of both sides, rotation
// angles, supp(x*), x* values, the subgradient off the support) is a pure
// function of (seed, counter), so any thread can recompute any draw.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace l1ls {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Counter tags (third counter word) of the draws.
constexpr uint32_t kTagPerm = 0x100u;     // | side (0: n side, 1: m side, 2: support)
constexpr uint32_t kTagAngle = 0x200u;    // | side
constexpr uint32_t kTagXstar = 0x300u;
constexpr uint32_t kTagSubgrad = 0x400u;
constexpr int kAngleAttempts = 32;
constexpr int kFeistelRounds = 4;

struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

struct Key {
    uint32_t k0, k1;
};

__host__ __device__ inline Key seed_key(uint64_t seed) {
    return Key{(uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32)};
}

// Uniform double in [0, 1): the top 53 bits of the 64-bit word hi:lo.
__host__ __device__ inline double unit_double(uint32_t lo, uint32_t hi) {
    const uint64_t w = ((uint64_t)hi << 32) | lo;
    return (double)(w >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Random bijection of [0, N): a 4-round balanced Feistel network on 2h bits
// (h = ceil(ceil(log2 N) / 2)), round function = low h bits of Philox word 0
// at counter (R, round, tag, 0), then cycle-walking back into [0, N).
// ---------------------------------------------------------------------------
__host__ __device__ inline int feistel_half_bits(int64_t N) {
    int bits = 1;
    while (bits < 62 && ((int64_t)1 << bits) < N) ++bits;
    return (bits + 1) / 2;
}

__host__ __device__ inline uint64_t feistel_encrypt(uint64_t x, int half, uint32_t tag, Key key) {
    const uint64_t mask = ((uint64_t)1 << half) - 1;
    uint64_t L = x >> half, R = x & mask;
#pragma unroll
    for (int t = 0; t < kFeistelRounds; ++t) {
        const uint64_t f = philox4x32_10((uint32_t)R, (uint32_t)t, tag, 0u, key.k0, key.k1).x & mask;
        const uint64_t nl = R;
        R = L ^ f;
        L = nl;
    }
    return (L << half) | R;
}

__host__ __device__ inline uint64_t feistel_decrypt(uint64_t y, int half, uint32_t tag, Key key) {
    const uint64_t mask = ((uint64_t)1 << half) - 1;
    uint64_t L = y >> half, R = y & mask;
#pragma unroll
    for (int t = kFeistelRounds - 1; t >= 0; --t) {
        const uint64_t f = philox4x32_10((uint32_t)L, (uint32_t)t, tag, 0u, key.k0, key.k1).x & mask;
        const uint64_t nr = L;
        L = R ^ f;
        R = nr;
    }
    return (L << half) | R;
}

// pi(a): the walk visits the cycle of a inside [0, 2^(2h)), which returns to
// [0, N) at the latest when it comes back to a itself.
__host__ __device__ inline int64_t bijection(int64_t a, int64_t N, uint32_t tag, Key key) {
    const int half = feistel_half_bits(N);
    uint64_t y = feistel_encrypt((uint64_t)a, half, tag, key);
    while (y >= (uint64_t)N) y = feistel_encrypt(y, half, tag, key);
    return (int64_t)y;
}

__host__ __device__ inline int64_t bijection_inverse(int64_t i, int64_t N, uint32_t tag, Key key) {
    const int half = feistel_half_bits(N);
    uint64_t y = feistel_decrypt((uint64_t)i, half, tag, key);
    while (y >= (uint64_t)N) y = feistel_decrypt(y, half, tag, key);
    return (int64_t)y;
}

// ---------------------------------------------------------------------------
// Rotation angle of pair k of stage t (1-based) on `side`: attempt a uses the
// Philox counter (k, a, kTagAngle|side, t); U, V uniform on [-1, 1) from the
// word pairs (0,1) and (2,3); the first attempt with 0 < U^2+V^2 <= 1 gives
// (c, s) = (U, V)/sqrt(U^2+V^2), a uniform direction.  Round-to-nearest
// intrinsics keep the arithmetic free of contraction, so the values are the
// IEEE results of exactly these operations.
// ---------------------------------------------------------------------------
__device__ inline void rotation_angle(int side, int t, uint32_t k, Key key, double* c, double* s) {
    for (int a = 0; a < kAngleAttempts; ++a) {
        const U4 w = philox4x32_10(k, (uint32_t)a, kTagAngle | (uint32_t)side, (uint32_t)t, key.k0, key.k1);
        const double U = __dadd_rn(__dmul_rn(2.0, unit_double(w.x, w.y)), -1.0);
        const double V = __dadd_rn(__dmul_rn(2.0, unit_double(w.z, w.w)), -1.0);
        const double q = __dadd_rn(__dmul_rn(U, U), __dmul_rn(V, V));
        if (q > 0.0 && q <= 1.0) {
            const double r = __dsqrt_rn(q);
            *c = __ddiv_rn(U, r);
            *s = __ddiv_rn(V, r);
            return;
        }
    }
    *c = 1.0;
    *s = 0.0;
}

}  // namespace l1ls
