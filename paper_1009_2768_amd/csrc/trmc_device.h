// trmc_device.h -- device helpers of libtrmc: counter-based random numbers, the
// written exp(-x), the majorant grid, the keyed permutation of roles, and
// deterministic block reductions.  gfx950, wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trmc_internal.h"

namespace trmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  Key {seed, uid},
// counter {index, tag << 24 | aux, cell, step}.
// ---------------------------------------------------------------------------
enum : uint32_t { TAG_SPLIT = 1, TAG_PERM = 2, TAG_TREE = 3, TAG_COLL = 4, TAG_MAXW = 5, TAG_INJ = 6 };

struct Key {
    uint32_t seed, uid, cell, step;
};

// Pointers known to address global memory: loads and stores become global_*
// instructions (scalar base + vector offset, counted by vmcnt only) instead of
// flat ones, which also count against the LDS wait counter.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p)
{
    return (gptr<T>)p;
}

// Values equal on every lane of a wave, moved to scalar registers (the first
// active lane's copy): cell indices, sizes, keys and base pointers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(v))); }
template <typename P>
__device__ __forceinline__ P* uni(P* p)
{
    return reinterpret_cast<P*>(uni((uint64_t)reinterpret_cast<uintptr_t>(p)));
}
__device__ __forceinline__ Key uni(const Key& k) { return Key{uni(k.seed), uni(k.uid), uni(k.cell), uni(k.step)}; }

__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 product each (v_mad_u64_u32) instead of separate low and
        // high halves (v_mul_lo_u32 + v_mul_hi_u32): half the multiplies
        const uint64_t pa = (uint64_t)0xD2511F53u * c0, pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo_a = (uint32_t)pa, hi_a = (uint32_t)(pa >> 32);
        const uint32_t lo_b = (uint32_t)pb, hi_b = (uint32_t)(pb >> 32);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(const Key& k, uint32_t index, uint32_t tag, uint32_t aux)
{
    return philox10(index, (tag << 24) | (aux & 0xFFFFFFu), k.cell, k.step, k.seed, k.uid);
}

// 53-bit uniform in [0,1): the high word supplies the top 21 bits.
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
    const uint64_t b = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return (double)b * 0x1.0p-53;
}
// 24-bit uniform in [0,1): equals the top 24 bits of u53(w, .).
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1.0p-24f; }

// Sub-level choice j in {0..l-1} of collision c of level l (uniform, Alg. 4.1/4.3).
__device__ __forceinline__ uint32_t tree_choice(const Key& k, uint32_t l, uint32_t c)
{
    const uint4 w = draw(k, c >> 2, TAG_TREE, l);
    const uint32_t s = (c & 3u) == 0 ? w.x : (c & 3u) == 1 ? w.y : (c & 3u) == 2 ? w.z : w.w;
    return __umulhi(s, l);
}

// ---------------------------------------------------------------------------
// exp(-x) for x >= 0 by a fixed written algorithm (Cody-Waite reduction with a
// two-part ln 2, degree-13 Taylor polynomial by Horner, scaling by 2^k), with
// contraction off, so that q = exp(-mu dt/eps) has reproducible bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_neg(double x)
{
#pragma clang fp contract(off)
    const double head = 0x1.62e42p-1;
    const double tail = 0x1.fdf473de6af28p-22;
    const double inv_ln2 = 0x1.71547652b82fep+0;
    if (!(x >= 0.0)) return x != x ? x : 1.0;
    if (x > 746.0) return 0.0;
    const double y = -x;
    const double k = floor(y * inv_ln2 + 0.5);
    const double r = (y - k * head) - k * tail;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

// Item b and local index k of flat block t, given the exclusive prefix of the
// items' block counts (prefix[b] <= t < prefix[b + 1]; nb items).
__device__ __forceinline__ void tile_of(const uint32_t* prefix, uint32_t nb, uint32_t t, uint32_t& b, uint32_t& k)
{
    uint32_t lo = 0, hi = nb;  // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid;
        else hi = mid;
    }
    b = lo;
    k = t - prefix[lo];
}

// Round a positive double up to 20 significant bits (grid of the VHS majorant).
__device__ __forceinline__ double grid_up20(double g)
{
    uint64_t b = (uint64_t)__double_as_longlong(g);
    const uint64_t low = (1ull << 33) - 1ull;
    if (b & low) b = (b | low) + 1ull;
    return __longlong_as_double((long long)b);
}

// Iround of Alg. 4.2 (floor(y) + 1 with probability frac(y)), contraction off.
__device__ __forceinline__ uint32_t iround_prod(double q, uint32_t rem, double u)
{
#pragma clang fp contract(off)
    const double y = q * (double)rem;
    const double f = floor(y);
    const uint32_t k = (uint32_t)f + (u < y - f ? 1u : 0u);
    return k < rem ? k : rem;  // q <= 1 keeps k <= rem; the bound only guards bad input
}

// ---------------------------------------------------------------------------
// Keyed permutation of roles: a 6-round alternating Feistel network on b bits,
// b = max(8, ceil(log2 n)), cycle walking into [0, n).  A value is a high part
// of ceil(b/2) bits and a low part of floor(b/2) bits; even rounds xor F(low)
// into the high part, odd rounds F(high) into the low part.  Round i keys with
// k[i & 3] ^ (i * 0x9E3779B9); F(x) = mix24(x ^ key), a multiply-xorshift
// finalizer built from 24-bit products (full-rate v_mul_u32_u24).
// perm_inverse(s) returns the role index of slot s.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t mix24(uint32_t x)
{
    uint32_t h = __umul24(x, 0xEBCA6Bu);
    h ^= h >> 15;
    h = __umul24(h, 0xB2AE35u);
    h ^= h >> 13;
    return h;
}

__device__ __forceinline__ uint32_t perm_bits(uint32_t n)
{
    const uint32_t b = (n <= 1u) ? 0u : 32u - __clz(n - 1u);  // ceil(log2 n)
    return b < 8u ? 8u : b;
}

__device__ __forceinline__ uint32_t feistel_dec(uint32_t y, uint32_t b, uint4 k)
{
    const uint32_t lo = b >> 1, hi = b - lo;
    const uint32_t mlo = (1u << lo) - 1u, mhi = (hi >= 32u) ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    uint32_t H = y >> lo, W = y & mlo;
    const uint32_t kk[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        const uint32_t rk = kk[i & 3] ^ ((uint32_t)i * 0x9E3779B9u);
        if ((i & 1) == 0) H ^= mix24(W ^ rk) & mhi;
        else W ^= mix24(H ^ rk) & mlo;
    }
    return (H << lo) | W;
}

__device__ __forceinline__ uint32_t perm_inverse(uint32_t s, uint32_t n, uint32_t b, uint4 k)
{
    uint32_t y = feistel_dec(s, b, k);
    while (y >= n) y = feistel_dec(y, b, k);
    return y;
}

// Role index of every slot in [r0, r1) of a cell, written to role[], by one
// wave whose lanes take the next slot as soon as their cycle walk ends: a wave
// evaluates about (sum of the walks) / 64 rounds of the network instead of the
// longest walk of its 64 slots per batch of 64.  R: the role's element type
// (16 bits for cells of at most 65536 particles).
template <typename R = uint32_t>
__device__ __forceinline__ void roles_by_wave(__attribute__((address_space(1))) R* role, uint32_t r0,
                                              uint32_t r1, uint32_t n, uint32_t b, uint4 k)
{
    const uint32_t lane = __lane_id();
    uint32_t cur = 0xFFFFFFFFu, val = 0, base = r0;
    for (;;) {
        // lanes without a slot take the next ones in order
        const bool need = cur == 0xFFFFFFFFu;
        const unsigned long long m = __ballot(need);
        const uint32_t cand = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        base += (uint32_t)__popcll(m);
        if (need && cand < r1) {
            cur = cand;
            val = cand;
        }
        if (__ballot(cur != 0xFFFFFFFFu) == 0ull) break;
        if (cur != 0xFFFFFFFFu) {
            val = feistel_dec(val, b, k);
            if (val < n) {
                role[cur] = (R)val;
                cur = 0xFFFFFFFFu;
            }
        }
    }
}

// The rounds in forward order: perm_forward(i) is the slot of role index i
// (perm_inverse(perm_forward(i)) == i; cycle walking keeps the pair inverse).
__device__ __forceinline__ uint32_t feistel_enc(uint32_t y, uint32_t b, uint4 k)
{
    const uint32_t lo = b >> 1, hi = b - lo;
    const uint32_t mlo = (1u << lo) - 1u, mhi = (hi >= 32u) ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    uint32_t H = y >> lo, W = y & mlo;
    const uint32_t kk[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (int i = 0; i <= 5; ++i) {
        const uint32_t rk = kk[i & 3] ^ ((uint32_t)i * 0x9E3779B9u);
        if ((i & 1) == 0) H ^= mix24(W ^ rk) & mhi;
        else W ^= mix24(H ^ rk) & mlo;
    }
    return (H << lo) | W;
}

__device__ __forceinline__ uint32_t perm_forward(uint32_t i, uint32_t n, uint32_t b, uint4 k)
{
    uint32_t y = feistel_enc(i, b, k);
    while (y >= n) y = feistel_enc(y, b, k);
    return y;
}

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed butterfly inside a wave, then waves in
// order).  `red` holds kCollideThreads/64 * K doubles of LDS.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = v[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
        v[k] = a;
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a += red[w * K + k];
        v[k] = a;
    }
}

}  // namespace trmc
