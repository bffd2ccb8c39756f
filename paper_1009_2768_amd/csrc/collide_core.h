// collide_core.h -- building blocks of the per-cell TRMC-R collision step
// shared by the whole-cell kernel (small cells, slab cells) and the tiled
// pipeline (large homogeneous cells).  A "group" of G threads (one wave, or a
// whole workgroup) owns one cell in the per-cell phases.
#pragma once
#include <hip/hip_runtime.h>

#include "trmc_device.h"
#include "trmc_internal.h"

namespace trmc {

template <typename T>
struct Vec3 {
    T x, y, z;
};

// ---------------------------------------------------------------------------
// Group primitives: a group of G threads works on one cell.  G = 64 is one wave
// (wave-synchronous: LDS traffic ordered by fences, no workgroup barrier);
// G = workgroup size uses workgroup barriers.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void gsync()
{
    if constexpr (G == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Synchronisation of the group for LDS traffic only (global stores stay in
// flight; they are ordered by a later gsync).
template <int G>
__device__ __forceinline__ void gsync_lds()
{
    if constexpr (G == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// Sum over the group; every thread receives the total.  Fixed order: butterfly
// inside each wave, then the waves in order.  `red` holds (G/64 + 1) * K
// doubles.  Thread k sums component k over the waves and every thread reads
// the K totals: each thread holds K doubles, not K per wave.
template <int G, int K>
__device__ __forceinline__ void gsum(double (&v)[K], double* red)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = v[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
        v[k] = a;
    }
    if constexpr (G > 64) {
        constexpr int NW = G / 64;
        const int tid = threadIdx.x % G, lane = tid & 63, wave = tid >> 6;
        gsync_lds<G>();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
        }
        gsync_lds<G>();
        if (tid < K) {
            double a = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) a += red[w * K + tid];
            red[NW * K + tid] = a;
        }
        gsync_lds<G>();
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = red[NW * K + k];
    }
}

template <int G>
__device__ __forceinline__ double gmax(double v, double* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if constexpr (G > 64) {
        const int lane = threadIdx.x & 63, wave = (threadIdx.x % G) >> 6;
        gsync_lds<G>();
        if (lane == 0) red[wave] = v;
        gsync_lds<G>();
        double a = red[0];
        for (int w = 1; w < G / 64; ++w) a = fmax(a, red[w]);
        v = a;
    }
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t gsum_u32(uint32_t v, uint32_t* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if constexpr (G > 64) {
        const int lane = threadIdx.x & 63, wave = (threadIdx.x % G) >> 6;
        gsync_lds<G>();
        if (lane == 0) red[wave] = v;
        gsync_lds<G>();
        uint32_t a = 0;
        for (int w = 0; w < G / 64; ++w) a += red[w];
        v = a;
    }
    return v;
}

__device__ __forceinline__ unsigned long long shfl64(unsigned long long v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Arithmetic of one collision and of the Maxwellian samples.
// FP64: library sqrt/sin/cos/log.  FP32: hardware transcendentals, with the
// angle in revolutions (sin(2 pi u) directly), log2 and sqrt.
// ---------------------------------------------------------------------------
// Collision draws: FP64 takes the high bits from block 0 and the low bits from
// block 1; FP32 takes block 0 only (its uniforms are the top 24 bits of FP64's).
template <typename T>
struct Draws;

template <>
struct Draws<double> {
    static __device__ __forceinline__ void coll(const Key& k, uint32_t l, uint32_t c, double& xi1, double& xi2,
                                                double& xacc)
    {
        const uint4 b0 = draw(k, c, TAG_COLL, l);
        const uint4 b1 = draw(k, c, TAG_COLL, l | (1u << 20));
        xi1 = u53(b0.x, b1.x);
        xi2 = u53(b0.y, b1.y);
        xacc = u53(b0.z, b1.z);
    }
    static __device__ __forceinline__ void sincos2pi(double u, double& s, double& c)
    {
        const double a = 6.283185307179586 * u;
        s = sin(a);
        c = cos(a);
    }
    static __device__ __forceinline__ double sqrt_(double a) { return sqrt(a); }
    static __device__ __forceinline__ double pow_(double a, double b) { return pow(a, b); }
    static __device__ __forceinline__ Vec3<double> normals(const Key& k, uint32_t t)
    {
        const uint4 b0 = draw(k, t, TAG_MAXW, 0);
        const uint4 b1 = draw(k, t, TAG_MAXW, 1);
        const double u0 = u53(b0.x, b1.x), u1 = u53(b0.y, b1.y), u2 = u53(b0.z, b1.z), u3 = u53(b0.w, b1.w);
        const double r1 = sqrt(-2.0 * log(1.0 - u0));
        const double r2 = sqrt(-2.0 * log(1.0 - u2));
        double s1, c1, s2, c2;
        sincos2pi(u1, s1, c1);
        sincos2pi(u3, s2, c2);
        return Vec3<double>{r1 * c1, r1 * s1, r2 * c2};
    }
};

template <>
struct Draws<float> {
    static __device__ __forceinline__ void coll(const Key& k, uint32_t l, uint32_t c, float& xi1, float& xi2,
                                                float& xacc)
    {
        const uint4 b0 = draw(k, c, TAG_COLL, l);
        xi1 = u24(b0.x);
        xi2 = u24(b0.y);
        xacc = u24(b0.z);
    }
    static __device__ __forceinline__ void sincos2pi(float u, float& s, float& c)
    {
        s = __builtin_amdgcn_sinf(u);  // sin(2 pi u)
        c = __builtin_amdgcn_cosf(u);
    }
    static __device__ __forceinline__ float sqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }
    static __device__ __forceinline__ float pow_(float a, float b)
    {
        return a > 0.0f ? __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(a)) : 0.0f;
    }
    static __device__ __forceinline__ Vec3<float> normals(const Key& k, uint32_t t)
    {
        const uint4 b0 = draw(k, t, TAG_MAXW, 0);
        // -2 ln(1-u) = -2 ln2 log2(1-u); 1 - u >= 2^-24
        const float r1 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(1.0f - u24(b0.x)));
        const float r2 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(1.0f - u24(b0.z)));
        float s1, c1, s2, c2;
        sincos2pi(u24(b0.y), s1, c1);
        sincos2pi(u24(b0.w), s2, c2);
        return Vec3<float>{r1 * c1, r1 * s1, r2 * c2};
    }
};

// One collision of eq. (Maxwell_coll-r); dummy (outputs = inputs) unless
// xi_acc * g < |q|^alpha.  Returns 1 if real.
template <typename T>
__device__ __forceinline__ int collide(const Vec3<T>& a, const Vec3<T>& b, T xi1, T xi2, T xacc, T alpha, T g,
                                       Vec3<T>& oa, Vec3<T>& ob, uint32_t& viol)
{
    const T qx = a.x - b.x, qy = a.y - b.y, qz = a.z - b.z;
    const T qn = Draws<T>::sqrt_(qx * qx + qy * qy + qz * qz);
    if (alpha != T(0)) {
        const T s = (alpha == T(1)) ? qn : Draws<T>::pow_(qn, alpha);
        viol += (s > g) ? 1u : 0u;
        if (!(xacc * g < s)) {
            oa = a;
            ob = b;
            return 0;
        }
    }
    const T ct = T(2) * xi1 - T(1);
    const T st2 = T(1) - ct * ct;
    const T st = Draws<T>::sqrt_(st2 > T(0) ? st2 : T(0));
    T sp, cp;
    Draws<T>::sincos2pi(xi2, sp, cp);
    const T h = T(0.5) * qn;
    const T sx = cp * st, sy = sp * st, sz = ct;
    const T cx = T(0.5) * (a.x + b.x), cy = T(0.5) * (a.y + b.y), cz = T(0.5) * (a.z + b.z);
    oa.x = cx + h * sx;
    oa.y = cy + h * sy;
    oa.z = cz + h * sz;
    ob.x = cx - h * sx;
    ob.y = cy - h * sy;
    ob.z = cz - h * sz;
    return 1;
}

// Scalars shared by a group.
struct CellShared {
    double mean[3];
    double Sn, q, g, ur[3], a_th, zbar[3], E1, kept0;
    double d2max0;  // largest |v - mean|^2 of the pre-step velocities (VHS; else 0)
    double g_last;  // majorant of the accepted attempt's last level
    double rs[4];  // tree-shape truncation: split remainder's sums of v - mean (3) and |v - mean|^2
    double wbz[9]; // tree-shape truncation: the dropped finals' sums (WbAcc, group totals)
    uint32_t me, split_rem, R0, N0, borrowed, n_th, folds, m, attempts, decision, overflow, wb_th;
    uint32_t ext_empty;  // the split continued past depth m would leave every level up to m_cap empty
    unsigned long long ncoll, work;
    uint32_t dummies, viol;
    double all_th[4];  // the whole cell about its mean: sum of v - m (3), of |v - m|^2 (moments pass)
    double zt[4];      // a cell predicted wholly thermalized: its normals' sums (moments pass)
};

// Level arrays of a group, lv_stride = m_cap + 2 entries each (dynamic LDS).
struct Levels {
    uint32_t *N, *Rtot, *C, *outoff, *run;
};

// LDS of one group (besides its level arrays).
template <int G>
struct GroupLds {
    CellShared sh;
    double red[(G / 64) * 12];
    uint32_t redu[(G / 64) * 2];
    uint32_t wcnt[G / 64][64];
    uint32_t wpre[G / 64][64];
    uint16_t jbuf[G];
};


// Pointers into one cell's scratch region (layout in trmc_internal.h).
// A velocity in scratch memory: one aligned 4-component record.
template <typename T>
struct alignas(16) Pack4 {
    T x, y, z, w;
};

template <typename T>
__device__ __forceinline__ Vec3<T> unpack(const Pack4<T>& p)
{
    return Vec3<T>{p.x, p.y, p.z};
}

template <typename T>
__device__ __forceinline__ Pack4<T> pack(T x, T y, T z)
{
    return Pack4<T>{x, y, z, T(0)};
}

// Record load and store through a global pointer (one 16-byte access in FP32).
template <typename T>
__device__ __forceinline__ Vec3<T> ld3(gptr<const Pack4<T>> p)
{
    return Vec3<T>{p->x, p->y, p->z};
}
template <typename T>
__device__ __forceinline__ Vec3<T> ld3(gptr<Pack4<T>> p)
{
    return ld3((gptr<const Pack4<T>>)p);
}
template <typename T>
__device__ __forceinline__ Pack4<T> ld4(gptr<const Pack4<T>> p)
{
    return Pack4<T>{p->x, p->y, p->z, p->w};
}
template <typename T>
__device__ __forceinline__ Pack4<T> ld4(gptr<Pack4<T>> p)
{
    return ld4((gptr<const Pack4<T>>)p);
}
template <typename T>
__device__ __forceinline__ void st4(gptr<Pack4<T>> p, T x, T y, T z, T w)
{
    p->x = x;
    p->y = y;
    p->z = z;
    p->w = w;
}
template <typename T>
__device__ __forceinline__ void st3(gptr<Pack4<T>> p, T x, T y, T z)
{
    p->x = x;
    p->y = y;
    p->z = z;
    p->w = T(0);
}

template <typename T, typename R = uint32_t>
struct CellMem {
    gptr<R> role;         // [n] role index of each slot (inverse of the keyed permutation)
    gptr<uint32_t> fwd;   // [n] slot of each role index (the permutation itself; tile path)
    gptr<Pack4<T>> leaf;  // [n] leaves by leaf rank (whole-cell path)
    gptr<Pack4<T>> fin;   // [n] finals by leaf rank (final r goes to the slot of leaf r)
    gptr<uint32_t> jarr;  // [cap] sub-level choice of each collision
    gptr<uint32_t> rA;    // [cap] rank of request A at level j
    gptr<uint32_t> rB;    // [cap] rank of request B at level l-1-j
    gptr<Pack4<T>> outv;  // [2 cap] outputs taken by requests
    uint64_t cap, ocap;
    __device__ __forceinline__ void init(const InstDev* I, uint32_t off, uint32_t cell, uint32_t n)
    {
        cap = coll_cap(n);
        ocap = 2ull * cap;
        // the cell is the same on every lane of the wave: scalar base pointers
        unsigned char* base = uni(I->scratch + I->scratch_bpp * (uint64_t)off + I->scratch_cpc * (uint64_t)cell);
        role = as_global(reinterpret_cast<R*>(base));
        base += align16(4ull * n);  // room for 32-bit roles either way
        fwd = as_global(reinterpret_cast<uint32_t*>(base));
        base += align16(4ull * n);
        leaf = as_global(reinterpret_cast<Pack4<T>*>(base));
        base += sizeof(Pack4<T>) * (uint64_t)n;
        fin = as_global(reinterpret_cast<Pack4<T>*>(base));
        base += sizeof(Pack4<T>) * (uint64_t)n;
        jarr = as_global(reinterpret_cast<uint32_t*>(base));
        base += align16(4ull * cap);
        rA = as_global(reinterpret_cast<uint32_t*>(base));
        base += align16(4ull * cap);
        rB = as_global(reinterpret_cast<uint32_t*>(base));
        base += align16(4ull * cap);
        outv = as_global(reinterpret_cast<Pack4<T>*>(base));
    }
};

__device__ __forceinline__ Levels levels_at(uint32_t* p, uint32_t stride)
{
    Levels L;
    L.N = p;
    L.Rtot = L.N + stride;
    L.C = L.Rtot + stride;
    L.outoff = L.C + stride;
    L.run = L.outoff + stride;
    return L;
}

// VHS majorant sigma(2 dv) = (2 dv)^alpha rounded up to the 20-bit grid, from the
// largest squared distance d2 = dv^2 to the cell mean (Sec. 4.2).
__device__ __forceinline__ double majorant_of(double alpha, double d2)
{
#pragma clang fp contract(off)
    const double two_dv = 2.0 * sqrt(d2);
    return grid_up20(alpha == 1.0 ? two_dv : pow(two_dv, alpha));
}

// The VHS majorant without a pass over the velocities for their largest
// distance to the mean, when a bracket settles it.  With d2c the largest squared
// distance of the velocities to a point c and delta = |mean - c|, the largest
// distance dv to the mean lies in [sqrt(d2c) - delta, sqrt(d2c) + delta]
// (triangle inequality).  Both ends are widened by far more than the rounding
// of either computation (and, for alpha < 1, of pow); if the widened ends give
// the same majorant on the 20-bit grid, majorant_of is monotone in between, so
// that is also the majorant of the exact largest distance.  Returns a d2 whose
// majorant_of is that value (the upper end), or -1 when the bracket does not
// settle it (the caller makes the exact pass).  0 < alpha <= 1.
__device__ __forceinline__ double majorant_bracket(double alpha, double d2c, double delta)
{
#pragma clang fp contract(off)
    if (!(d2c >= 0.0 && d2c <= 1e300 && delta >= 0.0 && delta <= 1e300)) return -1.0;
    const double r = sqrt(d2c);
    const double lo_r = r * (1.0 - 1e-12) - delta * (1.0 + 1e-12);
    if (!(lo_r > 0.0)) return -1.0;
    const double hi_r = r * (1.0 + 1e-12) + delta * (1.0 + 1e-12);
    const double lo = lo_r * lo_r * (1.0 - 1e-12), hi = hi_r * hi_r * (1.0 + 1e-12);
    double glo, ghi;
    if (alpha == 1.0) {
        glo = grid_up20(2.0 * sqrt(lo));
        ghi = grid_up20(2.0 * sqrt(hi));
    } else {
        glo = grid_up20(pow(2.0 * sqrt(lo), alpha) * (1.0 - 1e-14));
        ghi = grid_up20(pow(2.0 * sqrt(hi), alpha) * (1.0 + 1e-14));
    }
    return glo == ghi ? hi : -1.0;
}

// Majorant, relaxation parameter and depth of the step from the cell's moments
// (thread 0 of the group): g = (2 dv)^alpha on the 20-bit grid, mu = rho g,
// q = exp(-mu dt / eps) (Sec. 3.2, Sec. 4.2); m from the truncation mode.
__device__ __forceinline__ void cell_params(const InstDev* I, uint32_t cell, uint32_t n, double dmax,
                                            CellShared& sh)
{
    double g = 1.0;
    if (I->alpha != 0.0) g = majorant_of(I->alpha, dmax);
    sh.d2max0 = dmax;
    sh.g_last = g;
    const double eps = I->eps_cells[cell];
    double xarg;
    {
#pragma clang fp contract(off)
        const double rho = (double)n * I->rho_factor;
        const double mu = rho * g;
        xarg = mu * I->dt / eps;
    }
    sh.g = g;
    double q = exp_neg(xarg);
    if (!(q >= 0.0 && q <= 1.0)) q = 1.0;  // non-finite velocities: leave the cell unchanged
    sh.q = q;
    uint32_t m;
    if (I->trunc == TRUNC_FIXED) m = I->m_init;
    else if (I->trunc == TRUNC_ADAPTIVE || I->trunc == TRUNC_ADAPTIVE_REUSE) m = I->m_state[cell];
    else m = I->m_cap;
    if (m < 1) m = 1;
    if (m > I->m_cap) m = I->m_cap;
    sh.m = m;
    sh.attempts = 0;
    sh.work = 0;
    sh.overflow = 0;
    sh.wb_th = 0;
}

// Depth up to which a split looks ahead for the adaptive decision (0: none).
__device__ __forceinline__ uint32_t adaptive_look(const InstDev* I)
{
    const uint32_t t = uni(I->trunc);
    return (t == TRUNC_ADAPTIVE || t == TRUNC_ADAPTIVE_REUSE) ? uni(I->m_cap) : 0u;
}

// a. Split into collision sets (Alg. 4.2) at depth sh.m: wave 0 of the group
//    draws 64 levels at a time; every lane runs the (uniform) Iround chain.
//    With look = m_cap (adaptive depth) it also records whether the split,
//    continued from the remainder, would leave levels m+1..m_cap all empty: a
//    deeper attempt would then build the same trees, and is not made.
template <int G>
__device__ __forceinline__ void split_levels(const Key& key, uint32_t n, double q, const Levels& L, CellShared& sh,
                                             uint32_t tid, uint32_t look = 0)
{
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    if (wave == 0) {
        const uint32_t m = sh.m;
        uint32_t cbase = 0;
        uint4 w = draw(key, lane, TAG_SPLIT, 0);
        double u = u53(w.x, w.y);
        const uint32_t N0 = iround_prod(q, n, __shfl(u, 0));
        uint32_t rem = n - N0, k = 0;
        if (lane == 0) L.N[0] = N0;
        while (rem > 0 && k < m) {
            ++k;
            if (k - cbase >= 64u) {
                cbase += 64u;
                w = draw(key, cbase + lane, TAG_SPLIT, 0);
                u = u53(w.x, w.y);
            }
            const uint32_t Nk = iround_prod(q, rem, __shfl(u, (int)(k - cbase)));
            if (lane == 0) L.N[k] = Nk;
            rem -= Nk;
        }
        uint32_t ext_empty = 1;
        if (look > m && rem > 0) {
            double y;
            {
#pragma clang fp contract(off)
                y = q * (double)rem;  // Iround's argument at every deeper level while they stay empty
            }
            if (y >= 1.0) {
                ext_empty = 0;
            } else {
                // level k gets a particle iff its uniform is below y (floor(y) = 0)
                for (uint32_t kb = m + 1u; kb <= look && ext_empty; kb += 64u) {
                    const uint32_t kk = kb + lane;
                    bool hit = false;
                    if (kk <= look) {
                        const uint4 ww = draw(key, kk, TAG_SPLIT, 0);
                        hit = u53(ww.x, ww.y) < y;
                    }
                    if (__ballot(hit) != 0ull) ext_empty = 0;
                }
            }
        }
        if (lane == 0) {
            L.N[k + 1] = rem;
            sh.me = k;
            sh.split_rem = rem;
            sh.N0 = N0;
            sh.folds = 0;
            sh.attempts += 1;
            sh.ext_empty = ext_empty;
        }
    }
    gsync_lds<G>();
}

// b. Collision trees, deepest level first (Alg. 4.3 in level order).  Level l
//    with R_l requests runs ceil(R_l/2) + ceil(max(0, N_l - (R_l mod 2))/2)
//    collisions; collision c chooses j uniform in {0..l-1} and asks level j (A)
//    then level l-1-j (B); requests take stable ranks (collision order, A before
//    B), request r of level t receiving output r of level t.  While the leaves
//    R_0 exceed n, the deepest level is folded into the remainder.  Returns the
//    number of collisions (uniform over the group); sets sh.R0, sh.me, sh.folds
//    and sh.overflow (capacity).
//    REUSE (adaptive depth keeping a rejected attempt, Sec. 4.3): the trees are
//    built on top of earlier attempts' -- collision c of level l draws with index
//    coff[l] + c, the leaves fit when r0prev + R0 <= n, and only levels above
//    mfloor are folded.
template <int G, bool REUSE = false>
__device__ __forceinline__ unsigned long long build_trees(const Key& key, uint32_t n, uint64_t cap,
                                                          const Levels& L, GroupLds<G>& gl, CellShared& sh,
                                                          gptr<uint32_t> jarr, gptr<uint32_t> rA, gptr<uint32_t> rB,
                                                          uint32_t tid, const uint32_t* coff = nullptr,
                                                          uint32_t r0prev = 0, uint32_t mfloor = 0)
{
    constexpr int NWG = G / 64;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64u - lane));
    unsigned long long ncoll = 0;
    // Depth of the trees: the split's depth when its trees fit in the cell;
    // otherwise the largest depth whose trees fit, found by bisection.  The
    // leaves a depth needs never decrease with the depth (the levels below it
    // and their keyed choices are the same, and every level's collision count
    // grows with the requests it receives), so this is the depth at which the
    // fold rule's level-by-level descent stops, in O(log depth) builds.
    const uint32_t me_split = uni(sh.me);
    uint32_t lo = REUSE ? (mfloor < me_split ? mfloor : me_split) : 0u;  // a depth that fits
    uint32_t hi = me_split;  // a depth that does not fit, once the first build has failed
    uint32_t me = me_split;  // depth of the current build
    for (;;) {
        for (uint32_t l = tid; l <= me; l += G) L.run[l] = 0;
        gsync_lds<G>();
        ncoll = 0;
        bool ovf = false;
        for (uint32_t l = me; l >= 1; --l) {
            const uint32_t Rl = uni(L.run[l]);
            const uint32_t odd = Rl & 1u, Nl = uni(L.N[l]);
            const uint32_t own = Nl > odd ? (Nl - odd + 1u) / 2u : 0u;
            const uint32_t Cl = (Rl + 1u) / 2u + own;
            if (tid == 0) {
                L.C[l] = Cl;
                L.Rtot[l] = Rl;
            }
            if (Cl == 0) continue;
            if (ncoll + Cl > cap) {
                ovf = true;
                break;
            }
            const uint32_t fst = (uint32_t)ncoll;
            [[maybe_unused]] const uint32_t c_off = REUSE ? uni(coff[l]) : 0u;
            if (l <= 64u) {
                for (uint32_t b0 = 0; b0 < Cl; b0 += G) {
                    // sub-level choices: one Philox block per 4 collisions
                    if constexpr (REUSE) {
                        // the index offset need not be a multiple of 4: every lane
                        // draws its own collision's block
                        if (b0 + tid < Cl) gl.jbuf[tid] = (uint16_t)tree_choice(key, l, c_off + b0 + tid);
                    } else if (tid < G / 4u && b0 + 4u * tid < Cl) {
                        const uint4 wv = draw(key, (b0 >> 2) + tid, TAG_TREE, l);
                        gl.jbuf[4 * tid + 0] = (uint16_t)__umulhi(wv.x, l);
                        gl.jbuf[4 * tid + 1] = (uint16_t)__umulhi(wv.y, l);
                        gl.jbuf[4 * tid + 2] = (uint16_t)__umulhi(wv.z, l);
                        gl.jbuf[4 * tid + 3] = (uint16_t)__umulhi(wv.w, l);
                    }
                    gsync_lds<G>();
                    const uint32_t c = b0 + tid;
                    const bool valid = c < Cl;
                    const uint32_t j = valid ? (uint32_t)gl.jbuf[tid] : 0u;
                    const uint32_t h = l - 1u - j;
                    unsigned long long myM = 0ull;  // lane b: lanes of this wave whose A goes to level b
                    const uint32_t nvalid = (Cl - b0 < G ? Cl - b0 : (uint32_t)G);
                    if (nvalid >= 8u * l || l <= 8u) {
                        for (uint32_t b = 0; b < l; ++b) {
                            const unsigned long long M = __ballot(valid && j == b);
                            myM = (lane == b) ? M : myM;
                        }
                    } else {
                        // few collisions: iterate over the distinct levels present
                        bool pend = valid;
                        for (;;) {
                            const unsigned long long pm = __ballot(pend);
                            if (pm == 0ull) break;
                            const uint32_t t = (uint32_t)__shfl((int)j, __ffsll((long long)pm) - 1);
                            const unsigned long long M = __ballot(valid && j == t);
                            myM = (lane == t) ? M : myM;
                            pend = pend && j != t;
                        }
                    }
                    const unsigned long long Mj = shfl64(myM, (int)j), Mh = shfl64(myM, (int)h);
                    const unsigned long long Mrev = shfl64(myM, (int)(lane < l ? l - 1u - lane : 0u));
                    const uint32_t local = (uint32_t)(__popcll(Mj & lt) + __popcll(Mh & lt));
                    if (lane < l) gl.wcnt[wave][lane] = (uint32_t)(__popcll(myM) + __popcll(Mrev));
                    gsync_lds<G>();
                    if (tid < l) {
                        uint32_t acc = L.run[tid];
#pragma unroll
                        for (int w = 0; w < NWG; ++w) {
                            gl.wpre[w][tid] = acc;
                            acc += gl.wcnt[w][tid];
                        }
                        L.run[tid] = acc;
                    }
                    gsync_lds<G>();
                    if (valid) {
                        jarr[fst + c] = j;
                        rA[fst + c] = gl.wpre[wave][j] + local;
                        rB[fst + c] = gl.wpre[wave][h] + local + (j == h ? 1u : 0u);
                    }
                    gsync_lds<G>();
                }
            } else {
                // deep levels (natural depth): one wave, distinct target levels by ballot
                if (wave == 0) {
                    for (uint32_t b0 = 0; b0 < Cl; b0 += 64u) {
                        const uint32_t c = b0 + lane;
                        const bool valid = c < Cl;
                        const uint32_t j = valid ? tree_choice(key, l, (REUSE ? c_off : 0u) + c) : 0u;
                        const uint32_t ta = j, tb = l - 1u - j;
                        bool pa = valid, pb = valid;
                        uint32_t rkA = 0, rkB = 0;
                        for (;;) {
                            const unsigned long long mA = __ballot(pa), mB = __ballot(pb);
                            if (mA == 0ull && mB == 0ull) break;
                            const uint32_t t = mA ? (uint32_t)__shfl((int)ta, __ffsll((long long)mA) - 1)
                                                  : (uint32_t)__shfl((int)tb, __ffsll((long long)mB) - 1);
                            const bool hitA = pa && ta == t, hitB = pb && tb == t;
                            const unsigned long long eA = __ballot(hitA), eB = __ballot(hitB);
                            const uint32_t bcnt = __builtin_amdgcn_readfirstlane(L.run[t]);
                            const uint32_t before = (uint32_t)(__popcll(eA & lt) + __popcll(eB & lt));
                            if (hitA) {
                                rkA = bcnt + before;
                                pa = false;
                            }
                            if (hitB) {
                                rkB = bcnt + before + (ta == t ? 1u : 0u);
                                pb = false;
                            }
                            __builtin_amdgcn_wave_barrier();
                            if (lane == 0) L.run[t] = bcnt + (uint32_t)(__popcll(eA) + __popcll(eB));
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        }
                        if (valid) {
                            jarr[fst + c] = j;
                            rA[fst + c] = rkA;
                            rB[fst + c] = rkB;
                        }
                    }
                }
                gsync_lds<G>();
            }
            ncoll += Cl;
        }
        if (ovf) {
            if (tid == 0) sh.overflow = 1u;
            gsync_lds<G>();
            return ncoll;
        }
        if (tid == 0) sh.R0 = L.run[0];
        gsync_lds<G>();
        const bool fits = REUSE ? (r0prev + uni(sh.R0) <= n || me <= mfloor) : uni(sh.R0) <= n;
        if (fits) lo = me;
        else hi = me;
        if (fits && (me == me_split || hi - lo <= 1u)) break;  // the schedule of depth lo is built
        me = hi - lo <= 1u ? lo : lo + (hi - lo) / 2u;       // bisect, or rebuild the final depth
    }
    if (me < me_split) {
        // the levels above me are folded into the remainder
        if (tid == 0) {
            uint32_t rem = 0;
            for (uint32_t l = me + 1u; l <= me_split + 1u; ++l) rem += L.N[l];
            L.N[me + 1u] = rem;
            sh.me = me;
            sh.folds += me_split - me;
        }
        gsync_lds<G>();
    }
    return ncoll;
}

// Offsets of the outputs taken by requests, role thresholds, capacity
// (thread 0; the group synchronises).  Returns false on overflow.
template <int G>
__device__ __forceinline__ bool level_offsets(uint32_t n, unsigned long long ncoll, uint64_t ocap,
                                              const Levels& L, CellShared& sh, uint32_t tid)
{
    if (tid == 0) {
        const uint32_t me = sh.me, R0 = sh.R0;
        unsigned long long no = 0;
        for (uint32_t l = 1; l <= me; ++l) {
            L.outoff[l] = (uint32_t)no;
            no += L.Rtot[l];
        }
        sh.ncoll = ncoll;
        sh.work += ncoll;
        if (no > ocap) sh.overflow = 1u;
        const uint32_t N0 = sh.N0, P = n - N0;
        sh.borrowed = R0 > P ? R0 - P : 0u;
        sh.n_th = R0 < P ? P - R0 : 0u;
    }
    gsync<G>();
    return sh.overflow == 0u;
}

// Leaf rank of role index i in the leaf range [kept_end, leaf_end): roles N0,
// N0 + 1, ... are leaves 0, 1, ...; borrowed roles N0 - 1, N0 - 2, ... follow
// as leaves P, P + 1, ... (P = n - N0).
__device__ __forceinline__ uint32_t leaf_rank(uint32_t i, uint32_t N0, uint32_t P)
{
    return i >= N0 ? i - N0 : P + (N0 - 1u - i);
}

// Role index of leaf r (inverse of leaf_rank).
__device__ __forceinline__ uint32_t leaf_role(uint32_t r, uint32_t N0, uint32_t P)
{
    return r < P ? N0 + r : N0 - 1u - (r - P);
}

// Leaves and sums of the unchanged and thermalized sets over slots [s_begin,
// s_end) of a cell with NT threads (this thread's share): leaf r is copied to
// leaf[r] unless r < r_done (already there from an earlier attempt: the leaf of
// a rank does not depend on the depth); with pool_all (no borrowed leaves) the
// thermalized roles i are copied too, as rank i - N0, so that later attempts
// find their whole pool in rank order.  sums = {kept (vx-m)^2, thermalized
// (vx-m)^2, thermalized v-m (3), thermalized |v-m|^2}.  Roles below kept_end
// are unchanged, roles from leaf_end on are thermalized, the others are leaves.
// ALL_TH: an attempt with no unchanged slots and no leaves (kept_end = leaf_end
// = 0), whose roles are not read: every slot is thermalized.
template <typename T, int NT, bool ALL_TH = false, typename R = uint32_t>
__device__ __forceinline__ void gather_sets(gptr<const T> vx, gptr<const T> vy, gptr<const T> vz,
                                            gptr<const R> role, gptr<Pack4<T>> leaf,
                                            uint32_t n, uint32_t N0, uint32_t s_begin, uint32_t s_end,
                                            uint32_t kept_end, uint32_t leaf_end, uint32_t r_done, bool pool_all,
                                            double mx, double my, double mz, uint32_t tid, double (&sums)[6])
{
#ifndef TRMC_GATHER_UNROLL
#define TRMC_GATHER_UNROLL 4
#endif
    constexpr int U = TRMC_GATHER_UNROLL;  // slots per thread per batch
    const uint32_t P = n - N0;
    for (uint32_t s0 = s_begin + tid; s0 < s_end; s0 += NT * U) {
        uint32_t ro[U];
        T ax[U], ay[U], az[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = s0 + u * NT;
            const bool ok = i < s_end;
            ro[u] = ok ? (ALL_TH ? leaf_end : (uint32_t)role[i]) : 0xFFFFFFFFu;
            ax[u] = ok ? vx[i] : T(0);
            ay[u] = ok ? vy[i] : T(0);
            az[u] = ok ? vz[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = ro[u];
            if (i == 0xFFFFFFFFu) continue;
            if (i < kept_end) {
                const double d = (double)ax[u] - mx;
                sums[0] += d * d;
            } else if (i < leaf_end) {
                const uint32_t r = leaf_rank(i, N0, P);
                if (r >= r_done) st3(leaf + r, ax[u], ay[u], az[u]);
            } else {
                if (pool_all && i - N0 >= r_done) st3(leaf + (i - N0), ax[u], ay[u], az[u]);
                const double dx = (double)ax[u] - mx, dy = (double)ay[u] - my, dz = (double)az[u] - mz;
                sums[1] += dx * dx;
                sums[2] += dx;
                sums[3] += dy;
                sums[4] += dz;
                sums[5] += dx * dx + dy * dy + dz * dz;
            }
        }
    }
}

// d. Collisions, shallowest level first; all collisions of a level in parallel
//    (eq. Maxwell_coll-r, eq. n3d-r; Alg. 4.4 acceptance).  Leaf r is read
//    from leaf[r] (gathered before), or with FromSlots from its slot
//    fwd[leaf_role(r)] of the pre-step velocities (vx, vy, vz); final r is
//    stored at fin[r] (the write-back puts it in the slot of leaf r).
//    Per-thread counters and the finals' sum of (vx-m)^2.
#ifndef TRMC_BOTTOM_UP_BATCH
#define TRMC_BOTTOM_UP_BATCH 2
#endif
constexpr int kBU = TRMC_BOTTOM_UP_BATCH;  // collisions per thread per batch in bottom_up

// Majorant raised level by level (Remark 4.1): the bound of level l + 1 is the
// majorant of the largest distance to the cell mean among the pre-step
// velocities (d2seen starts at their largest squared distance) and the outputs
// of levels 1..l.  red: group reduction scratch; g: the bound of the next level.
struct DynMajorant {
    double* red;
    double alpha, d2seen, g;
};

// Tree-shape truncation: the finals longer than m_max, summed where they are
// made.  z: the normals of their slots (sum of the 3 components, sum of |z|^2);
// d: their values less the cell mean (3 sums, sum of |v - mean|^2); cnt: count.
struct WbAcc {
    double z[4], d[4], cnt;
};

template <typename T, int G, bool FromSlots, bool WB = false, bool REUSE = false, typename R = uint32_t>
__device__ __forceinline__ void bottom_up(const Key& key, uint32_t n, gptr<const T> vx, gptr<const T> vy,
                                          gptr<const T> vz,
                                          const Levels& L, const CellShared& sh, const CellMem<T, R>& M,
                                          unsigned long long ncoll, T alpha, T gT, double mx, uint32_t tid,
                                          uint32_t& dummies, uint32_t& viol, double& sfin, uint32_t wbk = 0,
                                          const uint32_t* coff = nullptr, uint32_t r0prev = 0,
                                          WbAcc* wba = nullptr, T wbmax = T(0), DynMajorant* dm = nullptr,
                                          uint32_t l_first = 1)
{
    const uint32_t N0 = uni(sh.N0), P = n - N0, me = uni(sh.me);
    // tree-shape truncation: a dropped final's slot is the permutation of its
    // leaf's role index, where its Maxwellian normals are drawn
    [[maybe_unused]] uint4 pk{};
    [[maybe_unused]] uint32_t pbits = 0;
    if constexpr (WB) {
        pk = draw(key, 0, TAG_PERM, 0);
        pbits = perm_bits(n);
    }
    unsigned long long above = ncoll;  // collisions of deeper levels precede level l's
    uint32_t fp = REUSE ? r0prev : 0u; // finals of shallower levels (and of earlier attempts)
    // leaves of this attempt: ranks from r0prev on (reuse) or from 0
    const gptr<Pack4<T>> leafb = M.leaf + (REUSE ? r0prev : 0u);
    for (uint32_t l = 1; l <= me; ++l) {
        const uint32_t Cl = uni(L.C[l]), Rl = uni(L.Rtot[l]);
        if (Cl == 0) continue;
        if (l < l_first) {
            // made elsewhere (the tile pipeline's level-1 kernel): only the offsets move on
            above -= Cl;
            fp += 2u * Cl - Rl;
            continue;
        }
        above -= Cl;
        const uint32_t fst = (uint32_t)above;
        const uint32_t oo = uni(L.outoff[l]);
        [[maybe_unused]] const uint32_t c_off = REUSE ? uni(coff[l]) : 0u;
        double lvmax = 0.0;  // dynamic majorant: largest |output - mean|^2 of this level (this thread)
        // kBU collisions per thread: every index and input load of the batch
        // is issued before the first collision is computed
        for (uint32_t c0 = tid; c0 < Cl; c0 += G * kBU) {
            Vec3<T> a[kBU], b[kBU];
            T len[kBU];  // tree-shape truncation: length of the collision's outputs
#pragma unroll
            for (int k = 0; k < kBU; ++k) {
                const uint32_t c = c0 + (uint32_t)k * G;
                const uint32_t id = fst + (c < Cl ? c : 0u);  // collision 0 stands in past the end
                const uint32_t j = M.jarr[id], h = l - 1u - j;
                const uint32_t ra = M.rA[id], rb = M.rB[id];
                T la = T(0), lb = T(0);  // a leaf has length 0
                if (j == 0) {
                    if constexpr (FromSlots) {
                        const uint32_t sl = M.fwd[leaf_role(ra, N0, P)];
                        a[k] = Vec3<T>{vx[sl], vy[sl], vz[sl]};
                    } else {
                        a[k] = ld3(leafb + ra);
                    }
                } else if constexpr (WB) {
                    const Pack4<T> p = ld4(M.outv + ((uint64_t)L.outoff[j] + ra));
                    a[k] = Vec3<T>{p.x, p.y, p.z};
                    la = p.w;
                } else {
                    a[k] = ld3(M.outv + ((uint64_t)L.outoff[j] + ra));
                }
                if (h == 0) {
                    if constexpr (FromSlots) {
                        const uint32_t sl = M.fwd[leaf_role(rb, N0, P)];
                        b[k] = Vec3<T>{vx[sl], vy[sl], vz[sl]};
                    } else {
                        b[k] = ld3(leafb + rb);
                    }
                } else if constexpr (WB) {
                    const Pack4<T> p = ld4(M.outv + ((uint64_t)L.outoff[h] + rb));
                    b[k] = Vec3<T>{p.x, p.y, p.z};
                    lb = p.w;
                } else {
                    b[k] = ld3(M.outv + ((uint64_t)L.outoff[h] + rb));
                }
                if constexpr (WB) {
                    // Sec. 4.4: def:2 is 1 + min, def:3 is 1 + mean of the inputs' lengths
#pragma clang fp contract(off)
                    len[k] = wbk == WB_MIN ? T(1) + (la < lb ? la : lb) : (la + lb) * T(0.5) + T(1);
                } else {
                    len[k] = T(0);
                }
            }
#pragma unroll
            for (int k = 0; k < kBU; ++k) {
                const uint32_t c = c0 + (uint32_t)k * G;
                if (c >= Cl) break;
                T xi1, xi2, xacc;
                Draws<T>::coll(key, l, REUSE ? c_off + c : c, xi1, xi2, xacc);
                Vec3<T> out[2];
                if (!collide<T>(a[k], b[k], xi1, xi2, xacc, alpha, gT, out[0], out[1], viol)) dummies++;
                if (dm) {
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const double ex = (double)out[e].x - mx, ey = (double)out[e].y - sh.mean[1],
                                     ez = (double)out[e].z - sh.mean[2];
                        const double d2 = ex * ex + ey * ey + ez * ez;
                        lvmax = d2 > lvmax ? d2 : lvmax;
                    }
                }
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const uint32_t o = 2u * c + (uint32_t)e;
                    if (o < Rl) {
                        st4(M.outv + ((uint64_t)oo + o), out[e].x, out[e].y, out[e].z, len[k]);
                    } else {
                        const uint32_t r = fp + (o - Rl);
                        st4(M.fin + r, out[e].x, out[e].y, out[e].z, len[k]);
                        const double d = (double)out[e].x - mx;
                        sfin += d * d;
                        if constexpr (WB) {
                            if (len[k] > wbmax) {
                                const uint32_t sl = perm_forward(leaf_role(r, N0, P), n, pbits, pk);
                                const Vec3<T> z = Draws<T>::normals(key, sl);  // keyed by the slot
                                const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
                                wba->z[0] += zx;
                                wba->z[1] += zy;
                                wba->z[2] += zz;
                                wba->z[3] += zx * zx + zy * zy + zz * zz;
                                const double dy = (double)out[e].y - sh.mean[1], dz = (double)out[e].z - sh.mean[2];
                                wba->d[0] += d;
                                wba->d[1] += dy;
                                wba->d[2] += dz;
                                wba->d[3] += d * d + dy * dy + dz * dz;
                                wba->cnt += 1.0;
                            }
                        }
                    }
                }
            }
        }
        fp += 2u * Cl - Rl;
        if (dm) {
            // the bound of the next level (every thread computes the same value)
            const double lm = gmax<G>(lvmax, dm->red);
            dm->d2seen = lm > dm->d2seen ? lm : dm->d2seen;
            dm->g = majorant_of(dm->alpha, dm->d2seen);
            gT = (T)dm->g;
        }
        gsync<G>();
    }
}

// e. Adaptive test of Sec. 4.3 (thread 0): S^{n+1,m} from the unchanged set, the
//    finals and the analytic Maxwellian part; halve / keep / redo at 2m.  Also
//    records the removed set's mean and energy.  all = {kept (vx-m)^2, th
//    (vx-m)^2, th v-m (3), th |v-m|^2, finals (vx-m)^2}.
__device__ __forceinline__ void decide(InstDev* I, uint32_t cell, uint32_t n, const double (&all)[7], double mx,
                                       double my, double mz, CellShared& sh)
{
    double Snew = all[0] + all[6];
    const uint32_t n_th = sh.n_th;
    if (n_th >= 2) {
        const double nt = (double)n_th;
        const double d0 = all[2] / nt, d1 = all[3] / nt, d2 = all[4] / nt;
        sh.ur[0] = mx + d0;
        sh.ur[1] = my + d1;
        sh.ur[2] = mz + d2;
        const double E = all[5] - nt * (d0 * d0 + d1 * d1 + d2 * d2);
        sh.a_th = E > 0.0 ? E : 0.0;  // energy of the removed set
        Snew += E / 3.0 + nt * d0 * d0;
    } else {
        Snew += all[1];
        sh.a_th = 0.0;
    }
    uint32_t decision = 1;  // accept
    sh.E1 = 0.0;
    if (I->trunc == TRUNC_ADAPTIVE || I->trunc == TRUNC_ADAPTIVE_REUSE) {
        const uint32_t m = sh.m;
        if (sh.Sn == 0.0) {
            I->m_state[cell] = m;
        } else {
#pragma clang fp contract(off)
            Snew /= (double)n;
            const double E1 = fabs(Snew - sh.Sn) / fabs(sh.Sn);
            sh.E1 = E1;
            if (E1 < I->delta1) I->m_state[cell] = (m / 2u > 1u) ? m / 2u : 1u;
            else if (E1 <= I->delta2) I->m_state[cell] = m;
            else if (m >= I->m_cap || sh.split_rem == 0u || sh.ext_empty) I->m_state[cell] = m;
            else {
                sh.m = (2u * m < I->m_cap) ? 2u * m : I->m_cap;
                decision = 0;
            }
        }
    }
    sh.decision = decision;
}

// Sums over the roles [lo, hi) of a cell, centred on the cell mean m: whole
// blocks of kRoleBlock roles from the block sums bs (8 doubles each: sum of
// v - m (3), of (vx - m)^2, of |v - m|^2), the partial blocks at both ends from
// the slots fwd[i] of the velocities.  This thread's share in out[5]; the
// caller reduces over the group.
template <typename T, int G>
__device__ __forceinline__ void range_sums(gptr<const T> vx, gptr<const T> vy, gptr<const T> vz,
                                           gptr<const uint32_t> fwd,
                                           const double* bs, uint32_t lo, uint32_t hi, double mx, double my,
                                           double mz, uint32_t tid, double (&out)[5])
{
    if (lo >= hi) return;
    const uint32_t b_lo = (lo + kRoleBlock - 1) / kRoleBlock, b_hi = hi / kRoleBlock;
    auto add_one = [&](uint32_t i) {
        const uint32_t sl = fwd[i];
        const double dx = (double)vx[sl] - mx, dy = (double)vy[sl] - my, dz = (double)vz[sl] - mz;
        out[0] += dx;
        out[1] += dy;
        out[2] += dz;
        out[3] += dx * dx;
        out[4] += dx * dx + dy * dy + dz * dz;
    };
    if (b_lo >= b_hi) {  // inside one block
        for (uint32_t i = lo + tid; i < hi; i += G) add_one(i);
        return;
    }
    for (uint32_t i = lo + tid; i < b_lo * kRoleBlock; i += G) add_one(i);
    for (uint32_t i = b_hi * kRoleBlock + tid; i < hi; i += G) add_one(i);
    for (uint32_t b = b_lo + tid; b < b_hi; b += G) {
        const double* p = bs + 8ull * b;
        out[0] += p[0];
        out[1] += p[1];
        out[2] += p[2];
        out[3] += p[3];
        out[4] += p[4];
    }
}

// Sums of an attempt: all = {kept (vx-m)^2, th (vx-m)^2, th v-m (3), th
// |v-m|^2, (finals, filled by the caller)}.
template <typename T, int G>
__device__ __forceinline__ void attempt_sums(gptr<const T> vx, gptr<const T> vy, gptr<const T> vz,
                                             gptr<const uint32_t> fwd,
                                             const double* bs, uint32_t n, uint32_t kept_end, uint32_t leaf_end,
                                             double mx, double my, double mz, uint32_t tid, double* red,
                                             double (&all)[7])
{
    double k5[5] = {0, 0, 0, 0, 0}, t5[5] = {0, 0, 0, 0, 0};
    range_sums<T, G>(vx, vy, vz, fwd, bs, 0u, kept_end, mx, my, mz, tid, k5);
    range_sums<T, G>(vx, vy, vz, fwd, bs, leaf_end, n, mx, my, mz, tid, t5);
    double v[6] = {k5[3], t5[3], t5[0], t5[1], t5[2], t5[4]};
    gsum<G, 6>(v, red);
    for (int q = 0; q < 6; ++q) all[q] = v[q];
}

// Wall-clock ticks since t_begin (100 MHz constant-rate counter), saturated to 32 bits.
__device__ __forceinline__ uint32_t elapsed_ticks(uint64_t t_begin)
{
    const uint64_t d = wall_clock64() - t_begin;
    return d > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)d;
}

__device__ __forceinline__ void write_stats(CellStats* st, uint32_t n, const CellShared& sh, uint32_t ticks = 0)
{
    CellStats s{};
    s.ticks = ticks;
    s.n = n;
    s.N0 = sh.N0;
    s.m_eff = sh.me;
    s.m_used = sh.m;
    s.attempts = sh.attempts;
    s.R0 = sh.R0;
    s.n_th = sh.n_th;
    s.wb_th = sh.wb_th;
    s.borrowed = sh.borrowed;
    s.folds = sh.folds;
    s.status = 0;
    s.collisions = sh.ncoll;
    s.dummies = sh.dummies;
    s.violations = sh.viol;
    s.work_collisions = sh.work;
    s.q = sh.q;
    s.g = sh.g_last;
    s.E1 = sh.E1;
    s.mean[0] = sh.mean[0];
    s.mean[1] = sh.mean[1];
    s.mean[2] = sh.mean[2];
    *st = s;
}

}  // namespace trmc
