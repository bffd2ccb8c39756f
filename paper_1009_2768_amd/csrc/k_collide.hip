// k_collide.hip -- the per-cell TRMC-R collision step (Trazzi, Pareschi and
// Wennberg, Sec. 4), one workgroup per cell.
//
// Per cell and step, in order:
//   1. FP64 moments of the cell: mean, dv = max|v - mean| (Sec. 4.2), S = P_xx.
//   2. Majorant g = (2 dv)^alpha on a 20-bit grid, mu = rho_c g, q = exp(-mu dt/eps)
//      (tau = 1 - q, Sec. 3.2).
//   3. Role index of every slot: inverse of a keyed permutation (who stays
//      unchanged, who is a leaf of a collision tree, who is thermalized).
//   4. Attempt loop at depth m (Sec. 4.3 redoes it at 2m):
//      a. split into collision sets N_0..N_{m+1} (Alg. 4.2, Iround, q directly);
//      b. counting pass of the trees, deepest level first: ceil(R_l/2) collisions
//         serve the R_l requests to level l, an odd R_l leaves a stored twin that
//         is final, the level's own loop adds ceil(max(0, N_l - odd)/2)
//         collisions; each collision asks level j and level l-1-j for an input,
//         j uniform in {0..l-1} (Alg. 4.3); while the leaves exceed n, fold the
//         deepest level into the remainder;
//      c. ranking pass: stable ranks of the requests at every level (wave ballot
//         over distinct target levels), so request r of level t takes output r;
//      d. gather the leaves, FP64 sums of the unchanged and thermalized sets;
//      e. collisions shallowest level first, all collisions of a level in
//         parallel (eq. Maxwell_coll-r, eq. n3d-r; Alg. 4.4 acceptance for VHS);
//      f. Box-Muller normals of the thermalized set and their FP64 sums;
//      g. adaptive test E_1 = |S^{n+1,m} - S^n| / |S^n| with the analytic
//         Maxwellian part (Sec. 4.3).
//   5. Write back: leaf slots take the finals, thermalized slots the Maxwellian
//      samples affinely rescaled to the removed particles' momentum and energy.
#include <hip/hip_runtime.h>

#include "trmc_device.h"
#include "trmc_internal.h"

namespace trmc {

template <typename T>
struct Vec3 {
    T x, y, z;
};

// Collision draws: FP64 takes the high bits from block 0 and the low bits from
// block 1; FP32 takes block 0 only (its uniforms are the top 24 bits of FP64's).
template <typename T>
__device__ __forceinline__ void coll_uniforms(const Key& k, uint32_t l, uint32_t c, bool need_acc, T& xi1, T& xi2,
                                              T& xacc);

template <>
__device__ __forceinline__ void coll_uniforms<double>(const Key& k, uint32_t l, uint32_t c, bool, double& xi1,
                                                      double& xi2, double& xacc)
{
    const uint4 b0 = draw(k, c, TAG_COLL, l);
    const uint4 b1 = draw(k, c, TAG_COLL, l | (1u << 20));
    xi1 = u53(b0.x, b1.x);
    xi2 = u53(b0.y, b1.y);
    xacc = u53(b0.z, b1.z);
}

template <>
__device__ __forceinline__ void coll_uniforms<float>(const Key& k, uint32_t l, uint32_t c, bool, float& xi1,
                                                     float& xi2, float& xacc)
{
    const uint4 b0 = draw(k, c, TAG_COLL, l);
    xi1 = u24(b0.x);
    xi2 = u24(b0.y);
    xacc = u24(b0.z);
}

__device__ __forceinline__ double tsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float tsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ void tsincos2pi(double u, double& s, double& c)
{
    const double a = 6.283185307179586 * u;
    s = sin(a);
    c = cos(a);
}
__device__ __forceinline__ void tsincos2pi(float u, float& s, float& c)
{
    const float a = 6.2831853071795865f * u;
    s = sinf(a);
    c = cosf(a);
}
__device__ __forceinline__ double tlog1m(double u) { return log(1.0 - u); }
__device__ __forceinline__ float tlog1m(float u) { return logf(1.0f - u); }
__device__ __forceinline__ double tpow(double a, double b) { return pow(a, b); }
__device__ __forceinline__ float tpow(float a, float b) { return powf(a, b); }

// One collision of eq. (Maxwell_coll-r); dummy (outputs = inputs) unless
// xi_acc * g < |q|^alpha.  Returns 1 if real.
template <typename T>
__device__ __forceinline__ int collide(const Vec3<T>& a, const Vec3<T>& b, T xi1, T xi2, T xacc, T alpha, T g,
                                       Vec3<T>& oa, Vec3<T>& ob, uint32_t& viol)
{
    const T qx = a.x - b.x, qy = a.y - b.y, qz = a.z - b.z;
    const T qn = tsqrt(qx * qx + qy * qy + qz * qz);
    if (alpha != T(0)) {
        const T s = (alpha == T(1)) ? qn : tpow(qn, alpha);
        viol += (s > g) ? 1u : 0u;
        if (!(xacc * g < s)) {
            oa = a;
            ob = b;
            return 0;
        }
    }
    const T ct = T(2) * xi1 - T(1);
    const T st2 = T(1) - ct * ct;
    const T st = tsqrt(st2 > T(0) ? st2 : T(0));
    T sp, cp;
    tsincos2pi(xi2, sp, cp);
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

// Three standard normals for thermalized ordinal t (Box-Muller on MAXW draws).
template <typename T>
__device__ __forceinline__ Vec3<T> maxw_normals(const Key& k, uint32_t t);

template <>
__device__ __forceinline__ Vec3<double> maxw_normals<double>(const Key& k, uint32_t t)
{
    const uint4 b0 = draw(k, t, TAG_MAXW, 0);
    const uint4 b1 = draw(k, t, TAG_MAXW, 1);
    const double u0 = u53(b0.x, b1.x), u1 = u53(b0.y, b1.y), u2 = u53(b0.z, b1.z), u3 = u53(b0.w, b1.w);
    const double r1 = sqrt(-2.0 * log(1.0 - u0));
    const double r2 = sqrt(-2.0 * log(1.0 - u2));
    double s1, c1, s2, c2;
    tsincos2pi(u1, s1, c1);
    tsincos2pi(u3, s2, c2);
    return Vec3<double>{r1 * c1, r1 * s1, r2 * c2};
}

template <>
__device__ __forceinline__ Vec3<float> maxw_normals<float>(const Key& k, uint32_t t)
{
    const uint4 b0 = draw(k, t, TAG_MAXW, 0);
    const float u0 = u24(b0.x), u1 = u24(b0.y), u2 = u24(b0.z), u3 = u24(b0.w);
    const float r1 = sqrtf(-2.0f * logf(1.0f - u0));
    const float r2 = sqrtf(-2.0f * logf(1.0f - u2));
    float s1, c1, s2, c2;
    tsincos2pi(u1, s1, c1);
    tsincos2pi(u3, s2, c2);
    return Vec3<float>{r1 * c1, r1 * s1, r2 * c2};
}

// Scalars shared by the workgroup.
struct CellShared {
    double mean[3];
    double Sn, q, g, ur[3], a_th, zbar[3], E1;
    uint32_t me, split_rem, R0, N0, borrowed, n_th, folds, m, attempts, decision, overflow;
    unsigned long long ncoll, work;
    uint32_t dummies, viol;
};

// Level arrays in dynamic LDS, (m_cap + 2) entries each.
struct Levels {
    uint32_t *N, *Rtot, *C, *first, *outoff, *Fpre, *run;
};

template <typename T>
__global__ __launch_bounds__(kCollideThreads) void k_collide(const CellRef* __restrict__ work, uint32_t n_work,
                                                             uint32_t lv_stride)
{
    extern __shared__ uint32_t lds_levels[];
    __shared__ double red[(kCollideThreads / 64) * 12];
    __shared__ unsigned long long redu[(kCollideThreads / 64) * 4];
    __shared__ CellShared sh;

    const uint32_t wi = blockIdx.x;
    if (wi >= n_work) return;
    const uint32_t tid = threadIdx.x, nth = blockDim.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    InstDev* __restrict__ I = work[wi].inst;
    const uint32_t cell = work[wi].cell;
    const uint32_t off = I->cell_off[cell];
    const uint32_t n = I->cell_off[cell + 1] - off;
    const uint32_t buf = (I->geometry == GEOM_SLAB) ? (I->cur ^ 1u) : 0u;
    T* __restrict__ vx = reinterpret_cast<T*>(I->vx[buf]) + off;
    T* __restrict__ vy = reinterpret_cast<T*>(I->vy[buf]) + off;
    T* __restrict__ vz = reinterpret_cast<T*>(I->vz[buf]) + off;
    CellStats* st = I->stats + cell;
    const Key key{I->seed, I->uid, cell, I->step};

    if (n < 2) {
        if (tid == 0) {
            CellStats s{};
            s.n = n;
            s.m_used = I->m_state[cell];
            s.attempts = 0;
            *st = s;
        }
        return;
    }

    // Scratch of this cell.
    const uint64_t cap = coll_cap(n);
    unsigned char* base = I->scratch + I->scratch_bpp * (uint64_t)off + I->scratch_cpc * (uint64_t)cell;
    uint32_t* role = reinterpret_cast<uint32_t*>(base);
    base += align16(4ull * n);
    T* leaf = reinterpret_cast<T*>(base);  // [3][n]
    base += 3 * align16(sizeof(T) * (uint64_t)n);
    T* fin = reinterpret_cast<T*>(base);   // [3][n]
    base += 3 * align16(sizeof(T) * (uint64_t)n);
    uint32_t* jarr = reinterpret_cast<uint32_t*>(base);
    base += align16(4ull * cap);
    uint32_t* rA = reinterpret_cast<uint32_t*>(base);
    base += align16(4ull * cap);
    uint32_t* rB = reinterpret_cast<uint32_t*>(base);
    base += align16(4ull * cap);
    T* outv = reinterpret_cast<T*>(base);  // [3][2 cap]
    const uint64_t ocap = 2ull * cap;

    Levels L;
    L.N = lds_levels;
    L.Rtot = L.N + lv_stride;
    L.C = L.Rtot + lv_stride;
    L.first = L.C + lv_stride;
    L.outoff = L.first + lv_stride;
    L.Fpre = L.outoff + lv_stride;
    L.run = L.Fpre + lv_stride;

    // ---- 1. moments of the cell -------------------------------------------
    {
        double s[3] = {0.0, 0.0, 0.0};
        for (uint32_t i = tid; i < n; i += nth) {
            s[0] += (double)vx[i];
            s[1] += (double)vy[i];
            s[2] += (double)vz[i];
        }
        block_sum<3>(s, red);
        const double inv = 1.0 / (double)n;
        const double mx = s[0] * inv, my = s[1] * inv, mz = s[2] * inv;
        double d2max = 0.0;
        double sx[1] = {0.0};
        for (uint32_t i = tid; i < n; i += nth) {
            const double dx = (double)vx[i] - mx, dy = (double)vy[i] - my, dz = (double)vz[i] - mz;
            const double d2 = dx * dx + dy * dy + dz * dz;
            d2max = d2 > d2max ? d2 : d2max;
            sx[0] += dx * dx;
        }
        const double dmax = block_max(d2max, red);
        block_sum<1>(sx, red);
        if (tid == 0) {
            sh.mean[0] = mx;
            sh.mean[1] = my;
            sh.mean[2] = mz;
            sh.Sn = sx[0] / (double)n;
            double g = 1.0;
            if (I->alpha != 0.0) {
#pragma clang fp contract(off)
                const double two_dv = 2.0 * sqrt(dmax);
                g = grid_up20(I->alpha == 1.0 ? two_dv : pow(two_dv, I->alpha));
            }
            const double eps = I->eps_cells[cell];
            double mu, xarg;
            {
#pragma clang fp contract(off)
                const double rho = (double)n * I->rho_factor;
                mu = rho * g;
                xarg = mu * I->dt / eps;
            }
            sh.g = g;
            double q = exp_neg(xarg);
            if (!(q >= 0.0 && q <= 1.0)) q = 1.0;  // non-finite velocities: leave the cell unchanged
            sh.q = q;
            uint32_t m;
            if (I->trunc == TRUNC_FIXED) m = I->m_init;
            else if (I->trunc == TRUNC_ADAPTIVE) m = I->m_state[cell];
            else m = I->m_cap;
            if (m < 1) m = 1;
            if (m > I->m_cap) m = I->m_cap;
            sh.m = m;
            sh.attempts = 0;
            sh.work = 0;
            sh.overflow = 0;
        }
    }
    // ---- 3. role index of every slot --------------------------------------
    {
        const uint4 pk = draw(key, 0, TAG_PERM, 0);
        const uint32_t half = perm_half(n);
        for (uint32_t s = tid; s < n; s += nth) role[s] = perm_inverse(s, n, half, pk);
    }
    __syncthreads();

    const double mx = sh.mean[0], my = sh.mean[1], mz = sh.mean[2];
    const double q = sh.q;
    const T alpha = (T)I->alpha;
    const T gT = (T)sh.g;

    // ---- 4. attempts ------------------------------------------------------
    for (;;) {
        // a. split (Alg. 4.2)
        if (tid == 0) {
            const uint32_t m = sh.m;
            uint4 w = draw(key, 0, TAG_SPLIT, 0);
            const uint32_t N0 = iround_prod(q, n, u53(w.x, w.y));
            uint32_t rem = n - N0, k = 0;
            L.N[0] = N0;
            while (rem > 0 && k < m) {
                ++k;
                w = draw(key, k, TAG_SPLIT, 0);
                const uint32_t Nk = iround_prod(q, rem, u53(w.x, w.y));
                L.N[k] = Nk;
                rem -= Nk;
            }
            L.N[k + 1] = rem;
            sh.me = k;
            sh.split_rem = rem;
            sh.N0 = N0;
            sh.folds = 0;
            sh.attempts += 1;
        }
        __syncthreads();

        // b. counting pass with folding
        for (;;) {
            const uint32_t me = sh.me;
            for (uint32_t l = tid; l <= me; l += nth) L.run[l] = 0;
            __syncthreads();
            for (uint32_t l = me; l >= 1; --l) {
                const uint32_t Rl = L.run[l];
                const uint32_t odd = Rl & 1u, Nl = L.N[l];
                const uint32_t own = Nl > odd ? (Nl - odd + 1u) / 2u : 0u;
                const uint32_t Cl = (Rl + 1u) / 2u + own;
                if (tid == 0) {
                    L.C[l] = Cl;
                    L.Rtot[l] = Rl;
                }
                for (uint32_t c = tid; c < Cl; c += nth) {
                    const uint32_t j = tree_choice(key, l, c);
                    atomicAdd(&L.run[j], 1u);
                    atomicAdd(&L.run[l - 1u - j], 1u);
                }
                __syncthreads();
            }
            if (tid == 0) {
                L.Rtot[0] = L.run[0];
                sh.R0 = L.run[0];
            }
            __syncthreads();
            if (sh.R0 <= n) break;
            if (tid == 0) {
                L.N[me] += L.N[me + 1];
                sh.me = me - 1u;
                sh.folds += 1;
            }
            __syncthreads();
        }
        const uint32_t me = sh.me;
        const uint32_t R0 = sh.R0;

        // level offsets and capacity
        if (tid == 0) {
            unsigned long long nc = 0, no = 0;
            uint32_t fp = 0;
            for (uint32_t l = me; l >= 1; --l) {
                L.first[l] = (uint32_t)nc;
                nc += L.C[l];
            }
            for (uint32_t l = 1; l <= me; ++l) {
                L.outoff[l] = (uint32_t)no;
                no += L.Rtot[l];
                L.Fpre[l] = fp;
                fp += 2u * L.C[l] - L.Rtot[l];
            }
            sh.ncoll = nc;
            sh.work += nc;
            sh.overflow = (nc > cap || no > ocap) ? 1u : 0u;
            const uint32_t N0 = sh.N0, P = n - N0;
            sh.borrowed = R0 > P ? R0 - P : 0u;
            sh.n_th = R0 < P ? P - R0 : 0u;
        }
        __syncthreads();
        if (sh.overflow) break;

        // c. ranking pass (wave 0; requests in order A_0, B_0, A_1, B_1, ...)
        for (uint32_t l = tid; l <= me; l += nth) L.run[l] = 0;
        __syncthreads();
        if (wave == 0) {
            const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64u - lane));
            for (uint32_t l = me; l >= 1; --l) {
                const uint32_t Cl = L.C[l], fst = L.first[l];
                for (uint32_t b0 = 0; b0 < Cl; b0 += 64u) {
                    const uint32_t c = b0 + lane;
                    const bool valid = c < Cl;
                    const uint32_t j = valid ? tree_choice(key, l, c) : 0u;
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
                        __builtin_amdgcn_wave_barrier();
                    }
                    if (valid) {
                        jarr[fst + c] = j;
                        rA[fst + c] = rkA;
                        rB[fst + c] = rkB;
                    }
                }
            }
        }
        __syncthreads();

        // d. leaves, and sums of the unchanged and thermalized sets
        const uint32_t N0 = sh.N0, borrowed = sh.borrowed, n_th = sh.n_th;
        const uint32_t P = n - N0;
        const uint32_t kept_end = N0 - borrowed;
        const uint32_t leaf_end = N0 + (R0 < P ? R0 : P);
        double sums[6] = {0, 0, 0, 0, 0, 0};  // Skept, Sth_x, dth(3), Eth(|v-mean|^2)
        for (uint32_t s = tid; s < n; s += nth) {
            const uint32_t i = role[s];
            if (i < kept_end) {
                const double d = (double)vx[s] - mx;
                sums[0] += d * d;
            } else if (i < leaf_end) {
                const uint32_t r = (i < N0) ? P + (N0 - 1u - i) : i - N0;
                leaf[r] = vx[s];
                leaf[n + r] = vy[s];
                leaf[2 * n + r] = vz[s];
            } else {
                const double dx = (double)vx[s] - mx, dy = (double)vy[s] - my, dz = (double)vz[s] - mz;
                sums[1] += dx * dx;
                sums[2] += dx;
                sums[3] += dy;
                sums[4] += dz;
                sums[5] += dx * dx + dy * dy + dz * dz;
            }
        }
        __syncthreads();  // leaves visible

        // e. collisions, shallowest level first
        uint32_t dummies = 0, viol = 0;
        double sfin[1] = {0.0};
        for (uint32_t l = 1; l <= me; ++l) {
            const uint32_t Cl = L.C[l], fst = L.first[l], Rl = L.Rtot[l];
            const uint32_t oo = L.outoff[l], fp = L.Fpre[l];
            for (uint32_t c = tid; c < Cl; c += nth) {
                const uint32_t id = fst + c;
                const uint32_t j = jarr[id], h = l - 1u - j;
                const uint32_t ra = rA[id], rb = rB[id];
                Vec3<T> a, b;
                if (j == 0) {
                    a = Vec3<T>{leaf[ra], leaf[n + ra], leaf[2 * n + ra]};
                } else {
                    const uint64_t p = (uint64_t)L.outoff[j] + ra;
                    a = Vec3<T>{outv[p], outv[ocap + p], outv[2 * ocap + p]};
                }
                if (h == 0) {
                    b = Vec3<T>{leaf[rb], leaf[n + rb], leaf[2 * n + rb]};
                } else {
                    const uint64_t p = (uint64_t)L.outoff[h] + rb;
                    b = Vec3<T>{outv[p], outv[ocap + p], outv[2 * ocap + p]};
                }
                T xi1, xi2, xacc;
                coll_uniforms<T>(key, l, c, alpha != T(0), xi1, xi2, xacc);
                Vec3<T> oa, ob;
                if (!collide<T>(a, b, xi1, xi2, xacc, alpha, gT, oa, ob, viol)) dummies++;
                const uint32_t o0 = 2u * c, o1 = 2u * c + 1u;
                if (o0 < Rl) {
                    const uint64_t p = (uint64_t)oo + o0;
                    outv[p] = oa.x;
                    outv[ocap + p] = oa.y;
                    outv[2 * ocap + p] = oa.z;
                } else {
                    const uint32_t r = fp + (o0 - Rl);
                    fin[r] = oa.x;
                    fin[n + r] = oa.y;
                    fin[2 * n + r] = oa.z;
                    const double d = (double)oa.x - mx;
                    sfin[0] += d * d;
                }
                if (o1 < Rl) {
                    const uint64_t p = (uint64_t)oo + o1;
                    outv[p] = ob.x;
                    outv[ocap + p] = ob.y;
                    outv[2 * ocap + p] = ob.z;
                } else {
                    const uint32_t r = fp + (o1 - Rl);
                    fin[r] = ob.x;
                    fin[n + r] = ob.y;
                    fin[2 * n + r] = ob.z;
                    const double d = (double)ob.x - mx;
                    sfin[0] += d * d;
                }
            }
            __syncthreads();
        }

        // f. Maxwellian normals of the thermalized set
        double zs[4] = {0, 0, 0, 0};
        if (n_th >= 2) {
            for (uint32_t t = tid; t < n_th; t += nth) {
                const Vec3<T> z = maxw_normals<T>(key, t);
                const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
                zs[0] += zx;
                zs[1] += zy;
                zs[2] += zz;
                zs[3] += zx * zx + zy * zy + zz * zz;
            }
        }
        double all[11] = {sums[0], sums[1], sums[2], sums[3], sums[4], sums[5], sfin[0], zs[0], zs[1], zs[2], zs[3]};
        block_sum<11>(all, red);
        unsigned long long cnt[2] = {dummies, viol};
        block_sum_u64<2>(cnt, redu);

        // g. decision
        if (tid == 0) {
            double Snew = all[0] + all[6];
            if (n_th >= 2) {
                const double nt = (double)n_th;
                const double d0 = all[2] / nt, d1 = all[3] / nt, d2 = all[4] / nt;
                sh.ur[0] = mx + d0;
                sh.ur[1] = my + d1;
                sh.ur[2] = mz + d2;
                const double E = all[5] - nt * (d0 * d0 + d1 * d1 + d2 * d2);
                const double zb0 = all[7] / nt, zb1 = all[8] / nt, zb2 = all[9] / nt;
                const double Z = all[10] - nt * (zb0 * zb0 + zb1 * zb1 + zb2 * zb2);
                sh.zbar[0] = zb0;
                sh.zbar[1] = zb1;
                sh.zbar[2] = zb2;
                sh.a_th = Z > 0.0 ? sqrt((E > 0.0 ? E : 0.0) / Z) : -1.0;
                Snew += E / 3.0 + nt * d0 * d0;
            } else {
                Snew += all[1];
                sh.a_th = -1.0;
            }
            sh.dummies = (uint32_t)cnt[0];
            sh.viol = (uint32_t)cnt[1];
            uint32_t decision = 1;  // accept
            sh.E1 = 0.0;
            if (I->trunc == TRUNC_ADAPTIVE) {
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
                    else if (m >= I->m_cap || sh.split_rem == 0u) I->m_state[cell] = m;
                    else {
                        sh.m = (2u * m < I->m_cap) ? 2u * m : I->m_cap;
                        decision = 0;
                    }
                }
            }
            sh.decision = decision;
        }
        __syncthreads();
        if (sh.decision) break;
    }

    if (sh.overflow) {
        if (tid == 0) {
            CellStats s{};
            s.n = n;
            s.status = CELL_OVERFLOW;
            s.m_used = sh.m;
            *st = s;
            atomicOr(I->error, CELL_OVERFLOW);
        }
        return;
    }

    // ---- 5. write back ------------------------------------------------------
    {
        const uint32_t N0 = sh.N0, R0 = sh.R0, n_th = sh.n_th, borrowed = sh.borrowed;
        const uint32_t P = n - N0;
        const uint32_t kept_end = N0 - borrowed;
        const uint32_t leaf_end = N0 + (R0 < P ? R0 : P);
        const double a = sh.a_th;
        const double u0 = sh.ur[0], u1 = sh.ur[1], u2 = sh.ur[2];
        const double z0 = sh.zbar[0], z1 = sh.zbar[1], z2 = sh.zbar[2];
        for (uint32_t s = tid; s < n; s += nth) {
            const uint32_t i = role[s];
            if (i < kept_end) continue;
            if (i < leaf_end) {
                const uint32_t r = (i < N0) ? P + (N0 - 1u - i) : i - N0;
                vx[s] = fin[r];
                vy[s] = fin[n + r];
                vz[s] = fin[2 * n + r];
            } else if (n_th >= 2 && a >= 0.0) {
                const uint32_t t = i - N0 - R0;
                const Vec3<T> z = maxw_normals<T>(key, t);
                vx[s] = (T)(u0 + a * ((double)z.x - z0));
                vy[s] = (T)(u1 + a * ((double)z.y - z1));
                vz[s] = (T)(u2 + a * ((double)z.z - z2));
            }
        }
    }
    if (tid == 0) {
        CellStats s{};
        s.n = n;
        s.N0 = sh.N0;
        s.m_eff = sh.me;
        s.m_used = sh.m;
        s.attempts = sh.attempts;
        s.R0 = sh.R0;
        s.n_th = sh.n_th;
        s.borrowed = sh.borrowed;
        s.folds = sh.folds;
        s.status = 0;
        s.collisions = sh.ncoll;
        s.dummies = sh.dummies;
        s.violations = sh.viol;
        s.work_collisions = sh.work;
        s.q = sh.q;
        s.g = sh.g;
        s.E1 = sh.E1;
        *st = s;
    }
}

template __global__ void k_collide<float>(const CellRef*, uint32_t, uint32_t);
template __global__ void k_collide<double>(const CellRef*, uint32_t, uint32_t);

}  // namespace trmc
