// k_tiled.hip -- the collision step of homogeneous cells as a pipeline of
// lean streaming kernels over fixed tiles of kTile slots (high occupancy, many
// loads in flight) around per-cell kernels for the parts that need the whole
// cell (the trees and the collisions):
//
//   k_tile_prep    tiles: role of every slot and slot of every role (keyed
//                  permutation and its inverse), partial sums for the mean
//   k_tile_bsum    tiles: sums over blocks of roles; max |v - mean|^2 (VHS majorant)
//   k_big_split    cells: moments, tau, split (Alg. 4.2); light / heavy lists
//   k_tile_roles,  tiles: roles and block sums of the cells predicted wholly
//   k_tile_bsum<T, true>  thermalized whose split keeps or collides particles
//   k_big_tree     cells: collision trees (Alg. 4.3)
//   k_big_level1   cells x 32 workgroups: level 1 of the first attempt
//   k_big_collide  cells: sums of the unchanged / thermalized sets from block
//                  sums, collisions level by level (leaves read through the
//                  slot of each role), adaptive test (Sec. 4.3); a rejected
//                  attempt is redone inside
//   k_tile_zsum    tiles: sums of the Maxwellian normals of the thermalized slots
//   k_tile_write   tiles: leaves take the finals, thermalized slots the rescaled
//                  Maxwellian samples (normals drawn again from their keys)
//
// Partial sums are combined in tile order, so the result does not depend on
// scheduling.  Same arithmetic as the whole-cell kernel; only the order of the
// FP64 reductions differs (fixed per cell by its size).
//
// A cell whose previous step thermalized every particle (small eps) most
// likely does so again: k_tile_prep then makes no roles and k_tile_bsum no
// role-order block sums (only the VHS bound, in slot order).  An attempt that
// thermalizes every particle needs neither: its sums are the whole cell's,
// from k_tile_prep's tile sums (taken for every cell, predicted or not), and
// every slot is thermalized.  When k_big_split finds that the first attempt
// keeps or collides particles after all, k_tile_roles and k_tile_bsum<T, true>
// make the roles and the block sums; when a redo inside k_big_collide does,
// k_big_collide makes them itself, in the same order.
#include <hip/hip_runtime.h>

#include "collide_core.h"

namespace trmc {

constexpr int kTT = 512;  // threads of every tiled kernel

// State of a large cell kept between the kernels of one step.
struct BigState {
    CellShared sh;
    unsigned long long ncoll;
    uint32_t roles;  // ROLES_MADE, ROLES_NONE (predicted, not needed so far), ROLES_FIX (made by the fix kernels)
    uint32_t pad;
};
constexpr uint32_t ROLES_MADE = 0, ROLES_NONE = 1, ROLES_FIX = 2;

#ifndef TRMC_TILE_LAZY_ROLES
#define TRMC_TILE_LAZY_ROLES 1
#endif
constexpr bool kTileLazyRoles = TRMC_TILE_LAZY_ROLES != 0;

// The cell's record of its previous step says every particle was thermalized.
// Read only by the kernels before k_big_collide, which writes this step's record.
__device__ __forceinline__ bool predicted_whole(const InstDev* I, uint32_t n)
{
    if constexpr (!kTileLazyRoles) return false;
    const CellStats* st = I->stats;
    return st->n == n && st->N0 == 0u && st->n_th == n && st->status == 0u;
}

// Roles of the slots [s_begin, s_end) (keyed permutation) and the slot of each.
__device__ __forceinline__ void tile_roles(const Key& key, uint32_t n, gptr<uint32_t> role, gptr<uint32_t> fwd,
                                           uint32_t s_begin, uint32_t s_end, uint32_t tid, uint32_t stride)
{
    const uint4 pk = draw(key, 0, TAG_PERM, 0);
    const uint32_t pbits = perm_bits(n);
    for (uint32_t i = s_begin + tid; i < s_end; i += stride) {
        const uint32_t r = perm_inverse(i, n, pbits, pk);
        role[i] = r;
        fwd[r] = i;
    }
}

// |v - m|^2, the same bits wherever it is taken (slot or role order).
template <typename T>
__device__ __forceinline__ double dist2(T x, T y, T z, double mx, double my, double mz)
{
#pragma clang fp contract(off)
    const double dx = (double)x - mx, dy = (double)y - my, dz = (double)z - mz;
    return dx * dx + dy * dy + dz * dz;
}

// One role's terms of a block sum: v - m (3), (vx - m)^2, |v - m|^2 (returned too).
template <typename T>
__device__ __forceinline__ double bsum_terms(T x, T y, T z, double mx, double my, double mz, double (&sv)[5])
{
#pragma clang fp contract(off)
    const double dx = (double)x - mx, dy = (double)y - my, dz = (double)z - mz;
    const double d2 = dx * dx + dy * dy + dz * dz;
    sv[0] += dx;
    sv[1] += dy;
    sv[2] += dz;
    sv[3] += dx * dx;
    sv[4] += d2;
    return d2;
}

static_assert(sizeof(BigState) <= kBigStateBytes, "BigState exceeds its reserved bytes");

__device__ __forceinline__ BigState* big_state(const InstDev* I) { return reinterpret_cast<BigState*>(I->bigstate); }
__device__ __forceinline__ uint32_t* big_levels(const InstDev* I)
{
    return reinterpret_cast<uint32_t*>(I->bigstate + kBigStateBytes);
}
// level-1 partial sums of kLevel1Blocks workgroups: {finals' (vx - m)^2, dummies, violations, 0} each
__device__ __forceinline__ double* big_parts(const InstDev* I)
{
    return reinterpret_cast<double*>(I->bigstate + kBigStateBytes + big_levels_bytes(I->m_cap));
}
// Level 1 of the first attempt is made by k_big_level1 (not for the majorant
// raised level by level, whose bound comes from the levels in turn).
__device__ __forceinline__ bool level1_apart(const InstDev* I)
{
    return !(I->majorant == MAJ_LEVEL && I->alpha != 0.0);
}

template <typename T>
struct CellView {
    InstDev* I;
    uint32_t n;
    T *vx, *vy, *vz;
    __device__ __forceinline__ CellView(InstDev* inst)
    {
        I = inst;
        n = I->cell_off[1] - I->cell_off[0];
        vx = reinterpret_cast<T*>(I->vx[0]);
        vy = reinterpret_cast<T*>(I->vy[0]);
        vz = reinterpret_cast<T*>(I->vz[0]);
    }
};

template <typename T>
__global__ __launch_bounds__(kTT) void k_tile_prep(const CellRef* __restrict__ bigs, const uint32_t* __restrict__ prefix,
                                                   uint32_t nb, uint32_t* __restrict__ list_count)
{
    if (blockIdx.x == 0 && threadIdx.x < 2u) list_count[threadIdx.x] = 0u;  // lists of this step
    __shared__ double t_red[(kTT / 64) * 8];
    uint32_t b, k;
    tile_of(prefix, nb, blockIdx.x, b, k);
    CellView<T> V(bigs[b].inst);
    const uint32_t n = V.n;
    const uint32_t s_begin = k * kTile, s_end = (s_begin + kTile < n) ? s_begin + kTile : n;
    const Key key{V.I->seed, V.I->uid, 0u, V.I->step};
    const uint4 pk = draw(key, 0, TAG_PERM, 0);
    const uint32_t pbits = perm_bits(n);
    CellMem<T> M;
    M.init(V.I, 0, 0, n);
    const gptr<uint32_t> role = M.role;
    const gptr<uint32_t> fwd = M.fwd;
    const bool make = !predicted_whole(V.I, n);
    // sums of v_x - c0, v_y, v_z, (v_x - c0)^2, (v_y - c1)^2, (v_z - c2)^2 (c: the first particle)
    const double c0 = (double)V.vx[0], c1 = (double)V.vy[0], c2 = (double)V.vz[0];
    constexpr int U = 4;
    double s[6] = {0, 0, 0, 0, 0, 0};
    T ax[U], ay[U], az[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t i = s_begin + threadIdx.x + u * kTT;
        const bool ok = i < s_end;
        ax[u] = ok ? V.vx[i] : T(0);
        ay[u] = ok ? V.vy[i] : T(0);
        az[u] = ok ? V.vz[i] : T(0);
    }
    for (uint32_t s0 = s_begin + threadIdx.x; s0 < s_end; s0 += kTT * U) {
        T bx[U], by[U], bz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = s0 + kTT * U + u * kTT;
            const bool ok = i < s_end;
            bx[u] = ok ? V.vx[i] : T(0);
            by[u] = ok ? V.vy[i] : T(0);
            bz[u] = ok ? V.vz[i] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = s0 + u * kTT;
            if (i < s_end) {
                const double dx = (double)ax[u] - c0;
                s[0] += dx;
                s[1] += (double)ay[u];
                s[2] += (double)az[u];
                s[3] += dx * dx;
                const double dy = (double)ay[u] - c1, dz = (double)az[u] - c2;
                s[4] += dy * dy;
                s[5] += dz * dz;
                if (make) {
                    const uint32_t r = perm_inverse(i, n, pbits, pk);
                    role[i] = r;
                    fwd[r] = i;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ax[u] = bx[u];
            ay[u] = by[u];
            az[u] = bz[u];
        }
    }
    gsum<kTT, 6>(s, t_red);
    if (threadIdx.x == 0) {
        double* tp = V.I->tpart + 8ull * k;  // [4] is the VHS bound (k_tile_bsum)
        tp[0] = s[0];
        tp[1] = s[1];
        tp[2] = s[2];
        tp[3] = s[3];
        tp[5] = s[4];
        tp[6] = s[5];
    }
}

// Roles of a cell found, after its split, to need them after all (ROLES_FIX).
template <typename T>
__global__ __launch_bounds__(kTT) void k_tile_roles(const CellRef* __restrict__ bigs,
                                                    const uint32_t* __restrict__ prefix, uint32_t nb)
{
    uint32_t b, k;
    tile_of(prefix, nb, blockIdx.x, b, k);
    InstDev* I = bigs[b].inst;
    if (big_state(I)->roles != ROLES_FIX) return;
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    const uint32_t s_begin = k * kTile, s_end = (s_begin + kTile < n) ? s_begin + kTile : n;
    CellMem<T> M;
    M.init(I, 0, 0, n);
    tile_roles(Key{I->seed, I->uid, 0u, I->step}, n, M.role, M.fwd, s_begin, s_end, threadIdx.x, kTT);
}

// Cell mean from the prep partials (tile order; identical wherever computed).
__device__ __forceinline__ void cell_mean(const InstDev* I, uint32_t n, double c0, double& mx, double& my, double& mz,
                                          double& Sn)
{
    const uint32_t nt = (n + kTile - 1) / kTile;
    double a = 0, b = 0, c = 0, d = 0;
    for (uint32_t t = 0; t < nt; ++t) {
        const double* tp = I->tpart + 8ull * t;
        a += tp[0];
        b += tp[1];
        c += tp[2];
        d += tp[3];
    }
    const double inv = 1.0 / (double)n;
    const double dxm = a * inv;
    mx = c0 + dxm;
    my = b * inv;
    mz = c * inv;
    const double sn = d * inv - dxm * dxm;
    Sn = sn > 0.0 ? sn : 0.0;
}

// Sums over blocks of kRoleBlock roles (each role read from its slot), centred on the
// cell mean (sum of v - m, of (vx - m)^2, of |v - m|^2), and for VHS the tile's
// max |v - m|^2.  Any role range's sums are then a few block sums plus two
// partial blocks (range_sums), so the attempts of the adaptive test cost
// O(n / kRoleBlock) instead of a pass over the cell.  A cell predicted wholly
// thermalized takes no block sums here (VHS: the max from its slots instead).
// FIX: only the block sums, of a cell whose roles were made by k_tile_roles.
template <typename T, bool FIX>
__global__ __launch_bounds__(kTT) void k_tile_bsum(const CellRef* __restrict__ bigs, const uint32_t* __restrict__ prefix,
                                                   uint32_t nb)
{
    __shared__ double t_red[(kTT / 64) * 8];
    __shared__ double mean[3];
    uint32_t b, k;
    tile_of(prefix, nb, blockIdx.x, b, k);
    if constexpr (FIX) {
        if (big_state(bigs[b].inst)->roles != ROLES_FIX) return;
    }
    CellView<T> V(bigs[b].inst);
    const uint32_t n = V.n;
    if (threadIdx.x == 0) {
        double Sn;
        cell_mean(V.I, n, (double)V.vx[0], mean[0], mean[1], mean[2], Sn);
    }
    __syncthreads();
    const double mx = mean[0], my = mean[1], mz = mean[2];
    CellMem<T> M;
    M.init(V.I, 0, 0, n);
    const gptr<const uint32_t> fwd = M.fwd;
    const uint32_t r_begin = k * kTile, r_end = (r_begin + kTile < n) ? r_begin + kTile : n;
    double d2max = 0.0;
    if (FIX || !predicted_whole(V.I, n)) {
        for (uint32_t b0 = r_begin; b0 < r_end; b0 += kRoleBlock) {
            const uint32_t b1 = (b0 + kRoleBlock < r_end) ? b0 + kRoleBlock : r_end;
            double sv[5] = {0, 0, 0, 0, 0};
            for (uint32_t i = b0 + threadIdx.x; i < b1; i += kTT) {
                const uint32_t sl = fwd[i];
                const double d2 = bsum_terms<T>(V.vx[sl], V.vy[sl], V.vz[sl], mx, my, mz, sv);
                d2max = d2 > d2max ? d2 : d2max;
            }
            gsum<kTT, 5>(sv, t_red);
            if (threadIdx.x == 0) {
                double* p = V.I->bsum + 8ull * (b0 / kRoleBlock);
                for (int q = 0; q < 5; ++q) p[q] = sv[q];
            }
        }
    } else if (!FIX && V.I->alpha != 0.0) {
        // no block sums: the bound from the slots of the tile, in slot order
        for (uint32_t i = r_begin + threadIdx.x; i < r_end; i += kTT) {
            const double d2 = dist2<T>(V.vx[i], V.vy[i], V.vz[i], mx, my, mz);
            d2max = d2 > d2max ? d2 : d2max;
        }
    }
    if (!FIX && V.I->alpha != 0.0) {
        d2max = gmax<kTT>(d2max, t_red);
        if (threadIdx.x == 0) V.I->tpart[8ull * k + 4] = d2max;
    }
}

// ---------------------------------------------------------------------------
// Per-cell kernels.  k_big_split runs one wave per cell and sorts the cells by
// the size of their trees: "light" cells (expected collisions at most
// kHeavyColl) are then processed one wave per cell, eight per workgroup, with
// no workgroup barriers, so that many cells' level-by-level chains overlap on a
// CU; "heavy" cells get a whole workgroup.  The lists are in device memory:
// list[0..count[0]) light, list[cap..cap+count[1]) heavy (order of arrival does
// not matter: every cell's arithmetic is its own).
// ---------------------------------------------------------------------------
constexpr uint32_t kHeavyColl = 1536;

struct CellLists {
    uint32_t* list;   // [2 * cap]
    uint32_t* count;  // [2]
    uint32_t cap;
};

// Group G of cell to process: light cells by wave, heavy cells by workgroup.
template <int G>
__device__ __forceinline__ bool pick_cell(const CellLists& cl, uint32_t& b)
{
    if constexpr (G == 64) {
        const uint32_t idx = blockIdx.x * (kTT / 64) + (threadIdx.x >> 6);
        if (idx >= cl.count[0]) return false;
        b = cl.list[idx];
    } else {
        if (blockIdx.x >= cl.count[1]) return false;
        b = cl.list[cl.cap + blockIdx.x];
    }
    return true;
}

template <typename T>
__global__ __launch_bounds__(kTT) void k_big_split(const CellRef* __restrict__ bigs, uint32_t nb, uint32_t lv_stride,
                                                   CellLists cl)
{
    extern __shared__ uint32_t lds_levels[];
    __shared__ CellShared shs[kTT / 64];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t b = blockIdx.x * (kTT / 64) + wave;
    if (b >= nb) return;
    InstDev* I = bigs[b].inst;
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    CellShared& sh = shs[wave];
    const Key key{I->seed, I->uid, 0u, I->step};
    Levels L = levels_at(lds_levels + (size_t)wave * 5u * lv_stride, lv_stride);
    bool pred = false;
    if (lane == 0) {
        pred = predicted_whole(I, n);  // before this step's record is written
        const T* vx = reinterpret_cast<const T*>(I->vx[0]);
        const T* vy = reinterpret_cast<const T*>(I->vy[0]);
        const T* vz = reinterpret_cast<const T*>(I->vz[0]);
        const double c0 = (double)vx[0], c1 = (double)vy[0], c2 = (double)vz[0];
        cell_mean(I, n, c0, sh.mean[0], sh.mean[1], sh.mean[2], sh.Sn);
        double dmax = 0.0;
        const uint32_t nt = (n + kTile - 1) / kTile;
        if (I->alpha != 0.0)
            for (uint32_t t = 0; t < nt; ++t) dmax = fmax(dmax, I->tpart[8ull * t + 4]);
        cell_params(I, 0, n, dmax, sh);
        sh.overflow = n < 2 ? 1u : 0u;  // cells of fewer than 2 particles are skipped
        // the whole cell's sums about its mean (tile order), for an attempt that
        // thermalizes every particle: sum of v - m (rounding only) and of |v - m|^2
        double a = 0, bb = 0, c = 0, d = 0, e = 0, f = 0;
        for (uint32_t t = 0; t < nt; ++t) {
            const double* tp = I->tpart + 8ull * t;
            a += tp[0];
            bb += tp[1];
            c += tp[2];
            d += tp[3];
            e += tp[5];
            f += tp[6];
        }
        const double nd = (double)n, dxm = a * (1.0 / nd);
        const double ey = sh.mean[1] - c1, ez = sh.mean[2] - c2;
        sh.all_th[0] = a - nd * dxm;
        sh.all_th[1] = bb - nd * sh.mean[1];
        sh.all_th[2] = c - nd * sh.mean[2];
        sh.all_th[3] = (d - nd * dxm * dxm) + (e - nd * ey * ey) + (f - nd * ez * ez);
    }
    gsync<64>();
    if (n >= 2) split_levels<64>(key, n, sh.q, L, sh, lane, adaptive_look(I));
    // expected collisions of the trees: a level-k sample costs H_k / 2 of them
    double est = 0.0, Hk = 0.0;
    if (n >= 2)
        for (uint32_t k = 1; k <= sh.me; ++k) {
            Hk += 1.0 / (double)k;
            est += 0.5 * Hk * (double)L.N[k];
        }
    BigState* S = big_state(I);
    uint32_t* gL = big_levels(I);
    for (uint32_t i = lane; i < 5u * lv_stride; i += 64u) gL[i] = L.N[i];
    if (lane == 0) {
        S->sh = sh;
        S->ncoll = 0;
        // roles of a cell predicted wholly thermalized: none yet, or made now by the
        // fix kernels when this attempt keeps or collides particles after all
        S->roles = (!pred || n < 2) ? ROLES_MADE : (sh.split_rem == n ? ROLES_NONE : ROLES_FIX);
        if (n >= 2) {
            const uint32_t heavy = est > (double)kHeavyColl ? 1u : 0u;
            const uint32_t idx = atomicAdd(&cl.count[heavy], 1u);
            cl.list[heavy * cl.cap + idx] = b;
        } else {
            CellStats s{};  // skipped: no attempt, no draws
            s.n = n;
            *I->stats = s;
        }
    }
}

template <typename T, int G>
__global__ __launch_bounds__(kTT) void k_big_tree(const CellRef* __restrict__ bigs, uint32_t lv_stride, CellLists cl)
{
    extern __shared__ uint32_t lds_levels[];
    __shared__ GroupLds<G> glds[kTT / G];
    uint32_t b;
    if (!pick_cell<G>(cl, b)) return;
    const uint32_t grp = threadIdx.x / G, tid = threadIdx.x % G;
    GroupLds<G>& gl = glds[grp];
    CellShared& sh = gl.sh;
    InstDev* I = bigs[b].inst;
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    const Key key{I->seed, I->uid, 0u, I->step};
    CellMem<T> M;
    M.init(I, 0, 0, n);
    uint32_t* lv = lds_levels + (size_t)grp * 5u * lv_stride;
    Levels L = levels_at(lv, lv_stride);
    BigState* S = big_state(I);
    uint32_t* gL = big_levels(I);
    for (uint32_t i = tid; i < lv_stride; i += G) lv[i] = gL[i];  // N[] of the split
    if (tid == 0) sh = S->sh;
    gsync<G>();
    const unsigned long long ncoll = build_trees<G>(key, n, M.cap, L, gl, sh, M.jarr, M.rA, M.rB, tid);
    if (!sh.overflow) level_offsets<G>(n, ncoll, M.ocap, L, sh, tid);
    for (uint32_t i = tid; i < 5u * lv_stride; i += G) gL[i] = lv[i];
    if (tid == 0) {
        S->sh = sh;
        S->ncoll = ncoll;
    }
}

// Level 1 of a large cell's first attempt, spread over kLevel1Blocks workgroups
// per cell (grid: cells x kLevel1Blocks).  Its collisions take two leaves each
// and nothing from other collisions, so each workgroup takes a contiguous share;
// outputs and finals go where the one-workgroup level loop puts them.  Each
// workgroup's sums (finals' (vx - m)^2, dummies, violations) go to the cell's
// partials, which k_big_collide adds in workgroup order.
template <typename T>
__global__ __launch_bounds__(kTT) void k_big_level1(const CellRef* __restrict__ bigs, uint32_t nb, uint32_t lv_stride)
{
    __shared__ double red[(kTT / 64) * 12 + 12];
    __shared__ uint32_t redu[(kTT / 64) * 2];
    const uint32_t b = blockIdx.x / kLevel1Blocks, w = blockIdx.x % kLevel1Blocks;
    if (b >= nb) return;
    InstDev* I = bigs[b].inst;
    const BigState* S = big_state(I);
    double* part = big_parts(I) + 4ull * w;
    const uint32_t* gL = big_levels(I);
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    const uint32_t tid = threadIdx.x;
    const bool run = !S->sh.overflow && S->sh.me >= 1u && level1_apart(I);
    const uint32_t Cl = run ? gL[2u * lv_stride + 1u] : 0u;
    const uint32_t share = (Cl + kLevel1Blocks - 1u) / kLevel1Blocks;
    const uint32_t c_begin = w * share < Cl ? w * share : Cl;
    const uint32_t c_end = c_begin + share < Cl ? c_begin + share : Cl;
    double sfin = 0.0;
    uint32_t dummies = 0, viol = 0;
    if (c_begin < c_end) {
        const uint32_t Rl = gL[lv_stride + 1u], oo = gL[3u * lv_stride + 1u];
        const uint32_t N0 = S->sh.N0, P = n - N0;
        const uint32_t fst = (uint32_t)(S->ncoll - Cl);  // level 1's collisions come last
        const double mx = S->sh.mean[0];
        const T alpha = (T)I->alpha, gT = (T)S->sh.g;
        const Key key{I->seed, I->uid, 0u, I->step};
        const gptr<const T> vx = as_global(reinterpret_cast<const T*>(I->vx[0]));
        const gptr<const T> vy = as_global(reinterpret_cast<const T*>(I->vy[0]));
        const gptr<const T> vz = as_global(reinterpret_cast<const T*>(I->vz[0]));
        CellMem<T> M;
        M.init(I, 0, 0, n);
        for (uint32_t c = c_begin + tid; c < c_end; c += kTT) {
            const uint32_t id = fst + c;
            const uint32_t sa = M.fwd[leaf_role(M.rA[id], N0, P)], sb = M.fwd[leaf_role(M.rB[id], N0, P)];
            const Vec3<T> a{vx[sa], vy[sa], vz[sa]}, bb{vx[sb], vy[sb], vz[sb]};
            T xi1, xi2, xacc;
            Draws<T>::coll(key, 1u, c, xi1, xi2, xacc);
            Vec3<T> out[2];
            if (!collide<T>(a, bb, xi1, xi2, xacc, alpha, gT, out[0], out[1], viol)) dummies++;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint32_t o = 2u * c + (uint32_t)e;
                if (o < Rl) {
                    st4(M.outv + ((uint64_t)oo + o), out[e].x, out[e].y, out[e].z, T(0));
                } else {
                    st4(M.fin + (o - Rl), out[e].x, out[e].y, out[e].z, T(0));
                    const double d = (double)out[e].x - mx;
                    sfin += d * d;
                }
            }
        }
    }
    double fs[1] = {sfin};
    gsum<kTT, 1>(fs, red);
    const uint32_t td = gsum_u32<kTT>(dummies, redu);
    const uint32_t tv = gsum_u32<kTT>(viol, redu);
    if (tid == 0) {
        part[0] = fs[0];
        part[1] = (double)td;
        part[2] = (double)tv;
        part[3] = 0.0;
    }
}

// Roles and block sums of a cell, made by its group in k_big_collide when a
// redo keeps or collides particles of a cell predicted wholly thermalized: the
// same roles as k_tile_prep's, the same block sums bit for bit as
// k_tile_bsum's (one role per thread of a 512-thread workgroup, each wave's
// butterfly sum, then the waves in order; a one-wave group takes the waves in
// turn).
template <typename T, int G>
__device__ void group_roles_bsums(InstDev* I, const Key& key, uint32_t n, const CellMem<T>& M, gptr<const T> vx,
                                  gptr<const T> vy, gptr<const T> vz, double mx, double my, double mz, uint32_t tid,
                                  double* red)
{
    tile_roles(key, n, M.role, M.fwd, 0u, n, tid, G);
    gsync<G>();  // roles and slots visible to the group
    const gptr<const uint32_t> fwd = M.fwd;
    const uint32_t nblk = (n + kRoleBlock - 1u) / kRoleBlock;
    for (uint32_t blk = 0; blk < nblk; ++blk) {
        const uint32_t b0 = blk * kRoleBlock, b1 = (b0 + kRoleBlock < n) ? b0 + kRoleBlock : n;
        double tot[5];
        if constexpr (G == kTT) {
            double sv[5] = {0, 0, 0, 0, 0};
            const uint32_t i = b0 + tid;
            if (i < b1) {
                const uint32_t sl = fwd[i];
                bsum_terms<T>(vx[sl], vy[sl], vz[sl], mx, my, mz, sv);
            }
            gsum<kTT, 5>(sv, red);
#pragma unroll
            for (int q = 0; q < 5; ++q) tot[q] = sv[q];
        } else {
            static_assert(G == 64, "a group is one wave or the whole workgroup");
#pragma unroll
            for (int q = 0; q < 5; ++q) tot[q] = 0.0;
            for (uint32_t w = 0; w < (uint32_t)(kTT / 64); ++w) {
                double sv[5] = {0, 0, 0, 0, 0};
                const uint32_t i = b0 + w * 64u + tid;
                if (i < b1) {
                    const uint32_t sl = fwd[i];
                    bsum_terms<T>(vx[sl], vy[sl], vz[sl], mx, my, mz, sv);
                }
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    double a = sv[q];
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
                    tot[q] += __shfl(a, 0);
                }
            }
        }
        if (tid == 0) {
            double* p = I->bsum + 8ull * blk;
#pragma unroll
            for (int q = 0; q < 5; ++q) p[q] = tot[q];
        }
    }
    gsync<G>();  // block sums visible
}

template <typename T, int G>
__global__ __launch_bounds__(kTT) void k_big_collide(const CellRef* __restrict__ bigs, uint32_t lv_stride,
                                                     CellLists cl)
{
    extern __shared__ uint32_t lds_levels[];
    __shared__ GroupLds<G> glds[kTT / G];
    uint32_t b;
    if (!pick_cell<G>(cl, b)) return;
    const uint32_t grp = threadIdx.x / G, tid = threadIdx.x % G;
    GroupLds<G>& gl = glds[grp];
    CellShared& sh = gl.sh;
    InstDev* I = bigs[b].inst;
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    BigState* S = big_state(I);
    uint32_t* gL = big_levels(I);
    uint32_t* lv = lds_levels + (size_t)grp * 5u * lv_stride;
    for (uint32_t i = tid; i < 5u * lv_stride; i += G) lv[i] = gL[i];
    if (tid == 0) sh = S->sh;
    gsync<G>();
    CellStats* st = I->stats;
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
    const Key key{I->seed, I->uid, 0u, I->step};
    const gptr<const T> vx = as_global(uni(reinterpret_cast<const T*>(I->vx[0])));
    const gptr<const T> vy = as_global(uni(reinterpret_cast<const T*>(I->vy[0])));
    const gptr<const T> vz = as_global(uni(reinterpret_cast<const T*>(I->vz[0])));
    CellMem<T> M;
    M.init(I, 0, 0, n);
    Levels L = levels_at(lv, lv_stride);
    const double mx = sh.mean[0], my = sh.mean[1], mz = sh.mean[2];
    const T alpha = (T)I->alpha;
    const T gT = (T)sh.g;
    unsigned long long ncoll = S->ncoll;
    bool first = true;  // the first attempt's level 1 was made by k_big_level1
    bool roles_made = S->roles != ROLES_NONE;
    for (;;) {
        // sums of the unchanged and thermalized sets of this attempt
        const uint32_t N0 = sh.N0, R0 = sh.R0, P = n - N0;
        const uint32_t kept_end = N0 - sh.borrowed, leaf_end = N0 + (R0 < P ? R0 : P);
        double all[7];
        if (leaf_end == 0u) {
            // every particle thermalized: the whole cell's sums (k_big_split)
            all[0] = 0.0;
            all[1] = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) all[2 + q] = sh.all_th[q];
        } else {
            if (!roles_made) {
                group_roles_bsums<T, G>(I, key, n, M, vx, vy, vz, mx, my, mz, tid, gl.red);
                roles_made = true;
            }
            attempt_sums<T, G>(vx, vy, vz, M.fwd, I->bsum, n, kept_end, leaf_end, mx, my, mz, tid, gl.red, all);
        }
        uint32_t dummies = 0, viol = 0;
        double sfin = 0.0;
        // the majorant raised level by level (Remark 4.1), from the step's bound
        DynMajorant dmj{gl.red, I->alpha, sh.d2max0, sh.g};
        const bool dyn = uni(I->majorant) == MAJ_LEVEL && I->alpha != 0.0;
        const bool apart = first && level1_apart(I);
        bottom_up<T, G, true>(key, n, vx, vy, vz, L, sh, M, ncoll, alpha, gT, mx, tid, dummies, viol, sfin, 0u,
                              nullptr, 0u, nullptr, T(0), dyn ? &dmj : nullptr, apart ? 2u : 1u);
        if (tid == 0) sh.g_last = dmj.g;
        double fs[1] = {sfin};
        gsum<G, 1>(fs, gl.red);
        uint32_t td = gsum_u32<G>(dummies, gl.redu);
        uint32_t tv = gsum_u32<G>(viol, gl.redu);
        if (tid == 0) {
            if (apart) {
                // level 1's sums, in workgroup order
                const double* part = big_parts(I);
                for (uint32_t w = 0; w < kLevel1Blocks; ++w) {
                    fs[0] += part[4u * w];
                    td += (uint32_t)part[4u * w + 1u];
                    tv += (uint32_t)part[4u * w + 2u];
                }
            }
            all[6] = fs[0];
            sh.dummies = td;
            sh.viol = tv;
            decide(I, 0, n, all, mx, my, mz, sh);
        }
        first = false;
        gsync<G>();
        if (sh.decision) break;
        // redo at depth sh.m
        split_levels<G>(key, n, sh.q, L, sh, tid, adaptive_look(I));
        ncoll = build_trees<G>(key, n, M.cap, L, gl, sh, M.jarr, M.rA, M.rB, tid);
        if (sh.overflow || !level_offsets<G>(n, ncoll, M.ocap, L, sh, tid)) break;
    }
    if (tid == 0) {
        if (sh.overflow) {
            CellStats s{};
            s.n = n;
            s.status = CELL_OVERFLOW;
            s.m_used = sh.m;
            *st = s;
            atomicOr(I->error, CELL_OVERFLOW);
        } else {
            write_stats(st, n, sh);
        }
        S->sh = sh;
    }
}

template <typename T>
__global__ __launch_bounds__(kTT) void k_tile_zsum(const CellRef* __restrict__ bigs,
                                                   const uint32_t* __restrict__ prefix, uint32_t nb)
{
    __shared__ double t_red[(kTT / 64) * 8];
    uint32_t b, k;
    tile_of(prefix, nb, blockIdx.x, b, k);
    InstDev* I = bigs[b].inst;
    const BigState* S = big_state(I);
    const uint32_t n_th = S->sh.n_th;
    if (S->sh.overflow || n_th < 2) return;
    const uint32_t n = I->cell_off[1] - I->cell_off[0];
    const uint32_t N0 = S->sh.N0, R0 = S->sh.R0, P = n - N0;
    const uint32_t leaf_end = N0 + (R0 < P ? R0 : P);
    const uint32_t s_begin = k * kTile, s_end = (s_begin + kTile < n) ? s_begin + kTile : n;
    const Key key{I->seed, I->uid, 0u, I->step};
    CellMem<T> M;
    M.init(I, 0, 0, n);
    double zs[4] = {0, 0, 0, 0};
    for (uint32_t s = s_begin + threadIdx.x; s < s_end; s += kTT) {
        if (leaf_end != 0u && M.role[s] < leaf_end) continue;  // (every slot thermalized: no roles read)
        const Vec3<T> z = Draws<T>::normals(key, s);  // keyed by the slot
        const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
        zs[0] += zx;
        zs[1] += zy;
        zs[2] += zz;
        zs[3] += zx * zx + zy * zy + zz * zz;
    }
    gsum<kTT, 4>(zs, t_red);
    if (threadIdx.x == 0) {
        double* tp = I->tpart + 8ull * k;
        for (int q = 0; q < 4; ++q) tp[q] = zs[q];
    }
}

template <typename T>
__global__ __launch_bounds__(kTT) void k_tile_write(const CellRef* __restrict__ bigs,
                                                    const uint32_t* __restrict__ prefix, uint32_t nb)
{
    uint32_t b, k;
    tile_of(prefix, nb, blockIdx.x, b, k);
    CellView<T> V(bigs[b].inst);
    const uint32_t n = V.n;
    const BigState* S = big_state(V.I);
    if (S->sh.overflow) return;
    const uint32_t N0 = S->sh.N0, R0 = S->sh.R0, P = n - N0, n_th = S->sh.n_th;
    const uint32_t kept_end = N0 - S->sh.borrowed, leaf_end = N0 + (R0 < P ? R0 : P);
    __shared__ double par[7];  // a, zbar (3), ur (3)
    if (threadIdx.x == 0 && n_th >= 2) {
        const uint32_t ntz = (n + kTile - 1) / kTile;
        double z[4] = {0, 0, 0, 0};
        for (uint32_t t = 0; t < ntz; ++t)
            for (int q = 0; q < 4; ++q) z[q] += V.I->tpart[8ull * t + q];
        const double nt = (double)n_th;
        const double zb0 = z[0] / nt, zb1 = z[1] / nt, zb2 = z[2] / nt;
        const double Z = z[3] - nt * (zb0 * zb0 + zb1 * zb1 + zb2 * zb2);
        par[0] = Z > 0.0 ? sqrt(S->sh.a_th / Z) : 0.0;
        par[1] = zb0;
        par[2] = zb1;
        par[3] = zb2;
        par[4] = S->sh.ur[0];
        par[5] = S->sh.ur[1];
        par[6] = S->sh.ur[2];
    }
    __syncthreads();
    const bool thermalize = n_th >= 2;
    const double a = thermalize ? par[0] : 0.0;
    const double z0 = thermalize ? par[1] : 0.0, z1 = thermalize ? par[2] : 0.0, z2 = thermalize ? par[3] : 0.0;
    const double u0 = thermalize ? par[4] : 0.0, u1 = thermalize ? par[5] : 0.0, u2 = thermalize ? par[6] : 0.0;
    const Key key{V.I->seed, V.I->uid, 0u, V.I->step};
    CellMem<T> M;
    M.init(V.I, 0, 0, n);
    const uint32_t s_begin = k * kTile, s_end = (s_begin + kTile < n) ? s_begin + kTile : n;
    constexpr int U = 4;
    for (uint32_t s0 = s_begin + threadIdx.x; s0 < s_end; s0 += kTT * U) {
        uint32_t ro[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = s0 + u * kTT;
            ro[u] = (i < s_end && leaf_end != 0u) ? M.role[i] : 0u;  // (leaf_end 0: every slot thermalized)
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t s = s0 + u * kTT;
            const uint32_t i = ro[u];
            if (s >= s_end || i < kept_end) continue;
            if (i < leaf_end) {
                const uint32_t r = leaf_rank(i, N0, P);  // final r goes to the slot of leaf r
                const Vec3<T> f = ld3(M.fin + r);
                V.vx[s] = f.x;
                V.vy[s] = f.y;
                V.vz[s] = f.z;
            } else if (thermalize) {
                const Vec3<T> z = Draws<T>::normals(key, s);
                V.vx[s] = (T)(u0 + a * ((double)z.x - z0));
                V.vy[s] = (T)(u1 + a * ((double)z.y - z1));
                V.vz[s] = (T)(u2 + a * ((double)z.z - z2));
            }
        }
    }
}

#define TRMC_TILED_INSTANTIATE(T)                                                              \
    template __global__ void k_tile_prep<T>(const CellRef*, const uint32_t*, uint32_t, uint32_t*); \
    template __global__ void k_tile_bsum<T, false>(const CellRef*, const uint32_t*, uint32_t); \
    template __global__ void k_tile_bsum<T, true>(const CellRef*, const uint32_t*, uint32_t);  \
    template __global__ void k_tile_roles<T>(const CellRef*, const uint32_t*, uint32_t);       \
    template __global__ void k_big_split<T>(const CellRef*, uint32_t, uint32_t, CellLists);    \
    template __global__ void k_big_tree<T, 64>(const CellRef*, uint32_t, CellLists);           \
    template __global__ void k_big_tree<T, kTT>(const CellRef*, uint32_t, CellLists);          \
    template __global__ void k_big_level1<T>(const CellRef*, uint32_t, uint32_t);               \
    template __global__ void k_big_collide<T, 64>(const CellRef*, uint32_t, CellLists);        \
    template __global__ void k_big_collide<T, kTT>(const CellRef*, uint32_t, CellLists);       \
    template __global__ void k_tile_zsum<T>(const CellRef*, const uint32_t*, uint32_t);        \
    template __global__ void k_tile_write<T>(const CellRef*, const uint32_t*, uint32_t);
TRMC_TILED_INSTANTIATE(float)
TRMC_TILED_INSTANTIATE(double)

}  // namespace trmc
