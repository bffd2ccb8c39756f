// k_collide.hip -- the per-cell TRMC-R collision step (Trazzi, Pareschi and
// Wennberg, Sec. 4) with the whole cell in one group of G threads: the whole
// workgroup (G = 512) or one wave (G = 64, eight cells per workgroup, no
// workgroup barriers); one launch serves both.  Used for slab cells and small
// homogeneous cells; large homogeneous cells take the tiled pipeline.
//
// Per cell and step, in order:
//   1. FP64 moments of the cell: mean, S = P_xx, and for VHS dv = max|v - mean|
//      (Sec. 4.2); the role index of every slot (inverse of a keyed permutation:
//      unchanged, leaf of a collision tree, or thermalized).
//   2. g = (2 dv)^alpha on a 20-bit grid, mu = rho_c g, q = exp(-mu dt/eps) (Sec. 3.2).
//   3. Attempts at depth m (Sec. 4.3 redoes a rejected attempt at 2m):
//      split (Alg. 4.2), collision trees in level order with stable request ranks
//      (Alg. 4.3), leaves and sums of the unchanged / thermalized sets,
//      collisions level by level (eq. Maxwell_coll-r, eq. n3d-r, Alg. 4.4),
//      adaptive test with the analytic Maxwellian part.
//   4. Maxwellian remainder: Box-Muller normals written in place, then affinely
//      rescaled to the removed particles' momentum and energy; leaves take the finals.
#include <hip/hip_runtime.h>

#include "collide_core.h"

namespace trmc {

#ifdef TRMC_PHASE_TIMING
// Profiling build only: per-phase wall-clock totals by cell-size class.
__device__ unsigned long long g_phase[4][12];
__device__ unsigned long long g_maxcell[12];
// per workgroup of a launch (at most 16384): first start and last end of its groups' steps
__device__ unsigned long long g_span[16384][2];
#define TRMC_PHASE_BEGIN() unsigned long long ph_t = wall_clock64(), ph_acc[10] = {0,0,0,0,0,0,0,0,0,0}
#define TRMC_PHASE(k)                                   \
    do {                                                \
        const unsigned long long ph_n = wall_clock64(); \
        ph_acc[k] += ph_n - ph_t;                       \
        ph_t = ph_n;                                    \
    } while (0)
#define TRMC_PHASE_END(nn)                                                        \
    do {                                                                          \
        if (tid == 0) {                                                           \
            const int cls = (nn) < 4096u ? 0 : ((nn) < 16384u ? 1 : 2);           \
            unsigned long long tot = 0;                                           \
            for (int k = 0; k < 10; ++k) {                                        \
                atomicAdd(&g_phase[cls][k], ph_acc[k]);                           \
                tot += ph_acc[k];                                                 \
            }                                                                     \
            atomicAdd(&g_phase[cls][10], 1ull);                                   \
            const unsigned long long prev = atomicMax(&g_phase[3][cls], tot);     \
            if (tot > prev && cls == 2) {                                         \
                for (int k = 0; k < 8; ++k) g_maxcell[k] = ph_acc[k];             \
                g_maxcell[8] = (nn);                                              \
                g_maxcell[9] = sh.attempts;                                       \
                g_maxcell[10] = sh.m;                                             \
                g_maxcell[11] = sh.me;                                            \
            }                                                                     \
        }                                                                         \
    } while (0)
#else
#define TRMC_PHASE_BEGIN() \
    do {                   \
    } while (0)
#define TRMC_PHASE(k) \
    do {              \
    } while (0)
#define TRMC_PHASE_END(nn) \
    do {                   \
    } while (0)
#endif

#ifndef TRMC_SLOT_UNROLL
#define TRMC_SLOT_UNROLL 2
#endif
#ifndef TRMC_SLOT_UNROLL_WAVE
#define TRMC_SLOT_UNROLL_WAVE 4
#endif
#ifndef TRMC_WRITE_UNROLL_WAVE
#define TRMC_WRITE_UNROLL_WAVE 8
#endif
#ifndef TRMC_WRITE_UNROLL
#define TRMC_WRITE_UNROLL 4
#endif
#ifndef TRMC_MAJ_BRACKET
#define TRMC_MAJ_BRACKET 1
#endif
constexpr bool kMajBracket = TRMC_MAJ_BRACKET != 0;  // the majorant bracket of workgroup cells
#ifndef TRMC_LAZY_ROLES
#define TRMC_LAZY_ROLES 1
#endif
constexpr bool kLazyRoles = TRMC_LAZY_ROLES != 0;  // roles made after the split for cells predicted all-thermalized
#ifndef TRMC_FAST_THERMAL
#define TRMC_FAST_THERMAL 1
#endif
constexpr bool kFastThermal = TRMC_FAST_THERMAL != 0 && kLazyRoles;  // sums of wholly thermalized cells in the moments pass
#ifndef TRMC_PREFETCH_ROLES
#define TRMC_PREFETCH_ROLES 1
#endif
constexpr bool kPrefetchRoles = TRMC_PREFETCH_ROLES != 0;  // next batch's roles loaded ahead in the slot passes
#ifndef TRMC_ROLES16
#define TRMC_ROLES16 1
#endif
constexpr bool kRoles16 = TRMC_ROLES16 != 0;  // 16-bit roles for cells of at most 65536 particles
constexpr int kUnroll = TRMC_SLOT_UNROLL;  // slots per thread per batch in the moment and normal passes

// LDS of the groups of a whole-cell workgroup (one group of the workgroup's
// size, or one per wave), shared by every instance of the step function: a
// workgroup runs one kind of group, each group one cell, one step at a time.
// One buffer instead of one per instance keeps the static LDS of the kernel to
// the largest kind.
constexpr size_t kGroupLdsBytes = sizeof(GroupLds<kCollideThreads>) > kSmallPerBlock * sizeof(GroupLds<64>)
                                      ? sizeof(GroupLds<kCollideThreads>)
                                      : kSmallPerBlock * sizeof(GroupLds<64>);
__shared__ __attribute__((aligned(16))) unsigned char g_group_lds[kGroupLdsBytes];

// One step of the cell of group blk / NGRP.  Kept out of line: the kernels call
// it once per step, and inlined into their step loops the compiler keeps
// per-step values live across the whole loop and spills them.
template <typename T, int NT, int G, bool WB = false, bool REUSE = false, bool DYN = false, typename R = uint32_t>
__device__ __attribute__((noinline)) void collide_cells(const CellRef* __restrict__ work, uint32_t n_work, uint32_t blk,
                                              uint32_t lv_stride, uint32_t soff)
{
    constexpr int NGRP = NT / G;  // groups per workgroup
    static_assert(NGRP * sizeof(GroupLds<G>) <= kGroupLdsBytes, "group LDS exceeds the shared buffer");
    // slots per thread per batch of the slot passes: a one-wave group keeps more loads in flight
    constexpr int kU = G == 64 ? TRMC_SLOT_UNROLL_WAVE : kUnroll;
    extern __shared__ uint32_t lds_levels[];
    GroupLds<G>* const glds = reinterpret_cast<GroupLds<G>*>(g_group_lds);

    const uint32_t grp = uni((uint32_t)(threadIdx.x / G));
    const uint32_t wi = blk * NGRP + grp;
    if (wi >= n_work) return;  // whole group leaves together
    GroupLds<G>& gl = glds[grp];
    CellShared& sh = gl.sh;
    const uint32_t tid = threadIdx.x % G;
    // everything about the cell is wave-uniform: keep it in scalar registers
    InstDev* __restrict__ I = uni(work[wi].inst);
    const uint32_t cell = uni(work[wi].cell);
    const uint32_t off = uni(I->cell_off[cell]);
    const uint32_t n = uni(I->cell_off[cell + 1]) - off;
    const uint32_t buf = (uni(I->geometry) == GEOM_SLAB) ? (uni(I->cur) ^ 1u) : 0u;
    const gptr<T> vx = as_global(uni(reinterpret_cast<T*>(I->vx[buf]) + off));
    const gptr<T> vy = as_global(uni(reinterpret_cast<T*>(I->vy[buf]) + off));
    const gptr<T> vz = as_global(uni(reinterpret_cast<T*>(I->vz[buf]) + off));
    CellStats* st = I->stats + cell;
    const Key key = uni(Key{I->seed, I->uid, cell, I->step + soff});  // step soff of this launch
    const uint64_t t_begin = wall_clock64();  // the step's duration orders the next launch

#ifndef TRMC_PRIO_CELL
#define TRMC_PRIO_CELL 16384u
#endif
    // the largest cells carry the longest dependent chains of the launch: their
    // waves take issue priority over the small cells sharing their compute unit
    if (n >= TRMC_PRIO_CELL) __builtin_amdgcn_s_setprio(2);
    if (n < 2) {
        if (tid == 0) {
            CellStats s{};  // skipped: no attempt, no draws
            s.n = n;
            *st = s;
        }
        return;
    }
    CellMem<T, R> M;
    M.init(I, off, cell, n);
    Levels L = levels_at(lds_levels + (size_t)grp * 5u * lv_stride, lv_stride);

    // Roles: each wave takes a contiguous share of the slots, its lanes refilled
    // as their cycle walks end (the walks vary in length).
    auto make_roles = [&]() {
        const uint4 pk = draw(key, 0, TAG_PERM, 0);
        const uint32_t pbits = perm_bits(n);
        constexpr uint32_t NW = G / 64;
        const uint32_t w = tid >> 6;
        const uint32_t share = (n + NW - 1u) / NW;
        const uint32_t r0 = w * share, r1 = r0 + share < n ? r0 + share : n;
        if (r0 < r1) roles_by_wave(M.role, r0, r1, n, pbits, pk);
    };
    // A cell whose previous step thermalized every particle (small eps) most
    // likely does so again: its roles are not made up front.  An attempt that
    // keeps or collides any particle makes them after its split; while none
    // has, every slot is thermalized and the slot passes read no roles (they
    // visit the same slots in the same order as with roles).
    bool roles_ready = true;
    if constexpr (kLazyRoles && !WB && !REUSE) {
        // the cell's record of its last step (this group's own previous step in a
        // fused launch: ordered by the group barrier between the steps)
        const bool all_th = st->n == n && st->N0 == 0u && st->n_th == n && st->status == 0u;
        roles_ready = !uni((uint32_t)all_th);
    }

    // Such a cell also sums, in the moments pass, the Maxwellian normals of its
    // slots (sum of z, of |z|^2; the same slots in the same order as the normal
    // pass): when its attempt does thermalize every particle, the normal pass is
    // not made.  Every cell's moments pass sums its velocities about the first
    // particle's (c), so that an attempt that thermalizes every particle takes
    // the removed set's sums from there instead of a gather pass; together,
    // two passes over the slots instead of four.  None of this depends on the
    // prediction: only whether the normals are summed early does.
    const bool fast = kFastThermal && !roles_ready;

    TRMC_PHASE_BEGIN();
    // ---- 1-2. moments, roles, parameters of the step ------------------------
    {
        const double c0 = (double)vx[0];  // shift for the one-pass P_xx
        const double c1 = (double)vy[0], c2 = (double)vz[0];
        // sums of v_x - c0, v_y, v_z, (v_x - c0)^2, (v_y - c1)^2, (v_z - c2)^2
        double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // VHS cells of a workgroup: the largest distance to the previous step's
        // mean (this group's last step of the cell, else the cell's record from
        // the last launch) brackets the majorant; the exact pass below runs only
        // when the bracket does not settle it.  Collisions conserve momentum, so
        // the two means differ by rounding only.
        const bool bk = kMajBracket && !DYN && G > 64 && uni((uint64_t)__double_as_longlong(I->alpha)) != 0ull;
        double bc0 = 0.0, bc1 = 0.0, bc2 = 0.0, d2c = 0.0;
        double zt[4] = {0, 0, 0, 0};  // this thread's sums of the normals (fast), then the group's
        if (bk) {
            bc0 = soff > 0 ? sh.mean[0] : st->mean[0];
            bc1 = soff > 0 ? sh.mean[1] : st->mean[1];
            bc2 = soff > 0 ? sh.mean[2] : st->mean[2];
        }
        // loads of the next batch are issued before the current batch is summed
        T ax[kU], ay[kU], az[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = tid + u * G;
            const bool ok = i < n;
            ax[u] = ok ? vx[i] : T(0);
            ay[u] = ok ? vy[i] : T(0);
            az[u] = ok ? vz[i] : T(0);
        }
        for (uint32_t s0 = tid; s0 < n; s0 += G * kU) {
            T bx[kU], by[kU], bz[kU];
            const uint32_t s1 = s0 + G * kU;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = s1 + u * G;
                const bool ok = i < n;
                bx[u] = ok ? vx[i] : T(0);
                by[u] = ok ? vy[i] : T(0);
                bz[u] = ok ? vz[i] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = s0 + u * G;
                if (i < n) {
                    const double dx = (double)ax[u] - c0;
                    s[0] += dx;
                    s[1] += (double)ay[u];
                    s[2] += (double)az[u];
                    s[3] += dx * dx;
                    const double dy = (double)ay[u] - c1, dz = (double)az[u] - c2;
                    s[4] += dy * dy;
                    s[5] += dz * dz;
                    if (bk) {
                        const double ex = (double)ax[u] - bc0, ey = (double)ay[u] - bc1, ez = (double)az[u] - bc2;
                        const double e2 = ex * ex + ey * ey + ez * ez;
                        d2c = e2 > d2c ? e2 : d2c;
                    }
                    if (fast) {
                        const Vec3<T> z = Draws<T>::normals(key, i);  // keyed by the slot
                        const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
                        zt[0] += zx;
                        zt[1] += zy;
                        zt[2] += zz;
                        zt[3] += zx * zx + zy * zy + zz * zz;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                ax[u] = bx[u];
                ay[u] = by[u];
                az[u] = bz[u];
            }
        }
        if (roles_ready) make_roles();
        gsum<G, 6>(s, gl.red);
        if (fast) {
            gsum<G, 4>(zt, gl.red);
            if (tid == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) sh.zt[q] = zt[q];
            }
        }
        const double inv = 1.0 / (double)n;
        const double dxm = s[0] * inv;
        const double mx = c0 + dxm, my = s[1] * inv, mz = s[2] * inv;
        if (tid == 0) {
            // the sums of the whole cell about its mean, for an attempt that
            // thermalizes every particle: sum of v - m (rounding only) and of |v - m|^2
            const double nd = (double)n, ey = my - c1, ez = mz - c2;
            sh.all_th[0] = s[0] - nd * dxm;
            sh.all_th[1] = s[1] - nd * my;
            sh.all_th[2] = s[2] - nd * mz;
            sh.all_th[3] = (s[3] - nd * dxm * dxm) + (s[4] - nd * ey * ey) + (s[5] - nd * ez * ez);
        }
        double dmax = 0.0;
        if (bk) {
            // every thread reduces the same values in the same order: a uniform verdict
            const double d2 = gmax<G>(d2c, gl.red);
            const double ex = mx - bc0, ey = my - bc1, ez = mz - bc2;
            dmax = majorant_bracket(I->alpha, d2, sqrt(ex * ex + ey * ey + ez * ez));
        }
        if (uni((uint64_t)__double_as_longlong(I->alpha)) != 0ull && !(dmax >= 0.0 && bk)) {
            // two batches of loads in flight: the next batch is issued before
            // the current one is reduced
            double d2max = 0.0;
            T ax2[kU], ay2[kU], az2[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = tid + u * G;
                const bool ok = i < n;
                ax2[u] = ok ? vx[i] : T(0);
                ay2[u] = ok ? vy[i] : T(0);
                az2[u] = ok ? vz[i] : T(0);
            }
            for (uint32_t s0 = tid; s0 < n; s0 += G * kU) {
                T bx[kU], by[kU], bz[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const uint32_t i = s0 + G * kU + u * G;
                    const bool ok = i < n;
                    bx[u] = ok ? vx[i] : T(0);
                    by[u] = ok ? vy[i] : T(0);
                    bz[u] = ok ? vz[i] : T(0);
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (s0 + u * G < n) {
                        const double dx = (double)ax2[u] - mx, dy = (double)ay2[u] - my, dz = (double)az2[u] - mz;
                        const double d2 = dx * dx + dy * dy + dz * dz;
                        d2max = d2 > d2max ? d2 : d2max;
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    ax2[u] = bx[u];
                    ay2[u] = by[u];
                    az2[u] = bz[u];
                }
            }
            dmax = gmax<G>(d2max, gl.red);
        }
        if (tid == 0) {
            sh.mean[0] = mx;
            sh.mean[1] = my;
            sh.mean[2] = mz;
            const double sn = s[3] * inv - dxm * dxm;
            sh.Sn = sn > 0.0 ? sn : 0.0;
            cell_params(I, cell, n, dmax, sh);
        }
        gsync<G>();
    }
    TRMC_PHASE(0);

    const double mx = uni(sh.mean[0]), my = uni(sh.mean[1]), mz = uni(sh.mean[2]);
    const T alpha = (T)I->alpha;
    const T gT = (T)sh.g;

    // ---- 3. attempts ------------------------------------------------------------
    // A redo keeps the unchanged set when no leaf is borrowed.  The first redo
    // copies the whole pool (roles from N0 on) in rank order; later redos sum
    // their thermalized set (ranks R0 .. P of the pool) from that copy.
    uint32_t leaves_done = 0;  // leaf ranks [0, leaves_done) are gathered
    uint32_t attempt = 0;
    bool pooled = false;
    // Reuse of rejected attempts (adaptive depth, Sec. 4.3): levels 1..mprev are
    // done, coff[l] counts level l's collisions so far (the draw offset of the
    // next ones), leaf and final ranks continue from r0prev.
    [[maybe_unused]] uint32_t* const coff =
        REUSE ? lds_levels + (size_t)NGRP * 5u * lv_stride + (size_t)grp * lv_stride : nullptr;
    [[maybe_unused]] uint32_t r0prev = 0, mprev = 0, folds_acc = 0, dum_acc = 0, viol_acc = 0;
    [[maybe_unused]] unsigned long long coll_acc = 0;
    [[maybe_unused]] double sfin_acc = 0.0;
    if constexpr (REUSE) {
        for (uint32_t l = tid; l < lv_stride; l += G) coff[l] = 0;  // visible after the split's barrier
    }
    for (;;) {
        [[maybe_unused]] const uint32_t m_att = REUSE ? uni(sh.m) : 0u;
        split_levels<G>(key, n, sh.q, L, sh, tid, adaptive_look(I));
        if constexpr (REUSE) {
            if (mprev) {
                const uint32_t me0 = uni(sh.me);
                for (uint32_t l = 1 + tid; l <= mprev && l <= me0; l += G) L.N[l] = 0;  // made earlier
                gsync_lds<G>();
            }
        }
        TRMC_PHASE(1);
        const unsigned long long ncoll =
            build_trees<G, REUSE>(key, n, M.cap, L, gl, sh, M.jarr, M.rA, M.rB, tid, coff, r0prev, mprev);
        TRMC_PHASE(2);
        if (sh.overflow) break;
        if constexpr (REUSE) {
            if (tid == 0) sh.R0 += r0prev;  // leaves of all attempts
            gsync_lds<G>();
        }
        if (!level_offsets<G>(n, ncoll, M.ocap, L, sh, tid)) break;

        const uint32_t N0 = sh.N0, R0 = sh.R0, P = n - N0;
        const uint32_t kept_end = N0 - sh.borrowed, leaf_end = N0 + (R0 < P ? R0 : P);
        if (!roles_ready && leaf_end != 0u) {
            make_roles();
            gsync<G>();  // roles visible to the gather
            roles_ready = true;
        }
        double sums[6] = {0, 0, 0, 0, 0, 0};
        const bool no_borrow = R0 <= P;
        if (pooled && no_borrow) {
            for (uint32_t r = R0 + tid; r < P; r += G) {
                const Vec3<T> v = ld3(M.leaf + r);
                const double dx = (double)v.x - mx, dy = (double)v.y - my, dz = (double)v.z - mz;
                sums[1] += dx * dx;
                sums[2] += dx;
                sums[3] += dy;
                sums[4] += dz;
                sums[5] += dx * dx + dy * dy + dz * dz;
            }
            if (tid == 0) sums[0] = sh.kept0;
        } else {
            // (an attempt without roles keeps no pool: its slots' ranks are not known)
            const bool whole = kFastThermal && !WB && !REUSE && leaf_end == 0u;
            const bool pool_all = attempt > 0 && no_borrow && roles_ready && !whole;
            if (whole) {
                // every slot thermalized: the whole cell's sums from the moments pass
                if (tid == 0) {
                    sums[2] = sh.all_th[0];
                    sums[3] = sh.all_th[1];
                    sums[4] = sh.all_th[2];
                    sums[5] = sh.all_th[3];
                }
            } else if (roles_ready)
                gather_sets<T, G, false, R>(vx, vy, vz, M.role, M.leaf, n, N0, 0u, n, kept_end, leaf_end,
                                            leaves_done, pool_all, mx, my, mz, tid, sums);
            else
                gather_sets<T, G, true, R>(vx, vy, vz, M.role, M.leaf, n, N0, 0u, n, kept_end, leaf_end,
                                           leaves_done, pool_all, mx, my, mz, tid, sums);
            leaves_done = pool_all ? P : (R0 > leaves_done ? R0 : leaves_done);
            pooled = pool_all;
        }
        ++attempt;
        gsync<G>();  // leaves visible
        TRMC_PHASE(3);

        uint32_t dummies = 0, viol = 0;
        double sfin = 0.0;
        [[maybe_unused]] WbAcc wba{};
        // the majorant raised level by level (Remark 4.1), from the step's bound
        DynMajorant dmj{gl.red, I->alpha, sh.d2max0, sh.g};
        const bool dyn = DYN && I->alpha != 0.0;
        bottom_up<T, G, false, WB, REUSE, R>(key, n, vx, vy, vz, L, sh, M, ncoll, alpha, gT, mx, tid, dummies, viol,
                                          sfin, WB ? uni(I->wb) : 0u, coff, r0prev, &wba,
                                          WB ? (T)uni(I->wb_mmax) : T(0), dyn ? &dmj : nullptr);
        if (tid == 0) sh.g_last = dmj.g;
        if constexpr (WB) {
            double v[9] = {wba.z[0], wba.z[1], wba.z[2], wba.z[3], wba.d[0], wba.d[1], wba.d[2], wba.d[3], wba.cnt};
            gsum<G, 9>(v, gl.red);
            if (tid == 0)
                for (int q = 0; q < 9; ++q) sh.wbz[q] = v[q];
        }
        TRMC_PHASE(4);
        if constexpr (REUSE) {
            sfin_acc += sfin;  // the finals of every attempt enter S
            sfin = sfin_acc;
        }

        double all[7] = {sums[0], sums[1], sums[2], sums[3], sums[4], sums[5], sfin};
        gsum<G, 7>(all, gl.red);
        const uint32_t td = gsum_u32<G>(dummies, gl.redu);
        const uint32_t tv = gsum_u32<G>(viol, gl.redu);
        if (tid == 0) {
            if constexpr (WB) {
                sh.rs[0] = all[2];
                sh.rs[1] = all[3];
                sh.rs[2] = all[4];
                sh.rs[3] = all[5];
            }
            sh.kept0 = all[0];
            sh.dummies = td;
            sh.viol = tv;
            if constexpr (REUSE) {
                sh.dummies += dum_acc;
                sh.viol += viol_acc;
                sh.ncoll += coll_acc;
                sh.folds += folds_acc;
            }
            decide(I, cell, n, all, mx, my, mz, sh);
        }
        gsync<G>();
        TRMC_PHASE(5);
        if (sh.decision) break;
        if constexpr (REUSE) {
            // keep this attempt: the next one builds on top of it
            const uint32_t me_a = uni(sh.me);
            for (uint32_t l = 1 + tid; l <= me_a; l += G) coff[l] += L.C[l];
            r0prev = uni(sh.R0);
            mprev = m_att;
            coll_acc = uni((uint64_t)sh.ncoll);
            folds_acc = uni(sh.folds);
            dum_acc = uni(sh.dummies);
            viol_acc = uni(sh.viol);
            gsync_lds<G>();
        }
    }

    if (sh.overflow) {
        if (tid == 0) {
            CellStats s{};
            s.n = n;
            s.status = CELL_OVERFLOW;
            s.m_used = sh.m;
            s.ticks = elapsed_ticks(t_begin);
            *st = s;
            atomicOr(I->error, CELL_OVERFLOW);
        }
        return;
    }

    // ---- 4. Maxwellian remainder and write-back ------------------------------
    const uint32_t N0 = sh.N0, R0 = sh.R0, P = n - N0;
    const uint32_t kept_end = N0 - sh.borrowed, leaf_end = N0 + (R0 < P ? R0 : P);
    [[maybe_unused]] const T wb_max = WB ? (T)uni(I->wb_mmax) : T(0);
    if constexpr (WB) {
        // tree-shape truncation (Sec. 4.4): finals longer than m_max join the
        // remainder; their dropped values join the removed set of the rescale.
        // The collision pass summed the dropped finals and their slots' normals
        // (sh.wbz); here the normals of the split remainder's slots.
        double zs[4] = {0, 0, 0, 0};
        for (uint32_t s = tid; s < n; s += G) {
            if (M.role[s] >= leaf_end) {
                const Vec3<T> z = Draws<T>::normals(key, s);  // keyed by the slot
                const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
                zs[0] += zx;
                zs[1] += zy;
                zs[2] += zz;
                zs[3] += zx * zx + zy * zy + zz * zz;
            }
        }
        gsum<G, 4>(zs, gl.red);
        if (tid == 0) {
            for (int q = 0; q < 4; ++q) zs[q] += sh.wbz[q];
            const double zs4 = sh.wbz[4], zs5 = sh.wbz[5], zs6 = sh.wbz[6], zs7 = sh.wbz[7];
            const uint32_t n_wb = (uint32_t)sh.wbz[8];
            const uint32_t total = sh.n_th + n_wb;
            sh.wb_th = n_wb;
            sh.n_th = total;
            if (total >= 2) {
                const double nt = (double)total;
                const double d0 = (sh.rs[0] + zs4) / nt, d1 = (sh.rs[1] + zs5) / nt, d2 = (sh.rs[2] + zs6) / nt;
                sh.ur[0] = mx + d0;
                sh.ur[1] = my + d1;
                sh.ur[2] = mz + d2;
                double E = (sh.rs[3] + zs7) - nt * (d0 * d0 + d1 * d1 + d2 * d2);
                E = E > 0.0 ? E : 0.0;
                const double zb0 = zs[0] / nt, zb1 = zs[1] / nt, zb2 = zs[2] / nt;
                const double Z = zs[3] - nt * (zb0 * zb0 + zb1 * zb1 + zb2 * zb2);
                sh.zbar[0] = zb0;
                sh.zbar[1] = zb1;
                sh.zbar[2] = zb2;
                sh.a_th = Z > 0.0 ? sqrt(E / Z) : 0.0;
            }
        }
        gsync<G>();
    }
    const uint32_t n_th = sh.n_th;
    const bool thermalize = n_th >= 2;
    if (!WB && thermalize) {
        // sums of the normals of the thermalized slots (keyed by the slot); the
        // write-back draws the same normals again and rescales them (cheaper
        // than storing and reloading them).  A cell whose moments pass summed
        // them (every slot thermalized) has them already.
        const bool zready = fast && leaf_end == 0u;
        double zs[4] = {0, 0, 0, 0};
        // the next batch's roles are loaded while this batch's normals are drawn
        uint32_t rz[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = tid + u * G;
            rz[u] = (kPrefetchRoles && !zready && i < n) ? (roles_ready ? M.role[i] : leaf_end) : 0u;
        }
        for (uint32_t s0 = tid; !zready && s0 < n; s0 += G * kU) {
            uint32_t ro[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t i = s0 + u * G;
                if constexpr (kPrefetchRoles) {
                    ro[u] = rz[u];
                    const uint32_t j = i + G * kU;
                    rz[u] = j < n ? (roles_ready ? M.role[j] : leaf_end) : 0u;
                } else {
                    ro[u] = i < n ? (roles_ready ? M.role[i] : leaf_end) : 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t s = s0 + u * G;
                if (s < n && ro[u] >= leaf_end) {
                    const Vec3<T> z = Draws<T>::normals(key, s);  // keyed by the slot
                    const double zx = (double)z.x, zy = (double)z.y, zz = (double)z.z;
                    zs[0] += zx;
                    zs[1] += zy;
                    zs[2] += zz;
                    zs[3] += zx * zx + zy * zy + zz * zz;
                }
            }
        }
        if (zready) {
#pragma unroll
            for (int q = 0; q < 4; ++q) zs[q] = sh.zt[q];  // (read by thread 0 only)
        } else {
            gsum<G, 4>(zs, gl.red);
        }
        if (tid == 0) {
            const double nt = (double)n_th;
            const double zb0 = zs[0] / nt, zb1 = zs[1] / nt, zb2 = zs[2] / nt;
            const double Z = zs[3] - nt * (zb0 * zb0 + zb1 * zb1 + zb2 * zb2);
            sh.zbar[0] = zb0;
            sh.zbar[1] = zb1;
            sh.zbar[2] = zb2;
            // a degenerate sample (zero spread) puts every thermalized particle at the removed mean
            sh.a_th = Z > 0.0 ? sqrt(sh.a_th / Z) : 0.0;
        }
        gsync<G>();
    }
    TRMC_PHASE(6);
    {
        const double a = uni(sh.a_th);
        const double u0 = uni(sh.ur[0]), u1 = uni(sh.ur[1]), u2 = uni(sh.ur[2]);
        const double z0 = uni(sh.zbar[0]), z1 = uni(sh.zbar[1]), z2 = uni(sh.zbar[2]);
        constexpr int kWU = G == 64 ? TRMC_WRITE_UNROLL_WAVE : TRMC_WRITE_UNROLL;
        // the roles of a batch, then the finals of its leaf slots (final r of
        // leaf r); thermalized slots draw their normals again
        // the next batch's roles are loaded while this batch is written
        uint32_t rw[kWU];
#pragma unroll
        for (int u = 0; u < kWU; ++u) {
            const uint32_t s = tid + u * G;
            rw[u] = (kPrefetchRoles && s < n) ? (roles_ready ? M.role[s] : leaf_end) : 0u;
        }
        for (uint32_t s0 = tid; s0 < n; s0 += G * kWU) {
            uint32_t ro[kWU];
            T fx[kWU], fy[kWU], fz[kWU];
#pragma unroll
            for (int u = 0; u < kWU; ++u) {
                const uint32_t s = s0 + u * G;
                if constexpr (kPrefetchRoles) {
                    ro[u] = rw[u];
                    const uint32_t j = s + G * kWU;
                    rw[u] = j < n ? (roles_ready ? M.role[j] : leaf_end) : 0u;
                } else {
                    ro[u] = s < n ? (roles_ready ? M.role[s] : leaf_end) : 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < kWU; ++u) {
                const uint32_t i = ro[u];
                const bool lf = s0 + u * G < n && i >= kept_end && i < leaf_end;
                const uint32_t r = lf ? leaf_rank(i, N0, P) : 0u;
                const Pack4<T> f = ld4(M.fin + (lf ? r : 0u));
                fx[u] = f.x;
                fy[u] = f.y;
                fz[u] = f.z;
                if constexpr (WB) {
                    // a final longer than m_max is replaced (when the remainder
                    // is a single particle it keeps the final's value)
                    if (lf && thermalize && f.w > wb_max) ro[u] = leaf_end;
                }
            }
#pragma unroll
            for (int u = 0; u < kWU; ++u) {
                const uint32_t s = s0 + u * G;
                const uint32_t i = ro[u];
                if (s >= n || i < kept_end) continue;
                if (i < leaf_end) {
                    vx[s] = fx[u];
                    vy[s] = fy[u];
                    vz[s] = fz[u];
                } else if (thermalize) {
                    const Vec3<T> z = Draws<T>::normals(key, s);
                    vx[s] = (T)(u0 + a * ((double)z.x - z0));
                    vy[s] = (T)(u1 + a * ((double)z.y - z1));
                    vz[s] = (T)(u2 + a * ((double)z.z - z2));
                }
            }
        }
    }
    TRMC_PHASE(7);
    TRMC_PHASE_END(n);
    if (tid == 0) write_stats(st, n, sh, elapsed_ticks(t_begin));
}

// Particles of a work item's cell (wave-uniform).
__device__ __forceinline__ uint32_t cell_size(const CellRef& r)
{
    const InstDev* I = uni(r.inst);
    const uint32_t c = uni(r.cell);
    return uni(I->cell_off[c + 1]) - uni(I->cell_off[c]);
}

// Groups of eight wave-per-cell cells occupy the first workgroups, cells of the
// workgroup-per-cell list the rest: the dispatcher starts workgroups in index
// order, and the few small-cell groups, whose deep trees make their waves run
// long, start with the longest big cells instead of at the end of the launch.
// Each group takes its cell through nsteps consecutive steps (nsteps > 1 only
// for homogeneous instances, whose cells depend on nothing but themselves); the
// group's barrier orders one step's stores before the next step's loads.  At
// the end, the cell's wall-clock time over the launch replaces the last step's
// in its counters: the cost by which the next launch is ordered.
template <typename T, bool REUSE = false>
__device__ __forceinline__ void collide_entry(const CellRef* __restrict__ big, uint32_t n_big, uint32_t lv_big,
                                              const CellRef* __restrict__ small, uint32_t n_small, uint32_t lv_small,
                                              uint32_t nsteps)
{
    const uint32_t small_blocks = (n_small + kSmallPerBlock - 1u) / kSmallPerBlock;
    const uint64_t t_launch = wall_clock64();
#ifdef TRMC_PHASE_TIMING
    if (threadIdx.x == 0 && blockIdx.x < 16384u) g_span[blockIdx.x][0] = wall_clock64();
#endif
    for (uint32_t s = 0; s < nsteps; ++s) {
        // an opaque copy of the block index: the cell's loads are made again in
        // every step instead of being kept live across the steps
        uint32_t b = blockIdx.x;
        asm volatile("" : "+s"(b));
        // cells of instances with the majorant raised level by level take their
        // own instance of the step (the plain one keeps its register budget)
        if (b >= small_blocks) {
            const uint32_t bb = b - small_blocks;
            if (!REUSE && uni(big[bb].inst->majorant) == MAJ_LEVEL)
                collide_cells<T, kCollideThreads, kCollideThreads, false, false, true>(big, n_big, bb, lv_big, s);
            else if (!REUSE && kRoles16 && bb < n_big && cell_size(big[bb]) <= 65536u)
                collide_cells<T, kCollideThreads, kCollideThreads, false, false, false, uint16_t>(big, n_big, bb,
                                                                                                 lv_big, s);
            else
                collide_cells<T, kCollideThreads, kCollideThreads, false, REUSE>(big, n_big, bb, lv_big, s);
            gsync<kCollideThreads>();
        } else {
            const uint32_t wi = b * kSmallPerBlock + uni((uint32_t)(threadIdx.x / 64));
            if (!REUSE && wi < n_small && uni(small[wi].inst->majorant) == MAJ_LEVEL)
                collide_cells<T, kCollideThreads, 64, false, false, true>(small, n_small, b, lv_small, s);
            else if (!REUSE && kRoles16 && wi < n_small && cell_size(small[wi]) <= 65536u)
                collide_cells<T, kCollideThreads, 64, false, false, false, uint16_t>(small, n_small, b, lv_small, s);
            else
                collide_cells<T, kCollideThreads, 64, false, REUSE>(small, n_small, b, lv_small, s);
            gsync<64>();
        }
    }
    // the cell's time over the whole launch (lane 0 of its group)
    {
        uint32_t b = blockIdx.x;
        asm volatile("" : "+s"(b));
        const CellRef* r = nullptr;
        if (b >= small_blocks) {
            if (threadIdx.x == 0 && b - small_blocks < n_big) r = &big[b - small_blocks];
        } else {
            const uint32_t wi = b * kSmallPerBlock + (uint32_t)(threadIdx.x / 64);
            if ((threadIdx.x & 63u) == 0 && wi < n_small) r = &small[wi];
        }
        if (r) r->inst->stats[r->cell].ticks = elapsed_ticks(t_launch);
    }
#ifdef TRMC_PHASE_TIMING
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x < 16384u) g_span[blockIdx.x][1] = wall_clock64();
#endif
}

// The per-cell chains are latency bound, so resident waves matter: the FP32
// kernel is held to TRMC_F32_WAVES_PER_EU waves per SIMD (its natural register count
// is a few registers above that bound; the spill is a few dwords).
#ifndef TRMC_F32_WAVES_PER_EU
#define TRMC_F32_WAVES_PER_EU 6
#endif
template <typename T>
__global__ void k_collide(const CellRef*, uint32_t, uint32_t, const CellRef*, uint32_t, uint32_t, uint32_t);

template <>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu(TRMC_F32_WAVES_PER_EU, 8))) void
k_collide<float>(const CellRef* __restrict__ big, uint32_t n_big, uint32_t lv_big, const CellRef* __restrict__ small,
                 uint32_t n_small, uint32_t lv_small, uint32_t nsteps)
{
    collide_entry<float>(big, n_big, lv_big, small, n_small, lv_small, nsteps);
}

// Cells of instances with tree-shape truncation: one workgroup per cell.
template <typename T>
__device__ __forceinline__ void collide_entry_wb(const CellRef* __restrict__ work, uint32_t n_work,
                                                 uint32_t lv_stride, uint32_t nsteps)
{
    for (uint32_t s = 0; s < nsteps; ++s) {
        uint32_t b = blockIdx.x;
        asm volatile("" : "+s"(b));  // per-step loads stay inside the loop
        collide_cells<T, kCollideThreads, kCollideThreads, true>(work, n_work, b, lv_stride, s);
        gsync<kCollideThreads>();
    }
}

#ifndef TRMC_WB_F32_WAVES_PER_EU
#define TRMC_WB_F32_WAVES_PER_EU 3
#endif
template <typename T>
__global__ void k_collide_wb(const CellRef*, uint32_t, uint32_t, uint32_t);

template <>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu(TRMC_WB_F32_WAVES_PER_EU, 8))) void
k_collide_wb<float>(const CellRef* __restrict__ work, uint32_t n_work, uint32_t lv_stride, uint32_t nsteps)
{
    collide_entry_wb<float>(work, n_work, lv_stride, nsteps);
}

template <>
__global__ __launch_bounds__(kCollideThreads) void k_collide_wb<double>(const CellRef* __restrict__ work,
                                                                        uint32_t n_work, uint32_t lv_stride,
                                                                        uint32_t nsteps)
{
    collide_entry_wb<double>(work, n_work, lv_stride, nsteps);
}

// Cells of instances with the adaptive depth that keeps rejected attempts, on
// the same two paths as k_collide (dynamic LDS per group: level arrays, then
// the draw offsets of each group).
template <typename T>
__global__ void k_collide_reuse(const CellRef*, uint32_t, uint32_t, const CellRef*, uint32_t, uint32_t, uint32_t);

template <>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu(TRMC_F32_WAVES_PER_EU, 8))) void
k_collide_reuse<float>(const CellRef* __restrict__ big, uint32_t n_big, uint32_t lv_big,
                       const CellRef* __restrict__ small, uint32_t n_small, uint32_t lv_small, uint32_t nsteps)
{
    collide_entry<float, true>(big, n_big, lv_big, small, n_small, lv_small, nsteps);
}

template <>
__global__ __launch_bounds__(kCollideThreads) void k_collide_reuse<double>(const CellRef* __restrict__ big,
                                                                           uint32_t n_big, uint32_t lv_big,
                                                                           const CellRef* __restrict__ small,
                                                                           uint32_t n_small, uint32_t lv_small,
                                                                           uint32_t nsteps)
{
    collide_entry<double, true>(big, n_big, lv_big, small, n_small, lv_small, nsteps);
}

// The FP64 kernel's natural register count (about 250) leaves two waves per
// SIMD; held to TRMC_F64_WAVES_PER_EU it spills a few hundred bytes per lane
// and runs faster.
#ifndef TRMC_F64_WAVES_PER_EU
#define TRMC_F64_WAVES_PER_EU 4
#endif
template <>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu(TRMC_F64_WAVES_PER_EU, 8))) void
k_collide<double>(const CellRef* __restrict__ big, uint32_t n_big,
                                                                     uint32_t lv_big,
                                                                     const CellRef* __restrict__ small,
                                                                     uint32_t n_small, uint32_t lv_small,
                                                                     uint32_t nsteps)
{
    collide_entry<double>(big, n_big, lv_big, small, n_small, lv_small, nsteps);
}

// Launch order of the whole-cell kernels: a work list sorted by the measured
// duration of each cell's last step, longest first, ties in their previous
// order (longest-processing-time-first: the dispatcher starts workgroups in
// index order as compute units free up, so the costliest cells start first and
// the launch ends on short ones).  Block b sorts list b in place, if it holds
// 2 to kOrderMax items.  The order decides when a cell runs, never what it
// computes.  Cells not yet stepped have duration 0 and keep the size order.
constexpr uint32_t kOrderMax = 8192;
constexpr uint32_t kOrderThreads = 1024;

__global__ __launch_bounds__(kOrderThreads) void k_order(CellRef* __restrict__ l0, uint32_t n0,
                                                          CellRef* __restrict__ l1, uint32_t n1)
{
    __shared__ uint64_t key[kOrderMax];
    CellRef* __restrict__ list = blockIdx.x == 0 ? l0 : l1;
    const uint32_t n = blockIdx.x == 0 ? n0 : n1;
    if (n < 2u || n > kOrderMax) return;
    uint32_t P = 2;
    while (P < n) P <<= 1;
    // key: (longest first, then previous position), padded with the largest key
    for (uint32_t i = threadIdx.x; i < P; i += kOrderThreads) {
        uint64_t k = ~0ull;
        if (i < n) {
            const CellRef r = list[i];
            const uint32_t t = r.inst->stats[r.cell].ticks;
            k = ((uint64_t)(0xFFFFFFFFu - t) << 32) | i;
        }
        key[i] = k;
    }
    __syncthreads();
    // bitonic sort, ascending
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kOrderThreads) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const uint64_t a = key[i], b = key[p];
                    if ((a > b) == ((i & k) == 0u)) {
                        key[i] = b;
                        key[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // every item's new entry is read before any is written
    constexpr int Q = kOrderMax / kOrderThreads;
    CellRef tmp[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t i = threadIdx.x + (uint32_t)q * kOrderThreads;
        if (i < n) tmp[q] = list[(uint32_t)key[i]];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t i = threadIdx.x + (uint32_t)q * kOrderThreads;
        if (i < n) list[i] = tmp[q];
    }
}

#ifdef TRMC_PHASE_TIMING
extern "C" int trmc_debug_phase_totals(unsigned long long* out /* 60 + 2 * 16384 */, int reset)
{
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), sizeof(g_phase)) != hipSuccess) return -5;
    if (hipMemcpyFromSymbol(out + 48, HIP_SYMBOL(g_maxcell), sizeof(g_maxcell)) != hipSuccess) return -5;
    if (hipMemcpyFromSymbol(out + 60, HIP_SYMBOL(g_span), sizeof(g_span)) != hipSuccess) return -5;
    if (reset) {
        static const unsigned long long zero[4][12] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase), zero, sizeof(zero)) != hipSuccess) return -5;
    }
    return 0;
}
#endif



}  // namespace trmc
