// k_slab.hip -- free flight in a slab with specular walls, stable counting sort
// of the particles by cell (the transport half of the first-order splitting of
// Sec. 3.1), per-cell moments, and the per-step advance of instance counters.
//
// Sort: the particles of an instance are cut into tiles of `tile` consecutive
// particles.  k_hist counts the new cells of each tile (LDS histogram, written
// densely as hist[tile][cell]); k_scan_tiles turns every column into exclusive
// tile bases and the column totals into cell offsets; k_scatter walks each tile
// in order, ranks equal cells inside a wave with ballots and across the waves of
// a chunk with short per-wave lists, and writes every particle to
// offset[cell] + base[tile][cell] + (earlier particles of that cell in the tile).
// The result is the stable order: by cell, then by previous position.
#include <hip/hip_runtime.h>

#include "../../include/trmc.h"
#include "trmc_device.h"
#include "trmc_internal.h"

namespace trmc {

template <typename T>
__device__ __forceinline__ uint32_t slab_move(T& x, T& v, T dt, T L, double inv_dx, uint32_t nc);

template <>
__device__ __forceinline__ uint32_t slab_move<double>(double& x, double& v, double dt, double L, double inv_dx,
                                                      uint32_t nc)
{
#pragma clang fp contract(off)
    double xn = fma(v, dt, x);
    double u = v;
    for (int it = 0; (xn < 0.0 || xn > L) && it < 64; ++it) {
        if (xn < 0.0) xn = -xn;
        else xn = 2.0 * L - xn;
        u = -u;
    }
    xn = xn < 0.0 ? 0.0 : (xn > L ? L : xn);  // only non-finite input gets here
    x = xn;
    v = u;
    const double cf = floor(xn * inv_dx);
    return cf < 0.0 ? 0u : (cf >= (double)nc ? nc - 1u : (uint32_t)cf);
}

template <>
__device__ __forceinline__ uint32_t slab_move<float>(float& x, float& v, float dt, float L, double inv_dx,
                                                     uint32_t nc)
{
#pragma clang fp contract(off)
    float xn = fmaf(v, dt, x);
    float u = v;
    for (int it = 0; (xn < 0.0f || xn > L) && it < 64; ++it) {
        if (xn < 0.0f) xn = -xn;
        else xn = 2.0f * L - xn;
        u = -u;
    }
    xn = xn < 0.0f ? 0.0f : (xn > L ? L : xn);  // only non-finite input gets here
    x = xn;
    v = u;
    const double cf = floor((double)xn * inv_dx);
    return cf < 0.0 ? 0u : (cf >= (double)nc ? nc - 1u : (uint32_t)cf);
}

// Free flight out of an open slab: a particle beyond either end has left and
// goes to the extra bucket nc.
template <typename T>
__device__ __forceinline__ uint32_t slab_move_open(T& x, T v, T dt, T L, double inv_dx, uint32_t nc)
{
#pragma clang fp contract(off)
    const T xn = (T)fma(v, dt, x);
    x = xn;
    if (xn < T(0) || xn > L) return nc;
    const double cf = floor((double)xn * inv_dx);
    return cf >= (double)nc ? nc - 1u : (uint32_t)cf;
}

template <typename T>
__device__ __forceinline__ uint32_t slab_step(const InstDev* I, T& x, T& v, T dt, T L, double inv_dx, uint32_t nc,
                                              bool open)
{
    return open ? slab_move_open<T>(x, v, dt, L, inv_dx, nc) : slab_move<T>(x, v, dt, L, inv_dx, nc);
}

// The sort kernels run every slab of a precision in one launch: flat block t is
// tile k of slab b (tile_of over the prefix of the slabs' tile counts).
template <typename T>
__global__ __launch_bounds__(1024) void k_hist(const CellRef* __restrict__ slabs, const uint32_t* __restrict__ prefix,
                                               uint32_t ns)
{
    extern __shared__ uint32_t hist[];
    uint32_t b, kt;
    tile_of(prefix, ns, blockIdx.x, b, kt);
    InstDev* __restrict__ I = slabs[b].inst;
    const uint32_t nc = I->n_cells;
    const bool open = I->bc != 0u;
    const uint32_t nb = nc + (open ? 1u : 0u);  // open slab: bucket nc holds the particles that left
    const uint32_t tile = sort_tile(nc);
    const uint64_t n = I->n_live;
    const uint64_t t0 = (uint64_t)kt * tile;
    const uint64_t t1 = (t0 + tile < n) ? t0 + tile : n;
    for (uint32_t c = threadIdx.x; c < nb; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    const uint32_t cur = I->cur;
    const T* __restrict__ x = reinterpret_cast<const T*>(I->x[cur]);
    const T* __restrict__ vx = reinterpret_cast<const T*>(I->vx[cur]);
    const T dt = (T)I->dt, L = (T)I->length;
    const double inv_dx = I->inv_dx;
    // four particles per thread per round: all loads of a round are issued before
    // the first count
    constexpr uint32_t kU = 4;
    for (uint64_t p0 = t0 + threadIdx.x; p0 < t1; p0 += (uint64_t)kU * blockDim.x) {
        T xp[kU], vp[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            const uint64_t p = p0 + (uint64_t)u * blockDim.x;
            xp[u] = p < t1 ? x[p] : T(0);
            vp[u] = p < t1 ? vx[p] : T(0);
        }
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            if (p0 + (uint64_t)u * blockDim.x < t1) {
                const uint32_t c = slab_step<T>(I, xp[u], vp[u], dt, L, inv_dx, nc, open);
                atomicAdd(&hist[c], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t* out = I->hist + (uint64_t)kt * nb;
    for (uint32_t c = threadIdx.x; c < nb; c += blockDim.x) out[c] = hist[c];
}

// Column scan over tiles: hist[t][c] <- sum_{t' < t} hist[t'][c]; totals to
// cell_off.  Flat block t is block k (256 cells) of slab b.
__global__ __launch_bounds__(256) void k_scan_tiles(const CellRef* __restrict__ slabs,
                                                    const uint32_t* __restrict__ prefix, uint32_t ns)
{
    uint32_t b, kb;
    tile_of(prefix, ns, blockIdx.x, b, kb);
    InstDev* __restrict__ I = slabs[b].inst;
    const uint32_t nb = I->n_cells + (I->bc != 0u ? 1u : 0u);
    const uint32_t c = kb * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const uint32_t nt = I->n_tiles;
    uint32_t* const col = I->hist + c;
    uint32_t acc = 0;
    uint32_t t = 0;
    // eight tiles per round: the round's loads are issued before its stores (the
    // rows are distinct, so no store of a round meets one of its loads)
    constexpr uint32_t kR = 8;
    for (; t + kR <= nt; t += kR) {
        uint32_t v[kR];
#pragma unroll
        for (uint32_t u = 0; u < kR; ++u) v[u] = col[(uint64_t)(t + u) * nb];
#pragma unroll
        for (uint32_t u = 0; u < kR; ++u) {
            col[(uint64_t)(t + u) * nb] = acc;
            acc += v[u];
        }
    }
    for (; t < nt; ++t) {
        const uint32_t v = col[(uint64_t)t * nb];
        col[(uint64_t)t * nb] = acc;
        acc += v;
    }
    I->cell_off[c + 1] = acc;  // counts, scanned by k_scan_cells
}

// Exclusive scan of the cell counts (one workgroup of 1024 threads per slab).
__global__ __launch_bounds__(1024) void k_scan_cells(const CellRef* __restrict__ slabs)
{
    __shared__ uint32_t part[1024];
    InstDev* __restrict__ I = slabs[blockIdx.x].inst;
    const uint32_t nc = I->n_cells + (I->bc != 0u ? 1u : 0u);  // buckets (open slab: + the leavers)
    const uint32_t per = (nc + 1023u) / 1024u;
    const uint32_t b = threadIdx.x * per;
    const uint32_t e = (b + per < nc) ? b + per : nc;
    uint32_t s = 0;
    for (uint32_t c = b; c < e; ++c) s += I->cell_off[c + 1];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024u; o <<= 1) {
        const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    // cell_off[c + 1] holds the count of cell c; each thread turns its own range
    // [b + 1, e] into offsets (read and written by the same thread only).
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (uint32_t c = b; c < e; ++c) {
        run += I->cell_off[c + 1];
        I->cell_off[c + 1] = run;
    }
    if (threadIdx.x == 0) I->cell_off[0] = 0u;
    if (I->bc != 0u) {
        __syncthreads();
        if (threadIdx.x == 0) I->n_next = I->cell_off[I->n_cells];  // particles still in the slab
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scatter(const CellRef* __restrict__ slabs,
                                                  const uint32_t* __restrict__ prefix, uint32_t ns)
{
    extern __shared__ uint32_t run[];              // [nc] next destination of each cell in this tile
    __shared__ uint32_t wl_cell[16][64];           // per-wave distinct cells of the chunk
    __shared__ uint32_t wl_cnt[16][64];
    __shared__ uint32_t wl_pre[16][64];
    __shared__ uint32_t wl_n[16];
    uint32_t b, kt;
    tile_of(prefix, ns, blockIdx.x, b, kt);
    InstDev* __restrict__ I = slabs[b].inst;
    const uint32_t nc = I->n_cells;
    const bool open = I->bc != 0u;
    const uint32_t nb = nc + (open ? 1u : 0u);
    const uint32_t tile = sort_tile(nc);
    const uint64_t n = I->n_live;
    const uint64_t t0 = (uint64_t)kt * tile;
    const uint64_t t1 = (t0 + tile < n) ? t0 + tile : n;
    const uint32_t* base = I->hist + (uint64_t)kt * nb;
    for (uint32_t c = threadIdx.x; c < nb; c += blockDim.x) run[c] = I->cell_off[c] + base[c];
    __syncthreads();
    const uint32_t cur = I->cur, nxt = cur ^ 1u;
    const T* __restrict__ x = reinterpret_cast<const T*>(I->x[cur]);
    const T* __restrict__ vx = reinterpret_cast<const T*>(I->vx[cur]);
    const T* __restrict__ vy = reinterpret_cast<const T*>(I->vy[cur]);
    const T* __restrict__ vz = reinterpret_cast<const T*>(I->vz[cur]);
    T* __restrict__ ox = reinterpret_cast<T*>(I->x[nxt]);
    T* __restrict__ ovx = reinterpret_cast<T*>(I->vx[nxt]);
    T* __restrict__ ovy = reinterpret_cast<T*>(I->vy[nxt]);
    T* __restrict__ ovz = reinterpret_cast<T*>(I->vz[nxt]);
    const T dt = (T)I->dt, L = (T)I->length;
    const double inv_dx = I->inv_dx;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64u - lane));
    // the next chunk's particle is loaded while this chunk is ranked and written
    T nx = T(0), nv = T(0), ny = T(0), nz = T(0);
    if (t0 + threadIdx.x < t1) {
        const uint64_t p = t0 + threadIdx.x;
        nx = x[p];
        nv = vx[p];
        ny = vy[p];
        nz = vz[p];
    }
    for (uint64_t cb = t0; cb < t1; cb += blockDim.x) {
        const uint64_t p = cb + threadIdx.x;
        const bool valid = p < t1;
        T xp = nx, vp = nv, wy = ny, wz = nz;
        const uint64_t pn = p + blockDim.x;
        if (pn < t1) {
            nx = x[pn];
            nv = vx[pn];
            ny = vy[pn];
            nz = vz[pn];
        }
        uint32_t c = 0;
        if (valid) c = slab_step<T>(I, xp, vp, dt, L, inv_dx, nc, open);
        // distinct cells of the wave, in lane order of first appearance
        bool pend = valid;
        uint32_t my_rank = 0, my_k = 0, k = 0;
        for (;;) {
            const unsigned long long m = __ballot(pend);
            if (m == 0ull) break;
            const uint32_t d = (uint32_t)__shfl((int)c, __ffsll((long long)m) - 1);
            const bool hit = pend && c == d;
            const unsigned long long e = __ballot(hit);
            if (hit) {
                my_rank = (uint32_t)__popcll(e & lt);
                my_k = k;
                pend = false;
            }
            if (lane == 0) {
                wl_cell[wave][k] = d;
                wl_cnt[wave][k] = (uint32_t)__popcll(e);
            }
            ++k;
        }
        if (lane == 0) wl_n[wave] = k;
        __syncthreads();
        // prefix over earlier waves of the same cell (leaders only)
        if (valid && my_rank == 0) {
            uint32_t pre = 0;
            for (uint32_t w = 0; w < wave; ++w) {
                const uint32_t kn = wl_n[w];
                for (uint32_t kk = 0; kk < kn; ++kk) pre += (wl_cell[w][kk] == c) ? wl_cnt[w][kk] : 0u;
            }
            wl_pre[wave][my_k] = pre;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = run[c] + wl_pre[wave][my_k] + my_rank;
            ox[dst] = xp;
            ovx[dst] = vp;
            ovy[dst] = wy;
            ovz[dst] = wz;
        }
        __syncthreads();
        if (valid && my_rank == 0) atomicAdd(&run[c], wl_cnt[wave][my_k]);
        __syncthreads();
        (void)nw;
    }
}


// ---------------------------------------------------------------------------
// Open slab (stationary shock, Sec. 5.2): each end is a Maxwellian reservoir.
// Per step, before transport, end e injects floor(lambda_e + U) particles,
// lambda_e the expected number crossing inward in dt.  The inward normal speed
// over sigma inverts the flux-weighted half-range law, density w phi(w - a) on
// w > 0, whose distribution function has the closed form
//   F(w) = phi(a) - phi(w - a) + a (Phi(w - a) - Phi(-a)),  F(inf) = phi(a) + a Phi(a),
// by 64 bisection steps; the tangential speeds are Maxwellian; the particle is
// placed outside by the part of the step it has not yet flown, so the transport
// that follows brings it in.  Entries go after the live particles, left end
// first.  Keys: cell field 0xFFFFFFF0 + end, tag INJ (count: index 0, aux 2;
// particle i: index i, aux 0 and 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double std_pdf(double t) { return exp(-0.5 * t * t) * 0.3989422804014327; }
__device__ __forceinline__ double std_cdf(double t) { return 0.5 * erfc(-t / 1.4142135623730951); }

__device__ __forceinline__ double flux_speed(double a, double u)
{
#pragma clang fp contract(off)
    const double pa = std_pdf(a), ca = std_cdf(-a);
    const double target = u * (pa + a * std_cdf(a));
    double lo = 0.0, hi = (a > 0.0 ? a : 0.0) + 12.0;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double F = (pa - std_pdf(mid - a)) + a * (std_cdf(mid - a) - ca);
        if (F < target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

template <typename T>
__global__ __launch_bounds__(256) void k_inject(const CellRef* __restrict__ slabs, uint32_t ns)
{
    InstDev* __restrict__ I = slabs[blockIdx.x].inst;
    if (I->bc == 0u) return;
    __shared__ uint32_t cnt[2];
    const uint32_t n = I->n_live, step = I->step;
    if (threadIdx.x < 2u) {
        const uint32_t e = threadIdx.x;
        const Key key{I->seed, I->uid, 0xFFFFFFF0u + e, step};
        const uint4 w = draw(key, 0, TAG_INJ, 2);
        const double k = floor(I->in_lam[e] + u53(w.x, w.y));
        cnt[e] = k < 4294967295.0 ? (uint32_t)k : 0xFFFFFFFFu;  // a huge count fails the capacity test
    }
    __syncthreads();
    const uint32_t kl = cnt[0], kr = cnt[1];
    if ((uint64_t)n + kl + kr > I->n) {  // arrays full: nothing enters, the step is flagged
        if (threadIdx.x == 0) atomicOr(I->error, INJECT_FULL);
        return;
    }
    const uint32_t cur = I->cur;
    T* __restrict__ x = reinterpret_cast<T*>(I->x[cur]);
    T* __restrict__ vx = reinterpret_cast<T*>(I->vx[cur]);
    T* __restrict__ vy = reinterpret_cast<T*>(I->vy[cur]);
    T* __restrict__ vz = reinterpret_cast<T*>(I->vz[cur]);
    const double dt = I->dt, L = I->length;
    for (uint32_t j = threadIdx.x; j < kl + kr; j += blockDim.x) {
#pragma clang fp contract(off)
        const uint32_t e = j < kl ? 0u : 1u;
        const uint32_t i = j < kl ? j : j - kl;
        const Key key{I->seed, I->uid, 0xFFFFFFF0u + e, step};
        const uint4 b0 = draw(key, i, TAG_INJ, 0);
        const uint4 b1 = draw(key, i, TAG_INJ, 1);
        const double u0 = u53(b0.x, b1.x), u1 = u53(b0.y, b1.y), u2 = u53(b0.z, b1.z), u3 = u53(b0.w, b1.w);
        const double sig = I->in_sig[e];
        const double vn = sig * flux_speed(I->in_a[e], u0);
        const double v = e == 0u ? vn : -vn;
        const double r = sqrt(-2.0 * log(1.0 - u2));
        double sn, cs;
        sincos(6.283185307179586 * u3, &sn, &cs);
        const uint64_t at = (uint64_t)n + j;
        x[at] = (T)(e == 0u ? -v * dt * u1 : L - v * dt * u1);
        vx[at] = (T)v;
        vy[at] = (T)(sig * (r * cs));
        vz[at] = (T)(sig * (r * sn));
    }
    __syncthreads();
    if (threadIdx.x == 0) I->n_live = n + kl + kr;
}

// Per-cell moments (FP64): rho, u, T, P_xx, P_yy, P_zz, M4 per unit mass.  With
// out, the cell's full record (moments, counters of the last step, adaptive
// depth) is also written to out[cell], which may be pinned host memory.
template <typename T>
__global__ __launch_bounds__(256) void k_moments(const CellRef* __restrict__ work, uint32_t n_work,
                                                 trmc_cell_moments* __restrict__ out)
{
    __shared__ double red[4 * 8];
    const uint32_t wi = blockIdx.x;
    if (wi >= n_work) return;
    InstDev* __restrict__ I = work[wi].inst;
    const uint32_t cell = work[wi].cell;
    const uint32_t buf = (I->geometry == GEOM_SLAB) ? I->cur : 0u;
    const uint32_t off = I->cell_off[cell];
    const uint32_t n = I->cell_off[cell + 1] - off;
    const T* vx = reinterpret_cast<const T*>(I->vx[buf]) + off;
    const T* vy = reinterpret_cast<const T*>(I->vy[buf]) + off;
    const T* vz = reinterpret_cast<const T*>(I->vz[buf]) + off;
    double s[3] = {0, 0, 0};
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        s[0] += (double)vx[i];
        s[1] += (double)vy[i];
        s[2] += (double)vz[i];
    }
    block_sum<3>(s, red);
    const double inv = n ? 1.0 / (double)n : 0.0;
    const double u0 = s[0] * inv, u1 = s[1] * inv, u2 = s[2] * inv;
    double p[4] = {0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double a = (double)vx[i], b = (double)vy[i], c = (double)vz[i];
        const double dx = a - u0, dy = b - u1, dz = c - u2;
        p[0] += dx * dx;
        p[1] += dy * dy;
        p[2] += dz * dz;
        const double e = a * a + b * b + c * c;
        p[3] += e * e;
    }
    block_sum<4>(p, red);
    if (threadIdx.x == 0) {
        double* o = I->moments + 9ull * cell;
        o[0] = (double)n * I->rho_factor;
        o[1] = u0;
        o[2] = u1;
        o[3] = u2;
        o[4] = (p[0] + p[1] + p[2]) * inv / 3.0;
        o[5] = p[0] * inv;
        o[6] = p[1] * inv;
        o[7] = p[2] * inv;
        o[8] = p[3] * inv;
        if (out) {
            const CellStats& st = I->stats[cell];
            trmc_cell_moments r;
            r.n = n;
            r.m_state = I->m_state[cell];
            r.rho = o[0];
            r.ux = o[1];
            r.uy = o[2];
            r.uz = o[3];
            r.T = o[4];
            r.Pxx = o[5];
            r.Pyy = o[6];
            r.Pzz = o[7];
            r.M4 = o[8];
            r.collisions = st.collisions;
            r.dummies = st.dummies;
            r.violations = st.violations;
            r.work_collisions = st.work_collisions;
            r.thermalized = st.n_th;
            r.borrowed = st.borrowed;
            r.m_eff = st.m_eff;
            r.m_used = st.m_used;
            r.attempts = st.attempts;
            r.N0 = st.N0;
            r.R0 = st.R0;
            r.status = st.status;
            r.wb_thermalized = st.wb_th;
            r.reserved = 0u;
            r.q = st.q;
            r.g = st.g;
            out[cell] = r;
        }
    }
}

// End of a step: advance the step counter, flip the slab buffer.
__global__ void k_advance(InstDev* const* __restrict__ insts, uint32_t n_inst, uint32_t inc)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    InstDev* I = insts[i];
    I->step += inc;  // inc > 1 only for homogeneous instances (fused steps)
    if (I->geometry == GEOM_SLAB) {
        I->cur ^= 1u;
        if (I->bc != 0u) I->n_live = I->n_next;
    }
}

template __global__ void k_hist<float>(const CellRef*, const uint32_t*, uint32_t);
template __global__ void k_hist<double>(const CellRef*, const uint32_t*, uint32_t);
template __global__ void k_scatter<float>(const CellRef*, const uint32_t*, uint32_t);
template __global__ void k_scatter<double>(const CellRef*, const uint32_t*, uint32_t);
template __global__ void k_moments<float>(const CellRef*, uint32_t, trmc_cell_moments*);
template __global__ void k_inject<float>(const CellRef*, uint32_t);
template __global__ void k_inject<double>(const CellRef*, uint32_t);
template __global__ void k_moments<double>(const CellRef*, uint32_t, trmc_cell_moments*);

}  // namespace trmc
