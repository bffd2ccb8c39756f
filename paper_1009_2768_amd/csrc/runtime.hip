// runtime.hip -- host runtime of libtrmc: validation, workspace layout, the
// instance table, the work lists of the collision kernel and the launch
// sequence of one step (transport + sort per slab, then one collision launch per
// precision over every active cell, then the device-side step advance).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/trmc.h"
#include "trmc_internal.h"

namespace trmc {
template <typename T>
__global__ void k_collide(const CellRef*, uint32_t, uint32_t, const CellRef*, uint32_t, uint32_t, uint32_t);
template <typename T>
__global__ void k_collide_wb(const CellRef*, uint32_t, uint32_t, uint32_t);
template <typename T>
__global__ void k_inject(const CellRef*, uint32_t);
template <typename T>
__global__ void k_collide_reuse(const CellRef*, uint32_t, uint32_t, const CellRef*, uint32_t, uint32_t, uint32_t);
template <typename T>
__global__ void k_hist(const CellRef*, const uint32_t*, uint32_t);
__global__ void k_scan_tiles(const CellRef*, const uint32_t*, uint32_t);
__global__ void k_scan_cells(const CellRef*);
template <typename T>
__global__ void k_scatter(const CellRef*, const uint32_t*, uint32_t);
template <typename T>
__global__ void k_moments(const CellRef*, uint32_t, trmc_cell_moments*);
struct CellLists {
    uint32_t* list;
    uint32_t* count;
    uint32_t cap;
};
template <typename T>
__global__ void k_tile_prep(const CellRef*, const uint32_t*, uint32_t, uint32_t*);
template <typename T, bool FIX>
__global__ void k_tile_bsum(const CellRef*, const uint32_t*, uint32_t);
template <typename T>
__global__ void k_tile_roles(const CellRef*, const uint32_t*, uint32_t);
template <typename T>
__global__ void k_big_split(const CellRef*, uint32_t, uint32_t, CellLists);
template <typename T, int G>
__global__ void k_big_tree(const CellRef*, uint32_t, CellLists);
template <typename T>
__global__ void k_big_level1(const CellRef*, uint32_t, uint32_t);
template <typename T, int G>
__global__ void k_big_collide(const CellRef*, uint32_t, CellLists);
template <typename T>
__global__ void k_tile_zsum(const CellRef*, const uint32_t*, uint32_t);
template <typename T>
__global__ void k_tile_write(const CellRef*, const uint32_t*, uint32_t);
__global__ void k_advance(InstDev* const*, uint32_t, uint32_t);
__global__ void k_order(CellRef*, uint32_t, CellRef*, uint32_t);
constexpr uint32_t kOrderThreads = 1024;
}  // namespace trmc

using namespace trmc;

namespace {

// The whole-cell kernels are built and tested with 512-thread workgroups only:
// a 256-thread build made a memory fault in the kernel of the adaptive depth
// with reuse, whose cause was not found.
static_assert(kCollideThreads == 512, "the whole-cell kernels support 512-thread workgroups only");

constexpr size_t kAlign = 256;
constexpr uint32_t kWaveSlabCells = 2048;  // fewest cells of a slab whose small cells default to WAVE
size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t inst, refs, eps, off, mstate, stats, mom, hist, bx, bvx, bvy, bvz, tpart, bsum, big, scratch, total;
    uint32_t n_tiles;
};

Layout layout_of(const trmc_desc& d)
{
    Layout L{};
    const size_t sz = d.precision == TRMC_FP64 ? 8 : 4;
    const uint32_t nc = d.geometry == TRMC_SLAB1D ? d.n_cells : 1u;
    const uint64_t n = d.n_particles;
    size_t p = 0;
    L.inst = p;    p += al(sizeof(InstDev));
    L.refs = p;    p += al(sizeof(CellRef) * nc);
    L.eps = p;     p += al(sizeof(double) * nc);
    L.off = p;     p += al(sizeof(uint32_t) * (nc + 2));  // + the open slab's bucket of leavers
    L.mstate = p;  p += al(sizeof(uint32_t) * nc);
    L.stats = p;   p += al(sizeof(CellStats) * nc);
    L.mom = p;     p += al(sizeof(double) * 9 * nc);
    L.n_tiles = 0;
    if (d.geometry == TRMC_SLAB1D) {
        const uint32_t tile = sort_tile(nc);
        L.n_tiles = (uint32_t)((n + tile - 1) / tile);
        L.hist = p;  p += al(sizeof(uint32_t) * (size_t)L.n_tiles * (nc + 1));
        L.bx = p;    p += al(sz * n);
        L.bvx = p;   p += al(sz * n);
        L.bvy = p;   p += al(sz * n);
        L.bvz = p;   p += al(sz * n);
    } else {
        // tiled pipeline of large homogeneous cells: tile sums, state and level arrays
        L.tpart = p; p += al(sizeof(double) * 8 * ((n + kTile - 1) / kTile));
        L.bsum = p;  p += al(sizeof(double) * 8 * ((n + kRoleBlock - 1) / kRoleBlock));
        // state, level arrays, and the level-1 partial sums of kLevel1Blocks workgroups
        L.big = p;   p += al(kBigStateBytes + big_levels_bytes(d.m_cap) + sizeof(double) * 4 * kLevel1Blocks);
    }
    L.scratch = p;
    p += al(scratch_bpp((uint32_t)sz) * n + scratch_cpc((uint32_t)sz) * nc);
    L.total = p;
    return L;
}

int validate(const trmc_desc* d)
{
    if (!d || d->struct_size != sizeof(trmc_desc)) return TRMC_EINVAL;
    if (d->geometry != TRMC_HOMOG && d->geometry != TRMC_SLAB1D) return TRMC_EINVAL;
    if (d->precision != TRMC_FP64 && d->precision != TRMC_FP32_MIXED) return TRMC_EINVAL;
    if (d->n_particles < 1 || d->n_particles > (1ull << 30)) return TRMC_EINVAL;
    if (d->geometry == TRMC_HOMOG && d->n_cells != 1) return TRMC_EINVAL;
    if (d->geometry == TRMC_SLAB1D && (d->n_cells < 1 || d->n_cells > kMaxSlabCells)) return TRMC_EINVAL;
    if (!(d->length > 0.0) || !std::isfinite(d->length)) return TRMC_EINVAL;
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return TRMC_EINVAL;
    if (!(d->particle_weight > 0.0) || !std::isfinite(d->particle_weight)) return TRMC_EINVAL;
    const uint32_t nc = d->geometry == TRMC_SLAB1D ? d->n_cells : 1u;
    if (d->eps_cells) {
        for (uint32_t c = 0; c < nc; ++c)
            if (!(d->eps_cells[c] > 0.0)) return TRMC_EINVAL;
    } else if (!(d->eps > 0.0)) {
        return TRMC_EINVAL;
    }
    if (!(d->alpha >= 0.0 && d->alpha <= 1.0)) return TRMC_EINVAL;
    if (d->trunc > TRMC_ADAPTIVE_REUSE) return TRMC_EINVAL;
    if (d->m_cap < 1 || d->m_cap > kMaxDepth) return TRMC_EINVAL;
    if (d->m_init < 1 || d->m_init > d->m_cap) return TRMC_EINVAL;
    if (d->trunc >= TRMC_ADAPTIVE && !(d->delta1 > 0.0 && d->delta1 < d->delta2)) return TRMC_EINVAL;
    if (d->wb > TRMC_WB_MEAN) return TRMC_EINVAL;
    if (d->bc > TRMC_BC_INFLOW || (d->bc == TRMC_BC_INFLOW && d->geometry != TRMC_SLAB1D)) return TRMC_EINVAL;
    if (d->bc == TRMC_BC_INFLOW) {
        for (const double* st : {d->in_left, d->in_right})
            if (!(st[0] > 0.0) || !(st[2] > 0.0) || !std::isfinite(st[0]) || !std::isfinite(st[1]) ||
                !std::isfinite(st[2]))
                return TRMC_EINVAL;
        if (d->n_live0 > d->n_particles) return TRMC_EINVAL;
    } else if (d->n_live0 != 0 && d->n_live0 != d->n_particles) {
        return TRMC_EINVAL;
    }
    if (d->wb != TRMC_WB_OFF && (d->trunc >= TRMC_ADAPTIVE || d->wb_mmax < 1)) return TRMC_EINVAL;
    if (d->majorant > TRMC_MAJORANT_LEVEL || d->reserved != 0) return TRMC_EINVAL;
    if (d->majorant == TRMC_MAJORANT_LEVEL && (d->wb != TRMC_WB_OFF || d->trunc == TRMC_ADAPTIVE_REUSE))
        return TRMC_EINVAL;
    if (d->m_state0) {
        for (uint32_t c = 0; c < nc; ++c)
            if (d->m_state0[c] < 1 || d->m_state0[c] > d->m_cap) return TRMC_EINVAL;
    }
    return 0;
}

struct Slot {
    bool active = false;
    trmc_desc desc{};
    trmc_particles user{};
    unsigned char* ws = nullptr;
    InstDev* dev = nullptr;
    InstDev host{};
    Layout lay{};
    uint64_t steps = 0;  // steps enqueued since admission
    uint64_t bytes = 0;  // device memory of the instance: its workspace and particle arrays
};

// Device memory an instance occupies: its workspace and its particle arrays.
uint64_t instance_bytes(const trmc_desc& d, const Layout& L)
{
    const uint64_t sz = d.precision == TRMC_FP64 ? 8 : 4;
    return (uint64_t)L.total + sz * d.n_particles * (d.geometry == TRMC_SLAB1D ? 4u : 3u);
}

}  // namespace

struct trmc_ctx {
    hipStream_t stream = nullptr;
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t max_inst = 0, max_cells = 0;
    uint32_t* error = nullptr;
    // work lists of the collision step, [precision: 0 FP32, 1 FP64][class]: class 0 =
    // workgroup per cell, 1 = wave per cell, 2 = tiled pipeline (large homogeneous
    // cells), 3 = workgroup per cell with tree-shape truncation; 4 and 5 = as 0
    // and 1 for the adaptive depth that keeps rejected attempts
    CellRef* work[2][6] = {};
    uint32_t n_work[2][6] = {};
    uint32_t lv_stride[2][6] = {{2, 2, 2, 2, 2, 2}, {2, 2, 2, 2, 2, 2}};
    uint32_t* tile_prefix[2] = {nullptr, nullptr};  // [n_work[k][2] + 1] first tile of each tiled cell
    uint32_t n_tiles[2] = {0, 0};
    uint32_t* cls_list[2] = {nullptr, nullptr};   // [2 * max_cells] light / heavy cells of the step
    uint32_t* cls_count[2] = {nullptr, nullptr};  // [2]
    // slabs of each precision, sorted together: tile and 256-cell block prefixes
    CellRef* slab_refs[2] = {nullptr, nullptr};
    uint32_t* slab_tpre[2] = {nullptr, nullptr};
    uint32_t* slab_cpre[2] = {nullptr, nullptr};
    uint32_t n_slab[2] = {0, 0}, slab_tiles[2] = {0, 0}, slab_cblk[2] = {0, 0}, slab_maxnc[2] = {0, 0};
    InstDev** inst_ptrs = nullptr;
    uint32_t n_active = 0;
    uint32_t cells_used = 0;
    // admission budget of device memory (trmc_set_budget; 0: none) and the
    // memory of the active instances
    uint64_t budget = 0, used = 0;
    std::vector<Slot> slots;
    int sticky = 0;
    uint32_t sched[TRMC_SCHED_BUCKETS] = {};  // TRMC_PATH_* per bucket of cell size
    // captured step: every launch of one step, replayed by trmc_step
    bool use_graph = false;
    bool graph_dirty = true;
    bool tables_dirty = false;  // admissions or retirements since the work lists were built
    // several steps in one launch per collision kernel: allowed (trmc_fuse_steps)
    // and possible (every active instance homogeneous, no cell on the tiled path)
    bool fuse = true;
    bool fusable = false;
    // whole-cell work lists re-sorted on the device before each launch by the
    // duration of every cell's last step, longest first (trmc_order_by_cost)
    bool order = true;
    hipStream_t cap_stream = nullptr;  // stream the step is captured on
    // the tile pipeline of large homogeneous cells runs on a second stream, beside
    // the slab sort and the whole-cell kernels (they touch different cells)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // uploads (descriptors at admission, work lists at rebuild) go through a ring
    // of pinned host buffers, each reused only after the event of its last
    // copies, so no upload waits for the stream to drain
    static constexpr int kStage = 8;
    unsigned char* stage[kStage] = {};
    size_t stage_cap[kStage] = {};
    hipEvent_t stage_ev[kStage] = {};
    bool stage_used[kStage] = {};
    int stage_next = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

size_t ctx_bytes(uint32_t max_inst, uint32_t max_cells)
{
    return al(sizeof(uint32_t)) + 12 * al(sizeof(CellRef) * std::max(1u, max_cells)) +
           2 * al(sizeof(uint32_t) * (std::max(1u, max_cells) + 1)) +
           2 * (al(sizeof(uint32_t) * 2 * std::max(1u, max_cells)) + al(2 * sizeof(uint32_t))) +
           2 * (al(sizeof(CellRef) * max_inst) + 2 * al(sizeof(uint32_t) * (max_inst + 1))) +
           al(sizeof(InstDev*) * std::max(1u, max_inst));
}

int hip_status(hipError_t e) { return e == hipSuccess ? 0 : TRMC_EIO; }

// Host data to upload: a byte blob and the (destination, offset, size) of each copy.
struct Uploads {
    std::vector<unsigned char> blob;
    struct Item {
        void* dst;
        size_t off, bytes;
    };
    std::vector<Item> items;
    void add(void* dst, const void* src, size_t bytes)
    {
        if (!bytes) return;
        const size_t off = (blob.size() + 15) & ~size_t(15);
        blob.resize(off + bytes);
        std::memcpy(blob.data() + off, src, bytes);
        items.push_back({dst, off, bytes});
    }
};

// Copy the uploads to the device on the context's stream through the next
// pinned staging buffer of the ring; returns without waiting for the copies.
int stage_uploads(trmc_ctx* c, const Uploads& u)
{
    if (u.items.empty()) return 0;
    const int i = c->stage_next;
    c->stage_next = (i + 1) % trmc_ctx::kStage;
    if (c->stage_used[i] && hipEventSynchronize(c->stage_ev[i]) != hipSuccess) return TRMC_EIO;
    if (c->stage_cap[i] < u.blob.size()) {
        // grow to at least twice the old size (and 64 KiB), so that growth is rare
        const size_t want = std::max(u.blob.size(), std::max<size_t>(size_t(1) << 16, 2 * c->stage_cap[i]));
        if (c->stage[i]) (void)hipHostFree(c->stage[i]);
        c->stage[i] = nullptr;
        c->stage_cap[i] = 0;
        void* p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return TRMC_EIO;
        c->stage[i] = static_cast<unsigned char*>(p);
        c->stage_cap[i] = want;
    }
    if (!c->stage_ev[i] && hipEventCreateWithFlags(&c->stage_ev[i], hipEventDisableTiming) != hipSuccess) {
        c->stage_ev[i] = nullptr;
        return TRMC_EIO;
    }
    std::memcpy(c->stage[i], u.blob.data(), u.blob.size());
    for (const auto& it : u.items)
        if (hipMemcpyAsync(it.dst, c->stage[i] + it.off, it.bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return TRMC_EIO;
    if (hipEventRecord(c->stage_ev[i], c->stream) != hipSuccess) return TRMC_EIO;
    c->stage_used[i] = true;
    return 0;
}

// Rebuild the device work lists and the instance list.  The path of a cell comes
// from the schedule bucket of its expected size; WAVE and TILED need m_cap <=
// kSmallDepth (which bounds the level arrays of eight cells in LDS) and TILED a
// homogeneous cell, else the cell takes GROUP.  Cells of instances with
// tree-shape truncation, or with the adaptive depth that keeps rejected
// attempts, take their own workgroup-per-cell lists.  Lists are ordered by
// expected size, largest first.
int rebuild_tables(trmc_ctx* c)
{
    std::vector<std::pair<double, CellRef>> order[2][6];
    std::vector<InstDev*> ptrs;
    uint32_t stride[2][6] = {{2, 2, 2, 2, 2, 2}, {2, 2, 2, 2, 2, 2}};
    for (auto& s : c->slots) {
        if (!s.active) continue;
        ptrs.push_back(s.dev);
        const int k = s.desc.precision == TRMC_FP64 ? 1 : 0;
        const bool slab = s.desc.geometry == TRMC_SLAB1D;
        const uint32_t nc = slab ? s.desc.n_cells : 1u;
        const double per = (double)s.desc.n_particles / nc;
        uint32_t bucket = 0;
        while (bucket + 1 < TRMC_SCHED_BUCKETS && per >= (double)(2ull << bucket)) ++bucket;
        uint32_t path = c->sched[bucket];
        if (path == TRMC_PATH_DEFAULT) {
            // a slab of fewer than kWaveSlabCells cells would fill too few workgroups
            // at eight cells each: one workgroup per cell instead
            if (slab) path = per <= (double)kSmallCell && nc >= kWaveSlabCells ? TRMC_PATH_WAVE : TRMC_PATH_GROUP;
            else if (per < (double)kSmallHomog) path = TRMC_PATH_WAVE;
            else path = per >= (double)kTiledCell ? TRMC_PATH_TILED : TRMC_PATH_GROUP;
        }
        const bool shallow = s.desc.m_cap <= kSmallDepth;
        int cls = 0;
        if (path == TRMC_PATH_TILED && !slab && shallow) cls = 2;
        else if (path == TRMC_PATH_WAVE && shallow) cls = 1;
        if (s.desc.wb != TRMC_WB_OFF) cls = 3;
        else if (s.desc.trunc == TRMC_ADAPTIVE_REUSE) cls = cls == 1 ? 5 : 4;
        for (uint32_t cc = 0; cc < nc; ++cc) order[k][cls].push_back({per, CellRef{s.dev, cc, 0}});
        stride[k][cls] = std::max(stride[k][cls], s.desc.m_cap + 2u);
    }
    Uploads up;
    std::vector<CellRef> w;
    std::vector<uint32_t> prefix;
    for (int k = 0; k < 2; ++k) {
        for (int cls = 0; cls < 6; ++cls) {
            auto& o = order[k][cls];
            std::stable_sort(o.begin(), o.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
            w.clear();
            for (auto& e : o) w.push_back(e.second);
            up.add(c->work[k][cls], w.data(), sizeof(CellRef) * w.size());
            c->n_work[k][cls] = (uint32_t)w.size();
            c->lv_stride[k][cls] = stride[k][cls];
            if (cls == 2) {
                prefix.assign(1, 0u);
                for (auto& e : o) prefix.push_back(prefix.back() + (uint32_t)((e.first + kTile - 1) / kTile));
                c->n_tiles[k] = prefix.back();
                up.add(c->tile_prefix[k], prefix.data(), sizeof(uint32_t) * prefix.size());
            }
        }
    }
    // slab sort tables, per precision
    std::vector<CellRef> sref[2];
    std::vector<uint32_t> tpre[2], cpre[2];
    for (int k = 0; k < 2; ++k) {
        tpre[k].assign(1, 0u);
        cpre[k].assign(1, 0u);
        c->slab_maxnc[k] = 0;
    }
    for (auto& s : c->slots) {
        if (!s.active || s.host.geometry != GEOM_SLAB) continue;
        const int k = s.host.precision == PREC_FP64 ? 1 : 0;
        sref[k].push_back(CellRef{s.dev, 0, 0});
        tpre[k].push_back(tpre[k].back() + s.lay.n_tiles);
        cpre[k].push_back(cpre[k].back() + (s.host.n_cells + 1u + 255u) / 256u);
        c->slab_maxnc[k] = std::max(c->slab_maxnc[k], s.host.n_cells + 1u);
    }
    for (int k = 0; k < 2; ++k) {
        c->n_slab[k] = (uint32_t)sref[k].size();
        c->slab_tiles[k] = tpre[k].back();
        c->slab_cblk[k] = cpre[k].back();
        if (sref[k].empty()) continue;
        up.add(c->slab_refs[k], sref[k].data(), sizeof(CellRef) * sref[k].size());
        up.add(c->slab_tpre[k], tpre[k].data(), sizeof(uint32_t) * tpre[k].size());
        up.add(c->slab_cpre[k], cpre[k].data(), sizeof(uint32_t) * cpre[k].size());
    }
    up.add(c->inst_ptrs, ptrs.data(), sizeof(InstDev*) * ptrs.size());
    c->n_active = (uint32_t)ptrs.size();
    c->fusable = c->n_active > 0 && c->n_slab[0] + c->n_slab[1] == 0 && c->n_work[0][2] + c->n_work[1][2] == 0;
    c->graph_dirty = true;
    return stage_uploads(c, up);  // stream-ordered before every later launch
}

// Reservoir constants of an open slab (the same closed forms as the CPU check,
// with contraction off, so that the mean number of entries has identical bits):
// sigma = sqrt(T), a = inward drift / sigma, lambda = (rho / weight) sigma
// (phi(a) + a Phi(a)) dt.
void reservoirs(const trmc_desc& d, InstDev& h)
{
#pragma clang fp contract(off)
    for (int e = 0; e < 2; ++e) {
        const double* st = e == 0 ? d.in_left : d.in_right;
        const double sigma = std::sqrt(st[2]);
        const double u_in = e == 0 ? st[1] : -st[1];
        const double a = u_in / sigma;
        const double phi = std::exp(-0.5 * a * a) * 0.3989422804014327;
        const double Phi = 0.5 * std::erfc(-a / std::sqrt(2.0));
        h.in_sig[e] = sigma;
        h.in_a[e] = a;
        h.in_lam[e] = st[0] / d.particle_weight * sigma * (phi + a * Phi) * d.dt;
    }
}

int admit_one(trmc_ctx* c, const trmc_desc* d, const trmc_particles* b, unsigned char* ws, size_t bytes,
              uint32_t* slot_out, bool rebuild)
{
    int rc = validate(d);
    if (rc) return rc;
    if (!b || !b->vx || !b->vy || !b->vz) return TRMC_EINVAL;
    if (d->geometry == TRMC_SLAB1D && !b->x) return TRMC_EINVAL;
    if (!ws || ((uintptr_t)ws & (kAlign - 1))) return TRMC_EINVAL;
    const Layout L = layout_of(*d);
    if (bytes < L.total) return TRMC_ENOMEM;
    const uint32_t nc = d->geometry == TRMC_SLAB1D ? d->n_cells : 1u;
    if (c->cells_used + nc > c->max_cells) return TRMC_ENOSPC;
    const uint64_t need = instance_bytes(*d, L);
    if (c->budget && c->used + need > c->budget) return TRMC_EBUSY;
    uint32_t slot = UINT32_MAX;
    for (uint32_t i = 0; i < c->slots.size(); ++i)
        if (!c->slots[i].active) { slot = i; break; }
    if (slot == UINT32_MAX) {
        if (c->slots.size() >= c->max_inst) return TRMC_ENOSPC;
        c->slots.emplace_back();
        slot = (uint32_t)c->slots.size() - 1;
    }
    Slot& s = c->slots[slot];
    s = Slot{};
    s.desc = *d;
    s.desc.eps_cells = nullptr;
    s.desc.m_state0 = nullptr;
    s.user = *b;
    s.ws = ws;
    s.lay = L;
    s.dev = reinterpret_cast<InstDev*>(ws + L.inst);
    InstDev& h = s.host;
    const size_t sz = d->precision == TRMC_FP64 ? 8 : 4;
    h.x[0] = b->x;
    h.vx[0] = b->vx;
    h.vy[0] = b->vy;
    h.vz[0] = b->vz;
    if (d->geometry == TRMC_SLAB1D) {
        h.x[1] = ws + L.bx;
        h.vx[1] = ws + L.bvx;
        h.vy[1] = ws + L.bvy;
        h.vz[1] = ws + L.bvz;
    } else {
        h.x[1] = b->x;
        h.vx[1] = b->vx;
        h.vy[1] = b->vy;
        h.vz[1] = b->vz;
    }
    h.n = d->n_particles;
    h.bc = d->bc;
    h.n_live = d->bc == TRMC_BC_INFLOW ? d->n_live0 : (uint32_t)d->n_particles;
    h.n_next = h.n_live;
    if (d->bc == TRMC_BC_INFLOW) reservoirs(*d, h);
    h.n_cells = nc;
    h.geometry = d->geometry == TRMC_SLAB1D ? GEOM_SLAB : GEOM_HOMOG;
    h.precision = d->precision == TRMC_FP64 ? PREC_FP64 : PREC_FP32;
    h.trunc = d->trunc;
    h.m_init = d->m_init;
    h.m_cap = d->m_cap;
    h.seed = d->seed;
    h.uid = d->uid;
    h.step = d->step0;
    h.cur = 0;
    h.n_tiles = L.n_tiles;
    h.wb = d->wb;
    h.wb_mmax = d->wb_mmax;
    h.majorant = d->majorant;
    h.length = d->length;
    h.dt = d->dt;
    const double volume = d->geometry == TRMC_SLAB1D ? d->length / (double)nc : d->length;
    h.rho_factor = d->particle_weight / volume;
    h.alpha = d->alpha;
    h.delta1 = d->delta1;
    h.delta2 = d->delta2;
    h.inv_dx = (double)nc / d->length;
    h.eps_cells = reinterpret_cast<const double*>(ws + L.eps);
    h.cell_off = reinterpret_cast<uint32_t*>(ws + L.off);
    h.m_state = reinterpret_cast<uint32_t*>(ws + L.mstate);
    h.stats = reinterpret_cast<CellStats*>(ws + L.stats);
    h.moments = reinterpret_cast<double*>(ws + L.mom);
    h.hist = d->geometry == TRMC_SLAB1D ? reinterpret_cast<uint32_t*>(ws + L.hist) : nullptr;
    h.scratch = ws + L.scratch;
    h.scratch_bpp = scratch_bpp((uint32_t)sz);
    h.scratch_cpc = scratch_cpc((uint32_t)sz);
    h.error = c->error;
    h.tpart = d->geometry == TRMC_SLAB1D ? nullptr : reinterpret_cast<double*>(ws + L.tpart);
    h.bsum = d->geometry == TRMC_SLAB1D ? nullptr : reinterpret_cast<double*>(ws + L.bsum);
    h.bigstate = d->geometry == TRMC_SLAB1D ? nullptr : ws + L.big;

    std::vector<double> eps(nc);
    std::vector<uint32_t> off(nc + 2, 0), ms(nc);
    std::vector<CellRef> refs(nc);
    for (uint32_t i = 0; i < nc; ++i) {
        eps[i] = d->eps_cells ? d->eps_cells[i] : d->eps;
        ms[i] = d->m_state0 ? d->m_state0[i] : d->m_init;
        refs[i] = CellRef{s.dev, i, 0};
    }
    off[nc] = h.n_live;  // homogeneous: one cell [0, n); slab: set by the sort
    off[nc + 1] = h.n_live;
    Uploads up;
    up.add(ws + L.inst, &h, sizeof(InstDev));
    up.add(ws + L.refs, refs.data(), sizeof(CellRef) * nc);
    up.add(ws + L.eps, eps.data(), sizeof(double) * nc);
    up.add(ws + L.off, off.data(), sizeof(uint32_t) * (nc + 2));
    up.add(ws + L.mstate, ms.data(), sizeof(uint32_t) * nc);
    hipError_t e = hipMemsetAsync(ws + L.stats, 0, sizeof(CellStats) * nc, c->stream);
    if (e != hipSuccess || stage_uploads(c, up) != 0) {
        s.active = false;
        return TRMC_EIO;
    }
    s.active = true;
    s.bytes = need;
    c->cells_used += nc;
    c->used += need;
    rc = rebuild ? rebuild_tables(c) : 0;
    if (rc) {
        s.active = false;
        c->cells_used -= nc;
        c->used -= need;
        return rc;
    }
    *slot_out = slot;
    return 0;
}

// Transport and counting sort of every slab of precision k (T), four launches
// whatever the number of slabs.
template <typename T>
int launch_slabs(trmc_ctx* c, int k)
{
    const uint32_t ns = c->n_slab[k];
    if (ns == 0 || c->slab_tiles[k] == 0) return 0;
    const size_t lds = sizeof(uint32_t) * c->slab_maxnc[k];
    hipLaunchKernelGGL(k_inject<T>, dim3(ns), dim3(256), 0, c->stream, c->slab_refs[k], ns);
    hipLaunchKernelGGL(k_hist<T>, dim3(c->slab_tiles[k]), dim3(1024), lds, c->stream, c->slab_refs[k],
                       c->slab_tpre[k], ns);
    hipLaunchKernelGGL(k_scan_tiles, dim3(c->slab_cblk[k]), dim3(256), 0, c->stream, c->slab_refs[k],
                       c->slab_cpre[k], ns);
    hipLaunchKernelGGL(k_scan_cells, dim3(ns), dim3(1024), 0, c->stream, c->slab_refs[k]);
    hipLaunchKernelGGL(k_scatter<T>, dim3(c->slab_tiles[k]), dim3(1024), lds, c->stream, c->slab_refs[k],
                       c->slab_tpre[k], ns);
    return hip_status(hipGetLastError());
}


// The tiled pipeline of the large homogeneous cells of precision k.
template <typename T>
int launch_tiled(trmc_ctx* c, int k)
{
    const uint32_t nt = c->n_work[k][2];
    if (nt) {
        const CellRef* bigs = c->work[k][2];
        const uint32_t* pre = c->tile_prefix[k];
        const uint32_t tiles = c->n_tiles[k];
        const uint32_t stride = c->lv_stride[k][2];
        const size_t lds1 = sizeof(uint32_t) * 5 * stride, lds8 = 8 * lds1;
        const CellLists cl{c->cls_list[k], c->cls_count[k], c->max_cells};
        const uint32_t wblocks = (nt + 7) / 8;
        hipLaunchKernelGGL(k_tile_prep<T>, dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt, c->cls_count[k]);
        hipLaunchKernelGGL((k_tile_bsum<T, false>), dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt);
        hipLaunchKernelGGL(k_big_split<T>, dim3(wblocks), dim3(512), lds8, c->stream, bigs, nt, stride, cl);
        // roles and block sums of the cells predicted wholly thermalized that are not
        // (their blocks return at once for every other cell)
        hipLaunchKernelGGL(k_tile_roles<T>, dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt);
        hipLaunchKernelGGL((k_tile_bsum<T, true>), dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt);
        hipLaunchKernelGGL((k_big_tree<T, 64>), dim3(wblocks), dim3(512), lds8, c->stream, bigs, stride, cl);
        hipLaunchKernelGGL((k_big_tree<T, 512>), dim3(nt), dim3(512), lds1, c->stream, bigs, stride, cl);
        hipLaunchKernelGGL(k_big_level1<T>, dim3(nt * kLevel1Blocks), dim3(512), 0, c->stream, bigs, nt, stride);
        hipLaunchKernelGGL((k_big_collide<T, 64>), dim3(wblocks), dim3(512), lds8, c->stream, bigs, stride, cl);
        hipLaunchKernelGGL((k_big_collide<T, 512>), dim3(nt), dim3(512), lds1, c->stream, bigs, stride, cl);
        hipLaunchKernelGGL(k_tile_zsum<T>, dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt);
        hipLaunchKernelGGL(k_tile_write<T>, dim3(tiles), dim3(512), 0, c->stream, bigs, pre, nt);
    }
    return hip_status(hipGetLastError());
}

// The whole-cell kernels of precision k (every cell not on the tiled pipeline),
// each cell taken through nsteps steps (nsteps > 1 only when the context is
// fusable).
template <typename T>
int launch_whole(trmc_ctx* c, int k, uint32_t nsteps = 1)
{
    const uint32_t nb = c->n_work[k][0], ns = c->n_work[k][1];
    if (c->order && (nb > 1 || ns > 1))
        hipLaunchKernelGGL(k_order, dim3(2), dim3(kOrderThreads), 0, c->stream, c->work[k][0], nb, c->work[k][1], ns);
    if (nb + ns) {
        const uint32_t small_blocks = (ns + kSmallPerBlock - 1) / kSmallPerBlock;
        const size_t lds = std::max(sizeof(uint32_t) * 5 * c->lv_stride[k][0],
                                    sizeof(uint32_t) * 5 * kSmallPerBlock * c->lv_stride[k][1]);
        hipLaunchKernelGGL(k_collide<T>, dim3(nb + small_blocks), dim3(kCollideThreads), lds, c->stream,
                           c->work[k][0], nb, c->lv_stride[k][0], c->work[k][1], ns, c->lv_stride[k][1], nsteps);
    }
    if (const uint32_t nw = c->n_work[k][3]) {
        hipLaunchKernelGGL(k_collide_wb<T>, dim3(nw), dim3(kCollideThreads), sizeof(uint32_t) * 5 * c->lv_stride[k][3],
                           c->stream, c->work[k][3], nw, c->lv_stride[k][3], nsteps);
    }
    const uint32_t rb = c->n_work[k][4], rs = c->n_work[k][5];
    if (c->order && (rb > 1 || rs > 1))
        hipLaunchKernelGGL(k_order, dim3(2), dim3(kOrderThreads), 0, c->stream, c->work[k][4], rb, c->work[k][5], rs);
    if (rb + rs) {
        const uint32_t small_blocks = (rs + kSmallPerBlock - 1) / kSmallPerBlock;
        const size_t lds = std::max(sizeof(uint32_t) * 6 * c->lv_stride[k][4],
                                    sizeof(uint32_t) * 6 * kSmallPerBlock * c->lv_stride[k][5]);
        hipLaunchKernelGGL(k_collide_reuse<T>, dim3(rb + small_blocks), dim3(kCollideThreads), lds, c->stream,
                           c->work[k][4], rb, c->lv_stride[k][4], c->work[k][5], rs, c->lv_stride[k][5], nsteps);
    }
    return hip_status(hipGetLastError());
}

}  // namespace

extern "C" {

int trmc_abi_version(void) { return TRMC_ABI_VERSION; }

const char* trmc_strerror(int status)
{
    switch (status) {
    case 0: return "success";
    case TRMC_EINVAL: return "invalid argument (descriptor, buffer or slot)";
    case TRMC_ENOMEM: return "workspace too small";
    case TRMC_ENOSPC: return "no free instance slot or cell capacity";
    case TRMC_EIO: return "HIP runtime error";
    case TRMC_EOVERFLOW: return "a cell's collision trees exceeded the scratch capacity (cell left unchanged)";
    case TRMC_EBUSY: return "admission would exceed the context's device-memory budget";
    default: return "unknown status";
    }
}

int trmc_workspace_size(const trmc_desc* descs, uint32_t n_inst, size_t* bytes)
{
    if (!bytes || (n_inst && !descs)) return TRMC_EINVAL;
    size_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        int rc = validate(&descs[i]);
        if (rc) return rc;
        total += layout_of(descs[i]).total;
    }
    *bytes = total;
    return 0;
}

int trmc_ctx_workspace_size(uint32_t max_instances, uint32_t max_cells, size_t* bytes)
{
    if (!bytes || max_instances == 0) return TRMC_EINVAL;
    *bytes = ctx_bytes(max_instances, max_cells);
    return 0;
}

int trmc_init(trmc_ctx** out, const trmc_desc* descs, uint32_t n_inst, const trmc_particles* bufs,
              void* workspace, size_t workspace_bytes, uint32_t max_instances, uint32_t max_cells,
              void* hip_stream)
{
    if (!out || (n_inst && (!descs || !bufs)) || !workspace || max_instances < n_inst || max_instances == 0)
        return TRMC_EINVAL;
    if ((uintptr_t)workspace & (kAlign - 1)) return TRMC_EINVAL;
    size_t need = ctx_bytes(max_instances, max_cells);
    uint32_t cells = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        int rc = validate(&descs[i]);
        if (rc) return rc;
        need += layout_of(descs[i]).total;
        cells += descs[i].geometry == TRMC_SLAB1D ? descs[i].n_cells : 1u;
    }
    if (cells > max_cells) return TRMC_ENOSPC;
    if (workspace_bytes < need) return TRMC_ENOMEM;
    trmc_ctx* c = new (std::nothrow) trmc_ctx();
    if (!c) return TRMC_ENOMEM;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = reinterpret_cast<unsigned char*>(workspace);
    c->ws_bytes = workspace_bytes;
    c->max_inst = max_instances;
    c->max_cells = max_cells;
    size_t p = 0;
    c->error = reinterpret_cast<uint32_t*>(c->ws + p);
    p += al(sizeof(uint32_t));
    for (int k = 0; k < 2; ++k) {
        for (int cls = 0; cls < 6; ++cls) {
            c->work[k][cls] = reinterpret_cast<CellRef*>(c->ws + p);
            p += al(sizeof(CellRef) * std::max(1u, max_cells));
        }
        c->tile_prefix[k] = reinterpret_cast<uint32_t*>(c->ws + p);
        p += al(sizeof(uint32_t) * (std::max(1u, max_cells) + 1));
        c->cls_list[k] = reinterpret_cast<uint32_t*>(c->ws + p);
        p += al(sizeof(uint32_t) * 2 * std::max(1u, max_cells));
        c->cls_count[k] = reinterpret_cast<uint32_t*>(c->ws + p);
        p += al(2 * sizeof(uint32_t));
    }
    for (int k = 0; k < 2; ++k) {
        c->slab_refs[k] = reinterpret_cast<CellRef*>(c->ws + p);
        p += al(sizeof(CellRef) * max_instances);
        c->slab_tpre[k] = reinterpret_cast<uint32_t*>(c->ws + p);
        p += al(sizeof(uint32_t) * (max_instances + 1));
        c->slab_cpre[k] = reinterpret_cast<uint32_t*>(c->ws + p);
        p += al(sizeof(uint32_t) * (max_instances + 1));
    }
    c->inst_ptrs = reinterpret_cast<InstDev**>(c->ws + p);
    p += al(sizeof(InstDev*) * std::max(1u, max_instances));
    if (hipMemsetAsync(c->error, 0, sizeof(uint32_t), c->stream) != hipSuccess) {
        delete c;
        return TRMC_EIO;
    }
    for (uint32_t i = 0; i < n_inst; ++i) {
        const size_t b = layout_of(descs[i]).total;
        uint32_t slot;
        int rc = admit_one(c, &descs[i], &bufs[i], c->ws + p, b, &slot, false);
        if (rc) {
            delete c;
            return rc;
        }
        p += b;
    }
    int rc = rebuild_tables(c);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return 0;
}

int trmc_admit(trmc_ctx* c, const trmc_desc* desc, const trmc_particles* buf, void* workspace,
               size_t workspace_bytes, uint32_t* slot)
{
    if (!c || !slot) return TRMC_EINVAL;
    // the work lists are rebuilt once, at the next step, for all admissions and
    // retirements since the last one
    const int rc = admit_one(c, desc, buf, reinterpret_cast<unsigned char*>(workspace), workspace_bytes, slot, false);
    if (!rc) c->tables_dirty = true;
    return rc;
}

int trmc_retire(trmc_ctx* c, uint32_t slot)
{
    if (!c || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    Slot& s = c->slots[slot];
    s.active = false;
    c->cells_used -= s.host.n_cells;
    c->used -= s.bytes;
    c->tables_dirty = true;  // no step is enqueued for it from now on
    return 0;
}

namespace {

// Every launch of one step on stream st: transport and sort of the slabs, the
// collision step of each precision, the step counters.
int enqueue_step(trmc_ctx* c, hipStream_t st)
{
    const hipStream_t keep = c->stream;
    int rc = 0;
    // fork: the tiled pipeline on the side stream, after everything before this step
    const bool fork = c->side && (c->n_work[0][2] + c->n_work[1][2]) > 0;
    if (fork) {
        if (hipEventRecord(c->ev_fork, st) != hipSuccess || hipStreamWaitEvent(c->side, c->ev_fork, 0) != hipSuccess)
            return TRMC_EIO;
        c->stream = c->side;
        for (int k = 0; k < 2 && !rc; ++k) rc = k == 0 ? launch_tiled<float>(c, 0) : launch_tiled<double>(c, 1);
        if (!rc && hipEventRecord(c->ev_join, c->side) != hipSuccess) rc = TRMC_EIO;
    }
    c->stream = st;
    if (!fork)
        for (int k = 0; k < 2 && !rc; ++k) rc = k == 0 ? launch_tiled<float>(c, 0) : launch_tiled<double>(c, 1);
    for (int k = 0; k < 2 && !rc; ++k) rc = k == 0 ? launch_slabs<float>(c, 0) : launch_slabs<double>(c, 1);
    for (int k = 0; k < 2 && !rc; ++k) rc = k == 0 ? launch_whole<float>(c, 0) : launch_whole<double>(c, 1);
    // join before the step counters advance
    if (fork && hipStreamWaitEvent(st, c->ev_join, 0) != hipSuccess && !rc) rc = TRMC_EIO;
    if (!rc && c->n_active)
        hipLaunchKernelGGL(k_advance, dim3((c->n_active + 255) / 256), dim3(256), 0, st, c->inst_ptrs,
                           c->n_active, 1u);
    if (!rc && hipGetLastError() != hipSuccess) rc = TRMC_EIO;
    c->stream = keep;
    return rc;
}

// n steps of a fusable context: one launch per collision kernel takes every
// cell through up to kFuseMax steps (a cell's step depends on its own previous
// step only), then the step counters advance by as many; longer calls are cut
// into such chunks so that no single launch runs for long.
constexpr uint32_t kFuseMax = 32;

int enqueue_fused(trmc_ctx* c, uint32_t n)
{
    int rc = 0;
    for (uint32_t done = 0; done < n && !rc;) {
        const uint32_t m = std::min(kFuseMax, n - done);
        for (int k = 0; k < 2 && !rc; ++k) rc = k == 0 ? launch_whole<float>(c, 0, m) : launch_whole<double>(c, 1, m);
        if (!rc)
            hipLaunchKernelGGL(k_advance, dim3((c->n_active + 255) / 256), dim3(256), 0, c->stream, c->inst_ptrs,
                               c->n_active, m);
        if (!rc && hipGetLastError() != hipSuccess) rc = TRMC_EIO;
        done += m;
    }
    return rc;
}

void drop_graph(trmc_ctx* c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// Capture one step on the context's private stream (the caller's stream may be
// the null stream, which cannot be captured).
// The side stream and its two events (default priority), made once.
int ensure_side(trmc_ctx* c)
{
    if (c->side) return 0;
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        c->side = nullptr;
        return TRMC_EIO;
    }
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
        return TRMC_EIO;
    return 0;
}

int capture_step(trmc_ctx* c)
{
    if (c->graph_exec && hipStreamSynchronize(c->stream) != hipSuccess) return TRMC_EIO;
    drop_graph(c);
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return TRMC_EIO;
    }
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return TRMC_EIO;
    const int rc = enqueue_step(c, c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : TRMC_EIO;
    }
    c->graph = g;
    if (hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        c->graph_exec = nullptr;
        drop_graph(c);
        return TRMC_EIO;
    }
    c->graph_dirty = false;
    return 0;
}

}  // namespace

int trmc_step(trmc_ctx* c, uint32_t n_steps)
{
    if (!c) return TRMC_EINVAL;
    if (c->sticky) return c->sticky;
    if (n_steps == 0) return 0;
    if (c->tables_dirty) {
        const int rc = rebuild_tables(c);
        if (rc) return c->sticky = rc;
        c->tables_dirty = false;
    }
    if (c->fuse && c->fusable && n_steps > 1) {
        const int rc = enqueue_fused(c, n_steps);
        if (rc) return c->sticky = rc;
        for (auto& s : c->slots)
            if (s.active) s.steps += n_steps;
        return 0;
    }
    if (const int rc = ensure_side(c)) return c->sticky = rc;
    if (c->use_graph && c->graph_dirty) {
        const int rc = capture_step(c);
        if (rc) return c->sticky = rc;
    }
    for (uint32_t it = 0; it < n_steps; ++it) {
        if (c->use_graph) {
            if (hipGraphLaunch(c->graph_exec, c->stream) != hipSuccess) return c->sticky = TRMC_EIO;
        } else {
            const int rc = enqueue_step(c, c->stream);
            if (rc) return c->sticky = rc;
        }
        for (auto& s : c->slots)
            if (s.active) s.steps++;
    }
    return 0;
}

int trmc_set_schedule(trmc_ctx* c, const uint32_t* paths, uint32_t n_buckets)
{
    if (!c || (n_buckets && !paths) || n_buckets > TRMC_SCHED_BUCKETS) return TRMC_EINVAL;
    for (uint32_t b = 0; b < n_buckets; ++b)
        if (paths[b] > TRMC_PATH_TILED) return TRMC_EINVAL;
    for (uint32_t b = 0; b < TRMC_SCHED_BUCKETS; ++b) c->sched[b] = b < n_buckets ? paths[b] : TRMC_PATH_DEFAULT;
    return rebuild_tables(c);
}

int trmc_get_schedule(const trmc_ctx* c, uint32_t* paths, uint32_t n_buckets)
{
    if (!c || (n_buckets && !paths) || n_buckets > TRMC_SCHED_BUCKETS) return TRMC_EINVAL;
    for (uint32_t b = 0; b < n_buckets; ++b) paths[b] = c->sched[b];
    return 0;
}

int trmc_fuse_steps(trmc_ctx* c, int on)
{
    if (!c) return TRMC_EINVAL;
    if (c->sticky) return c->sticky;
    c->fuse = on != 0;
    return 0;
}

int trmc_set_budget(trmc_ctx* c, uint64_t bytes)
{
    if (!c) return TRMC_EINVAL;
    c->budget = bytes;
    return 0;
}

int trmc_order_by_cost(trmc_ctx* c, int on)
{
    if (!c) return TRMC_EINVAL;
    if (c->sticky) return c->sticky;
    if (c->order != (on != 0)) {
        c->order = on != 0;
        c->graph_dirty = true;
        if (!c->order) return rebuild_tables(c);  // back to the size order
    }
    return 0;
}

int trmc_use_graph(trmc_ctx* c, int on)
{
    if (!c) return TRMC_EINVAL;
    if (c->sticky) return c->sticky;
    c->use_graph = on != 0;
    if (!c->use_graph) {
        // launches already enqueued keep the executable graph alive until they end
        if (hipStreamSynchronize(c->stream) != hipSuccess) return c->sticky = TRMC_EIO;
        drop_graph(c);
        c->graph_dirty = true;
    }
    return 0;
}

int trmc_sync(trmc_ctx* c)
{
    if (!c) return TRMC_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return c->sticky = TRMC_EIO;
    uint32_t err = 0;
    if (hipMemcpy(&err, c->error, sizeof err, hipMemcpyDeviceToHost) != hipSuccess) return c->sticky = TRMC_EIO;
    if (err) {
        const uint32_t zero = 0;
        if (hipMemcpy(c->error, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return TRMC_EIO;
        return (err & INJECT_FULL) ? TRMC_ENOSPC : TRMC_EOVERFLOW;
    }
    return c->sticky;
}

int trmc_state(trmc_ctx* c, uint32_t slot, trmc_particles* out)
{
    if (!c || !out || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    const Slot& s = c->slots[slot];
    const uint32_t cur = s.host.geometry == GEOM_SLAB ? (uint32_t)(s.steps & 1u) : 0u;
    out->x = s.host.x[cur];
    out->vx = s.host.vx[cur];
    out->vy = s.host.vy[cur];
    out->vz = s.host.vz[cur];
    return 0;
}

int trmc_moments(trmc_ctx* c, uint32_t slot, trmc_cell_moments* host_out, uint32_t cap)
{
    if (!c || !host_out || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    Slot& s = c->slots[slot];
    const uint32_t nc = s.host.n_cells;
    if (cap < nc) return TRMC_EINVAL;
    const CellRef* refs = reinterpret_cast<const CellRef*>(s.ws + s.lay.refs);
    if (s.host.precision == PREC_FP64)
        hipLaunchKernelGGL(k_moments<double>, dim3(nc), dim3(256), 0, c->stream, refs, nc, nullptr);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(nc), dim3(256), 0, c->stream, refs, nc, nullptr);
    if (hipGetLastError() != hipSuccess) return c->sticky = TRMC_EIO;
    std::vector<double> mom(9ull * nc);
    std::vector<CellStats> st(nc);
    std::vector<uint32_t> ms(nc);
    hipError_t e = hipMemcpyAsync(mom.data(), s.host.moments, sizeof(double) * 9 * nc, hipMemcpyDeviceToHost,
                                  c->stream);
    e = e == hipSuccess ? hipMemcpyAsync(st.data(), s.host.stats, sizeof(CellStats) * nc, hipMemcpyDeviceToHost,
                                         c->stream) : e;
    e = e == hipSuccess ? hipMemcpyAsync(ms.data(), s.host.m_state, sizeof(uint32_t) * nc, hipMemcpyDeviceToHost,
                                         c->stream) : e;
    if (e != hipSuccess) return c->sticky = TRMC_EIO;
    int rc = trmc_sync(c);
    for (uint32_t i = 0; i < nc; ++i) {
        trmc_cell_moments& o = host_out[i];
        std::memset(&o, 0, sizeof o);
        const double* m = &mom[9ull * i];
        o.rho = m[0];
        o.ux = m[1];
        o.uy = m[2];
        o.uz = m[3];
        o.T = m[4];
        o.Pxx = m[5];
        o.Pyy = m[6];
        o.Pzz = m[7];
        o.M4 = m[8];
        o.n = (uint32_t)llround(m[0] / s.host.rho_factor);
        o.m_state = ms[i];
        o.collisions = st[i].collisions;
        o.dummies = st[i].dummies;
        o.violations = st[i].violations;
        o.work_collisions = st[i].work_collisions;
        o.thermalized = st[i].n_th;
        o.wb_thermalized = st[i].wb_th;
        o.borrowed = st[i].borrowed;
        o.m_eff = st[i].m_eff;
        o.m_used = st[i].m_used;
        o.attempts = st[i].attempts;
        o.N0 = st[i].N0;
        o.R0 = st[i].R0;
        o.status = st[i].status;
        o.q = st[i].q;
        o.g = st[i].g;
    }
    return rc;
}

int trmc_moments_async(trmc_ctx* c, uint32_t slot, trmc_cell_moments* out, uint32_t cap)
{
    if (!c || !out || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    if (c->sticky) return c->sticky;
    Slot& s = c->slots[slot];
    const uint32_t nc = s.host.n_cells;
    if (cap < nc) return TRMC_EINVAL;
    const CellRef* refs = reinterpret_cast<const CellRef*>(s.ws + s.lay.refs);
    if (s.host.precision == PREC_FP64)
        hipLaunchKernelGGL(k_moments<double>, dim3(nc), dim3(256), 0, c->stream, refs, nc, out);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(nc), dim3(256), 0, c->stream, refs, nc, out);
    return hipGetLastError() == hipSuccess ? 0 : (c->sticky = TRMC_EIO);
}

int trmc_read(trmc_ctx* c, uint32_t slot, void* x, void* vx, void* vy, void* vz, uint32_t* m_state,
              uint32_t* step)
{
    if (!c || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    Slot& s = c->slots[slot];
    trmc_particles cur{};
    trmc_state(c, slot, &cur);
    int rc = trmc_sync(c);
    uint64_t live = s.host.n;
    if (s.host.bc != 0u) {
        uint32_t nl = 0;
        if (hipMemcpy(&nl, &s.dev->n_live, sizeof nl, hipMemcpyDeviceToHost) != hipSuccess) return c->sticky = TRMC_EIO;
        live = nl;
    }
    const size_t bytes = (s.host.precision == PREC_FP64 ? 8 : 4) * live;
    hipError_t e = hipSuccess;
    if (x && s.host.geometry == GEOM_SLAB) e = e == hipSuccess ? hipMemcpy(x, cur.x, bytes, hipMemcpyDeviceToHost) : e;
    if (vx) e = e == hipSuccess ? hipMemcpy(vx, cur.vx, bytes, hipMemcpyDeviceToHost) : e;
    if (vy) e = e == hipSuccess ? hipMemcpy(vy, cur.vy, bytes, hipMemcpyDeviceToHost) : e;
    if (vz) e = e == hipSuccess ? hipMemcpy(vz, cur.vz, bytes, hipMemcpyDeviceToHost) : e;
    if (m_state)
        e = e == hipSuccess ? hipMemcpy(m_state, s.host.m_state, sizeof(uint32_t) * s.host.n_cells,
                                        hipMemcpyDeviceToHost) : e;
    if (step) *step = s.desc.step0 + (uint32_t)s.steps;
    if (e != hipSuccess) return c->sticky = TRMC_EIO;
    return rc;
}

int trmc_count(trmc_ctx* c, uint32_t slot, uint64_t* n_live)
{
    if (!c || !n_live || slot >= c->slots.size() || !c->slots[slot].active) return TRMC_EINVAL;
    const Slot& s = c->slots[slot];
    const int rc = trmc_sync(c);
    if (s.host.bc == 0u) {
        *n_live = s.host.n;
        return rc;
    }
    uint32_t nl = 0;
    if (hipMemcpy(&nl, &s.dev->n_live, sizeof nl, hipMemcpyDeviceToHost) != hipSuccess) return c->sticky = TRMC_EIO;
    *n_live = nl;
    return rc;
}

int trmc_destroy(trmc_ctx* c)
{
    if (!c) return TRMC_EINVAL;
    const hipError_t e = hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (int i = 0; i < trmc_ctx::kStage; ++i) {
        if (c->stage_ev[i]) (void)hipEventDestroy(c->stage_ev[i]);
        if (c->stage[i]) (void)hipHostFree(c->stage[i]);
    }
    delete c;
    return e == hipSuccess ? 0 : TRMC_EIO;
}

}  // extern "C"
