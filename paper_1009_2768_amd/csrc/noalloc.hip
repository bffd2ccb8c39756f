// noalloc.hip -- trmc_step_static: the collision steps of one space-homogeneous
// instance with all of the library's working memory (instance record, cell
// tables, the per-cell scratch of roles, leaves, finals, tree schedule and level
// outputs, and the work list) in a static device array, so that the call
// allocates nothing: for callers that cannot allocate (code under stream
// capture, allocation-free serving loops).
//
// The array is `scratch` below, kStaticBytes per device, held by every GPU the
// library runs on until the process ends.  Its device address is taken once per
// device with hipGetSymbolAddress (in host code the array's name is a host-side
// stand-in, not a device address) and only that address is handed to kernels.
// Every call on a device shares that device's array and leaves the last call's
// contents in it; calls that overlap on one device (two streams, two host
// threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/trmc.h"
#include "trmc_internal.h"

namespace trmc {
template <typename T>
__global__ void k_collide(const CellRef*, uint32_t, uint32_t, const CellRef*, uint32_t, uint32_t, uint32_t);
__global__ void k_advance(InstDev* const*, uint32_t, uint32_t);
}  // namespace trmc

using namespace trmc;

namespace {

constexpr size_t kStaticBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
constexpr uint32_t kStaticFuseMax = 32;  // steps per launch, as the context path

__device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_ptr_lock;
unsigned char* g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The device address of this device's array (taken on the first call on it).
int scratch_ptr(unsigned char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TRMC_EIO;
    if (dev >= kMaxDevices) return TRMC_EINVAL;
    std::lock_guard<std::mutex> lock(g_ptr_lock);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TRMC_EIO;
        g_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_ptr[dev];
    return 0;
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Offsets of the pieces inside the array (one homogeneous cell).
struct StaticLayout {
    size_t inst, ref, ptr, eps, off, mstate, stats, mom, err, cells, total;
};

StaticLayout static_layout(uint64_t n, uint32_t sz)
{
    StaticLayout L{};
    size_t p = 0;
    L.inst = p;   p += al256(sizeof(InstDev));
    L.ref = p;    p += al256(sizeof(CellRef));
    L.ptr = p;    p += al256(sizeof(InstDev*));
    L.eps = p;    p += al256(sizeof(double));
    L.off = p;    p += al256(sizeof(uint32_t) * 3);
    L.mstate = p; p += al256(sizeof(uint32_t));
    L.stats = p;  p += al256(sizeof(CellStats));
    L.mom = p;    p += al256(sizeof(double) * 9);
    L.err = p;    p += al256(sizeof(uint32_t));
    L.cells = p;  p += al256(scratch_bpp(sz) * n + scratch_cpc(sz));
    L.total = p;
    return L;
}

// Fills the instance record and the cell tables inside the array (one thread):
// everything the collision kernel reads, and the state that must start afresh
// (adaptive depth, counters, error word).
__global__ void k_static_setup(InstDev h, unsigned char* base, StaticLayout L, double eps)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    InstDev* I = reinterpret_cast<InstDev*>(base + L.inst);
    h.eps_cells = reinterpret_cast<const double*>(base + L.eps);
    h.cell_off = reinterpret_cast<uint32_t*>(base + L.off);
    h.m_state = reinterpret_cast<uint32_t*>(base + L.mstate);
    h.stats = reinterpret_cast<CellStats*>(base + L.stats);
    h.moments = reinterpret_cast<double*>(base + L.mom);
    h.scratch = base + L.cells;
    h.error = reinterpret_cast<uint32_t*>(base + L.err);
    *I = h;
    *reinterpret_cast<double*>(base + L.eps) = eps;
    uint32_t* off = reinterpret_cast<uint32_t*>(base + L.off);
    off[0] = 0u;
    off[1] = (uint32_t)h.n;
    off[2] = (uint32_t)h.n;
    *reinterpret_cast<uint32_t*>(base + L.mstate) = h.m_init;
    *reinterpret_cast<CellStats*>(base + L.stats) = CellStats{};
    *reinterpret_cast<uint32_t*>(base + L.err) = 0u;
    *reinterpret_cast<CellRef*>(base + L.ref) = CellRef{I, 0u, 0u};
    *reinterpret_cast<InstDev**>(base + L.ptr) = I;
}

}  // namespace

extern "C" int trmc_step_static(const trmc_desc* d, const trmc_particles* b, uint32_t n_steps, void* hip_stream)
{
    if (!d || !b || !b->vx || !b->vy || !b->vz) return TRMC_EINVAL;
    size_t ws = 0;
    if (int rc = trmc_workspace_size(d, 1, &ws)) return rc;  // validates the descriptor (host only)
    if (d->geometry != TRMC_HOMOG || d->eps_cells || d->m_state0 || d->wb != TRMC_WB_OFF ||
        d->trunc == TRMC_ADAPTIVE_REUSE)
        return TRMC_EINVAL;
    const uint32_t sz = d->precision == TRMC_FP64 ? 8u : 4u;
    const StaticLayout L = static_layout(d->n_particles, sz);
    if (L.total > kStaticBytes) return TRMC_ENOMEM;  // the instance does not fit in the static array
    if (n_steps == 0) return 0;
    unsigned char* base = nullptr;
    if (int rc = scratch_ptr(&base)) return rc;
    const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);

    InstDev h{};
    for (int k = 0; k < 2; ++k) {
        h.x[k] = b->x;
        h.vx[k] = b->vx;
        h.vy[k] = b->vy;
        h.vz[k] = b->vz;
    }
    h.n = d->n_particles;
    h.n_cells = 1;
    h.geometry = GEOM_HOMOG;
    h.precision = d->precision == TRMC_FP64 ? PREC_FP64 : PREC_FP32;
    h.trunc = d->trunc;
    h.m_init = d->m_init;
    h.m_cap = d->m_cap;
    h.seed = d->seed;
    h.uid = d->uid;
    h.step = d->step0;
    h.n_live = (uint32_t)d->n_particles;
    h.n_next = h.n_live;
    h.wb = TRMC_WB_OFF;
    h.majorant = d->majorant;
    h.length = d->length;
    h.dt = d->dt;
    h.rho_factor = d->particle_weight / d->length;
    h.alpha = d->alpha;
    h.delta1 = d->delta1;
    h.delta2 = d->delta2;
    h.inv_dx = 1.0 / d->length;
    h.scratch_bpp = scratch_bpp(sz);
    h.scratch_cpc = scratch_cpc(sz);
    hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(64), 0, st, h, base, L, d->eps);

    // the cell takes the whole-cell kernel: one wave below 1024 particles (when
    // its depth fits the wave path), one workgroup otherwise
    const bool wave = d->n_particles < 1024u && d->m_cap <= 256u;
    const uint32_t lv = d->m_cap + 2u;
    const CellRef* ref = reinterpret_cast<const CellRef*>(base + L.ref);
    InstDev* const* ptrs = reinterpret_cast<InstDev* const*>(base + L.ptr);
    const size_t lds = sizeof(uint32_t) * 5 * lv * (wave ? kSmallPerBlock : 1u);
    for (uint32_t done = 0; done < n_steps;) {
        const uint32_t m = n_steps - done < kStaticFuseMax ? n_steps - done : kStaticFuseMax;
        if (d->precision == TRMC_FP64)
            hipLaunchKernelGGL(k_collide<double>, dim3(1), dim3(kCollideThreads), lds, st, wave ? nullptr : ref,
                               wave ? 0u : 1u, lv, wave ? ref : nullptr, wave ? 1u : 0u, lv, m);
        else
            hipLaunchKernelGGL(k_collide<float>, dim3(1), dim3(kCollideThreads), lds, st, wave ? nullptr : ref,
                               wave ? 0u : 1u, lv, wave ? ref : nullptr, wave ? 1u : 0u, lv, m);
        hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, ptrs, 1u, m);
        done += m;
    }
    return hipGetLastError() == hipSuccess ? 0 : TRMC_EIO;
}
