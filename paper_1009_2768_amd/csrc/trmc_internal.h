// trmc_internal.h -- device-side tables shared by the host runtime and the kernels
// of libtrmc (private to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trmc {

enum : uint32_t { GEOM_HOMOG = 1, GEOM_SLAB = 2 };
enum : uint32_t { PREC_FP64 = 1, PREC_FP32 = 2 };
enum : uint32_t { TRUNC_NATURAL = 0, TRUNC_FIXED = 1, TRUNC_ADAPTIVE = 2, TRUNC_ADAPTIVE_REUSE = 3 };
enum : uint32_t { WB_OFF = 0, WB_MIN = 1, WB_MEAN = 2 };  // tree-shape truncation (Sec. 4.4)
enum : uint32_t { CELL_OVERFLOW = 1u, INJECT_FULL = 2u };  // context error word bits
enum : uint32_t { MAJ_STEP = 0, MAJ_LEVEL = 1 };  // VHS majorant (Sec. 4.2, Remark 4.1)

constexpr uint32_t kMaxDepth = 2048;     // largest m_cap accepted
constexpr uint32_t kMaxSlabCells = 12288;  // LDS histogram of the sort
constexpr uint32_t kSortTile = 4096;     // fewest particles per tile of the counting sort
#ifndef TRMC_SORT_TILE_CELLS
#define TRMC_SORT_TILE_CELLS 2
#endif
// Particles per tile of the counting sort of a slab with n_cells cells (host and
// device): TRMC_SORT_TILE_CELLS particles per counter of the tile's dense
// histogram, rounded up to 1024, at least kSortTile.
__host__ __device__ inline uint32_t sort_tile(uint32_t n_cells)
{
    uint32_t t = TRMC_SORT_TILE_CELLS * n_cells;
    t = (t + 1023u) & ~1023u;
    return t < kSortTile ? kSortTile : t;
}
constexpr uint32_t kTile = 8192;         // slots per tile of the tiled collision pipeline
constexpr uint32_t kBigStateBytes = 1024; // per-cell state of the tiled pipeline (before its level arrays)
constexpr uint32_t kLevel1Blocks = 32;    // workgroups per large cell for the collisions of its level 1
// bytes of a large cell's level arrays (5 x (m_cap + 2) u32), rounded up to 8
__host__ __device__ inline uint64_t big_levels_bytes(uint32_t m_cap) { return (20ull * (m_cap + 2ull) + 7ull) & ~7ull; }
constexpr uint32_t kRoleBlock = 512;     // roles per block sum of the tiled pipeline
#ifndef TRMC_COLLIDE_THREADS
#define TRMC_COLLIDE_THREADS 512
#endif
constexpr uint32_t kCollideThreads = TRMC_COLLIDE_THREADS;  // threads per workgroup of the whole-cell kernel
constexpr uint32_t kSmallPerBlock = kCollideThreads / 64;  // wave-per-cell groups per workgroup
constexpr uint32_t kSmallCell = 4096;  // cells expected to hold at most this many particles use one wave
// Default path of a homogeneous cell (measured crossovers on the batched
// workload): one wave below kSmallHomog particles, the tile pipeline from
// kTiledCell on, one workgroup between.
constexpr uint32_t kSmallHomog = 1024;
constexpr uint32_t kTiledCell = 65536;
constexpr uint32_t kSmallDepth = 256;  // ... if their m_cap is at most this

// Counters of one cell's last collision step.
struct CellStats {
    uint32_t n, N0, m_eff, m_used, attempts, R0, n_th, borrowed, folds, status, wb_th;
    uint32_t ticks;  // wall-clock duration of the cell's step (100 MHz counter): its cost in the launch order
    unsigned long long collisions, dummies, violations, work_collisions;
    double q, g, E1;
    double mean[3];  // the step's pre-collision mean velocity (centre of the next step's majorant bracket)
};

// One instance, resident in its workspace.  Kernels read parameters from here;
// the step counter and the current slab buffer are advanced on the device so
// that a captured sequence of launches can be replayed step after step.
struct InstDev {
    void* x[2];
    void* vx[2];
    void* vy[2];
    void* vz[2];
    uint64_t n;
    uint32_t n_cells, geometry, precision, trunc;
    uint32_t m_init, m_cap, seed, uid;
    uint32_t step, cur;     // next step index; slab: buffer holding the state
    uint32_t n_tiles, pad0;
    uint32_t wb, wb_mmax;   // tree-shape truncation: WB_* and m_max
    uint32_t bc;            // slab ends: 0 specular walls, 1 reservoirs (open slab)
    uint32_t n_live;        // particles in the slab (open slab: changes every step; else n)
    uint32_t n_next;        // open slab: particles left after this step's transport
    uint32_t majorant;      // MAJ_STEP, or MAJ_LEVEL: the VHS bound raised level by level
    double in_sig[2], in_a[2], in_lam[2];  // reservoirs: sqrt(T), inward drift / sqrt(T), mean entries per step
    double length, dt, rho_factor, alpha, delta1, delta2, inv_dx;
    const double* eps_cells;  // [n_cells]
    uint32_t* cell_off;       // [n_cells + 1]
    uint32_t* m_state;        // [n_cells]
    CellStats* stats;         // [n_cells]
    double* moments;          // [n_cells][9]
    uint32_t* hist;           // slab: [n_tiles][n_cells] tile histograms, then tile bases
    unsigned char* scratch;   // collision scratch
    uint64_t scratch_bpp;     // scratch bytes per particle
    uint64_t scratch_cpc;     // scratch bytes per cell
    uint32_t* error;          // context error word
    double* tpart;            // tiled pipeline: [ceil(n / kTile)][8] partial sums
    double* bsum;             // tiled pipeline: [ceil(n / kRoleBlock)][8] sums over blocks of roles
    unsigned char* bigstate;  // tiled pipeline: state and level arrays between kernels
};

// One work item of the collision kernel: a cell of an instance.
struct CellRef {
    InstDev* inst;
    uint32_t cell;
    uint32_t pad;
};

// Collision capacity of a cell with n particles (trees beyond it are flagged).
__host__ __device__ inline uint64_t coll_cap(uint64_t n) { return 4ull * n + 256ull; }
__host__ __device__ inline uint64_t align16(uint64_t b) { return (b + 15ull) & ~15ull; }

// Per-cell scratch regions: role[n] u32 | fwd[n] u32 | leaf[n] | fin[n] |
// j[cap] u32 | rA[cap] u32 | rB[cap] u32 | out[2 cap], where leaf, fin and out
// hold velocities as 4-component records of `sz`-byte elements (x, y, z, pad;
// one 16- or 32-byte access per velocity).  The region of cell c starts at
// bpp * offset(c) + cpc * c, which never overlaps the next one because its size
// is at most bpp * n + cpc.
__host__ __device__ inline uint64_t scratch_bpp(uint32_t sz) { return align16(56ull + 40ull * sz); }
__host__ __device__ inline uint64_t scratch_cpc(uint32_t sz)
{
    return ((256ull * (12ull + 8ull * sz) + 195ull + 255ull) / 256ull) * 256ull;
}

}  // namespace trmc
