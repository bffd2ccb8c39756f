/*
 * trmc.h -- C ABI of the MI355X (gfx950) TRMC-R library.
 *
 * One time step is the first-order splitting of Sec. 3.1 of Trazzi, Pareschi and
 * Wennberg: free flight (1-D slab only), a stable counting sort of the particles
 * by cell, then the space-homogeneous collision step of every cell by recursive
 * time-relaxed Monte Carlo (Alg. 4.2 split into collision sets, Alg. 4.3 / 4.4
 * recursive collision trees with dummy collisions, Maxwellian remainder) with
 * optional adaptive depth (Sec. 4.3).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success, a negative errno-style code otherwise
 *     (TRMC_EINVAL, TRMC_ENOMEM, TRMC_ENOSPC, TRMC_EIO, TRMC_EOVERFLOW, TRMC_EBUSY);
 *     trmc_strerror() gives the text.  No exception crosses the ABI.
 *   - Arguments are validated before anything is enqueued; a failing call leaves
 *     the context unchanged.  Errors of asynchronous GPU work surface at the next
 *     synchronising call (trmc_sync, trmc_moments, trmc_read).
 *   - Device memory is never allocated or freed by the library: particle arrays
 *     and workspaces are owned by the caller and must outlive the context.  The
 *     context owns only host-side objects: a second stream and its events, the
 *     captured graph, and a ring of pinned host staging buffers for its uploads
 *     (grown on demand, freed by trmc_destroy).
 *   - Work is enqueued on the HIP stream given at creation; calls on one context
 *     must come from one host thread at a time.
 *   - Results depend only on (descriptor, initial particles, number of steps)
 *     and, in their last bits, on each cell's kernel path: not on the slot an
 *     instance occupies, on the other instances in the batch, on the launch
 *     order, on graph replay or on fused steps.  The kernel path of a cell (one
 *     workgroup, one wave or the tile pipeline; trmc_set_schedule) fixes the
 *     order of its FP64 cell sums, so two paths agree to rounding (FP64: within
 *     1e-12 of the thermal speed), and an integer decision taken from such a sum
 *     (the adaptive indicator at a threshold, the majorant's 20-bit grid) can in
 *     rare cases differ; a fixed schedule table gives the same bits every run.
 */
#ifndef TRMC_H
#define TRMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRMC_ABI_VERSION 2

#define TRMC_EINVAL (-22)
#define TRMC_ENOMEM (-12)
#define TRMC_ENOSPC (-28)
#define TRMC_EIO (-5)
#define TRMC_EOVERFLOW (-75)
#define TRMC_EBUSY (-16)

/* geometry */
#define TRMC_HOMOG 1  /* one space-homogeneous cell (eq. HOM-r), no transport */
#define TRMC_SLAB1D 2 /* slab [0, length], n_cells equal cells, specular walls */
/* precision */
#define TRMC_FP64 1        /* velocities, positions and all arithmetic in double */
#define TRMC_FP32_MIXED 2  /* float velocities/positions and collision arithmetic;
                              double per-cell sums and conservation rescale */
/* truncation of the collision trees */
#define TRMC_NATURAL 0  /* depth limited only by m_cap */
#define TRMC_FIXED 1    /* depth m_init every step */
#define TRMC_ADAPTIVE 2 /* depth adapted per cell from m_init (Sec. 4.3); a rejected attempt is
                           recomputed at twice the depth */
#define TRMC_ADAPTIVE_REUSE 3 /* as TRMC_ADAPTIVE, but a rejected attempt is kept and the levels
                                 m+1..2m are built on top of it (Sec. 4.3, collisions reused) */
/* tree-shape truncation (Sec. 4.4, TRMC-WB of Alg. 4.6): a final sample whose
   collision tree is longer than wb_mmax is replaced by a Maxwellian sample */
#define TRMC_WB_OFF 0  /* off */
#define TRMC_WB_MIN 1  /* length 1 + min of the two subtrees' lengths (definition def:2) */
#define TRMC_WB_MEAN 2 /* length 1 + mean of the two subtrees' lengths (definition def:3) */
/* VHS majorant of the dummy-collision acceptance (Sec. 4.2, Remark 4.1) */
#define TRMC_MAJORANT_STEP 0  /* sigma(2 dv) of the step's pre-collision velocities for every level;
                                 pairs above it collide with probability 1 and are counted */
#define TRMC_MAJORANT_LEVEL 1 /* raised level by level: level l uses sigma(2 dv_l), dv_l the largest
                                 distance from the cell mean among the pre-step velocities and the
                                 outputs of levels below l (no pair can exceed it); not combined with
                                 TRMC_ADAPTIVE_REUSE or tree-shape truncation */
/* ends of a slab */
#define TRMC_BC_SPECULAR 0 /* specular walls (closed slab) */
#define TRMC_BC_INFLOW 1   /* open slab (Sec. 5.2 stationary shock): each end is a Maxwellian
                              reservoir whose particles enter every step; particles that fly
                              past an end leave.  The particle count changes from step to step. */

typedef struct trmc_ctx trmc_ctx;

/* One instance: a homogeneous solve or a 1-D slab.  Host memory, read at admission. */
typedef struct trmc_desc {
    uint32_t struct_size;   /* sizeof(trmc_desc) (ABI guard) */
    uint32_t seed;          /* Philox key word 0 */
    uint32_t uid;           /* Philox key word 1: a request-stable id, never a slot number */
    uint32_t geometry;      /* TRMC_HOMOG or TRMC_SLAB1D */
    uint64_t n_particles;   /* 2 .. 2^31 */
    uint32_t n_cells;       /* 1 for TRMC_HOMOG; 1 .. 12288 for TRMC_SLAB1D */
    uint32_t precision;     /* TRMC_FP64 or TRMC_FP32_MIXED */
    double length;          /* slab length L, or the volume of a homogeneous instance */
    double dt;              /* time step */
    double particle_weight; /* mass of one particle: rho_c = n_c * weight / (cell volume) */
    double eps;             /* Knudsen number, used when eps_cells is NULL */
    const double* eps_cells;/* host [n_cells] Knudsen number per cell, or NULL */
    double alpha;           /* VHS exponent of B = K |q|^alpha, K = 1/(4 pi): 0 Maxwell molecules, 1 hard spheres */
    uint32_t trunc;         /* TRMC_NATURAL / TRMC_FIXED / TRMC_ADAPTIVE / TRMC_ADAPTIVE_REUSE */
    uint32_t m_init;        /* initial (ADAPTIVE) or fixed (FIXED) depth, >= 1 */
    uint32_t m_cap;         /* maximum depth, 1 .. 2048 */
    uint32_t step0;         /* index of the first step (restart from a saved state) */
    double delta1, delta2;  /* adaptive thresholds, 0 < delta1 < delta2 (Sec. 4.3) */
    const uint32_t* m_state0; /* host [n_cells] saved adaptive depths, or NULL (use m_init) */
    uint32_t wb;            /* TRMC_WB_OFF / TRMC_WB_MIN / TRMC_WB_MEAN; not with the adaptive depth */
    uint32_t wb_mmax;       /* m_max of the tree-shape truncation, >= 1 */
    uint32_t bc;            /* TRMC_BC_SPECULAR or TRMC_BC_INFLOW (TRMC_SLAB1D only) */
    uint32_t n_live0;       /* TRMC_BC_INFLOW: particles present at admission (<= n_particles,
                               which is then the capacity of the arrays); otherwise 0 or n_particles */
    double in_left[3];      /* TRMC_BC_INFLOW: reservoir at x = 0: mass density, mean x velocity, temperature */
    double in_right[3];     /* TRMC_BC_INFLOW: reservoir at x = length (same units; entries move along -x) */
    uint32_t majorant;      /* TRMC_MAJORANT_STEP or TRMC_MAJORANT_LEVEL (only matters for alpha > 0) */
    uint32_t reserved;      /* 0 */
} trmc_desc;

/* Caller-owned device arrays of one instance, SoA, n_particles elements each, of
 * double (TRMC_FP64) or float (TRMC_FP32_MIXED).  x is ignored (may be NULL) for
 * TRMC_HOMOG.  A slab's particles may be in any order and any cell at admission. */
typedef struct trmc_particles {
    void* x;
    void* vx;
    void* vy;
    void* vz;
} trmc_particles;

/* Per-cell moments of the current state (Sec. 2 and 5.1: rho, u, T, P_ii, M4 per
 * unit mass) and counters of the last step (the paper's cost unit of Sec. 5:
 * collisions, and Maxwellian samples). */
typedef struct trmc_cell_moments {
    uint32_t n;            /* particles in the cell */
    uint32_t m_state;      /* adaptive depth for the next step */
    double rho, ux, uy, uz, T, Pxx, Pyy, Pzz, M4;
    uint64_t collisions;   /* collisions of the accepted tree (real + dummy) */
    uint64_t dummies;      /* rejected (dummy) collisions, VHS only */
    uint64_t violations;   /* pairs whose |q|^alpha exceeded the majorant */
    uint64_t work_collisions; /* collisions over all adaptive attempts */
    uint32_t thermalized;  /* particles replaced by Maxwellian samples */
    uint32_t borrowed;     /* leaves taken from the unchanged block */
    uint32_t m_eff;        /* depth of the accepted tree */
    uint32_t m_used;       /* truncation depth of the accepted attempt */
    uint32_t attempts;     /* adaptive attempts (1 = accepted at once) */
    uint32_t N0;           /* particles kept unchanged by the split */
    uint32_t R0;           /* leaves (initial-density samples) used by the trees */
    uint32_t status;       /* 0, or TRMC_CELL_* flags */
    uint32_t wb_thermalized; /* finals replaced by tree shape (included in thermalized) */
    uint32_t reserved;
    double q;              /* exp(-mu dt / eps) = 1 - tau */
    double g;              /* majorant (2 dv)^alpha on the 20-bit grid (TRMC_MAJORANT_LEVEL: of the last level) */
} trmc_cell_moments;

#define TRMC_CELL_OVERFLOW 1u /* scratch too small for this cell's trees: cell left unchanged */

/* Bytes of device workspace needed by these instances (pure, host only): the
 * slab double buffer, sort histograms, per-cell state and collision scratch.
 * Fails with TRMC_EINVAL on an invalid descriptor. */
int trmc_workspace_size(const trmc_desc* descs, uint32_t n_inst, size_t* bytes);

/* Bytes of device workspace of the context itself: instance and work tables for
 * up to max_instances instances and max_cells cells (pure, host only). */
int trmc_ctx_workspace_size(uint32_t max_instances, uint32_t max_cells, size_t* bytes);

/* Create a context holding the given instances, all stepped together by trmc_step.
 * descs/bufs: host arrays of n_inst entries (n_inst may be 0); workspace:
 * caller-owned device memory, 256-byte aligned, of at least
 * trmc_ctx_workspace_size(max_instances, max_cells) + trmc_workspace_size(descs,
 * n_inst) bytes; hip_stream: a hipStream_t (NULL = default stream).  Capacity
 * for later admissions: max_instances (>= n_inst) instances and max_cells cells
 * in total. */
int trmc_init(trmc_ctx** out, const trmc_desc* descs, uint32_t n_inst, const trmc_particles* bufs,
              void* workspace, size_t workspace_bytes, uint32_t max_instances, uint32_t max_cells,
              void* hip_stream);

/* Advance every active instance by n_steps steps (transport, sort, collisions),
 * asynchronously on the context's stream.  When every active instance is
 * space-homogeneous and no cell is on the TILED path, and step fusion is on
 * (trmc_fuse_steps, the default), n_steps > 1 runs as one launch per collision
 * kernel for every 32 steps, in which each cell goes through those steps back to
 * back (a homogeneous cell's step reads nothing but its own previous step); the
 * results are identical to n_steps single steps. */
int trmc_step(trmc_ctx* ctx, uint32_t n_steps);

/* Moments and counters of instance `slot`, one entry per cell (cap >= n_cells).
 * Synchronises the stream. */
int trmc_moments(trmc_ctx* ctx, uint32_t slot, trmc_cell_moments* host_out, uint32_t cap);

/* As trmc_moments, without waiting: the moments and counters of `slot` are
 * computed and written to out[0 .. n_cells) by the device, in stream order.
 * out (cap >= n_cells entries) must be memory the device can write: device
 * memory, or pinned host memory (hipHostMalloc).  Its contents are valid once
 * the stream has passed this call (trmc_sync, or an event recorded after it);
 * the slot's arrays and workspace must stay allocated until then, also when
 * the slot is retired right after.  The serving loop reads the results of
 * finished requests this way, so that the device never waits for the host. */
int trmc_moments_async(trmc_ctx* ctx, uint32_t slot, trmc_cell_moments* out, uint32_t cap);

/* Current device arrays of instance `slot` (a slab alternates between the
 * caller's arrays and a workspace copy; the pointers change after every step). */
int trmc_state(trmc_ctx* ctx, uint32_t slot, trmc_particles* out);

/* Copy the current particles of `slot` to host arrays (any may be NULL), in cell
 * order for a slab; m_state (host [n_cells], may be NULL) receives the adaptive
 * depths; *step receives the index of the next step.  An open slab copies its
 * current count (trmc_count) of particles; the arrays must hold n_particles.
 * Synchronises the stream. */
int trmc_read(trmc_ctx* ctx, uint32_t slot, void* x, void* vx, void* vy, void* vz, uint32_t* m_state,
              uint32_t* step);

/* Number of particles of `slot` now (an open slab's count changes every step;
 * otherwise n_particles).  Synchronises the stream.  TRMC_ENOSPC when an open
 * slab's arrays could not take a step's entering particles (that step injected
 * none). */
int trmc_count(trmc_ctx* ctx, uint32_t slot, uint64_t* n_live);

/* Serving: add one instance while others run.  workspace: its own caller-owned
 * device memory of trmc_workspace_size(desc, 1) bytes.  On success *slot receives
 * the slot number.  TRMC_ENOSPC when the slot table or the cell capacity is full;
 * TRMC_EBUSY when the instance's device memory (workspace plus particle arrays)
 * would take the active instances past the budget of trmc_set_budget. */
int trmc_admit(trmc_ctx* ctx, const trmc_desc* desc, const trmc_particles* buf, void* workspace,
               size_t workspace_bytes, uint32_t* slot);

/* Remove instance `slot` from the active set (its memory is the caller's again
 * once the stream has passed this point).  Admissions and retirements take
 * effect at the next trmc_step, which rebuilds the work lists once for all of
 * them. */
int trmc_retire(trmc_ctx* ctx, uint32_t slot);

/* Batching: the kernel path of each cell, chosen per bucket of the expected
 * particles per cell p of its instance, bucket floor(log2(max(p, 1))) (32
 * buckets).  paths[b] is one of the TRMC_PATH_* values below; n_buckets <= 32
 * entries are read, the rest keep TRMC_PATH_DEFAULT.  A path a cell cannot take
 * (WAVE or TILED with m_cap > 256, TILED for a slab cell) gives it the GROUP
 * path.  Results do not depend on the schedule beyond the rounding order of the
 * FP64 cell sums.  Synchronises the stream; TRMC_EINVAL on an unknown path. */
#define TRMC_SCHED_BUCKETS 32
#define TRMC_PATH_DEFAULT 0u /* library rule: homogeneous cells WAVE below 1024 particles, TILED from
                              * 65536 on, GROUP between; cells of a slab of at least 2048 cells WAVE
                              * up to 4096 particles, GROUP otherwise */
#define TRMC_PATH_GROUP 1u   /* one 512-thread workgroup per cell */
#define TRMC_PATH_WAVE 2u    /* one 64-lane wave per cell, eight cells per workgroup */
#define TRMC_PATH_TILED 3u   /* tile kernels over the cell's slots plus per-cell tree kernels */
int trmc_set_schedule(trmc_ctx* ctx, const uint32_t* paths, uint32_t n_buckets);

/* Current schedule (n_buckets <= 32 entries written). */
int trmc_get_schedule(const trmc_ctx* ctx, uint32_t* paths, uint32_t n_buckets);

/* on != 0: trmc_step replays one captured HIP graph of the step's launches
 * (captured on first use after the work tables change); on == 0: launches each
 * kernel directly.  Both enqueue the same kernels with the same arguments. */
int trmc_use_graph(trmc_ctx* ctx, int on);

/* Batching (a scheduling choice, not a passage of the paper: the step of a
 * space-homogeneous instance, eq. HOM-r, has no transport, so each cell's next
 * step reads only that cell).  on != 0 (the default): trmc_step fuses the steps
 * of a call when it can (see trmc_step); on == 0: one step after another, each
 * its own launches (or graph replay).  Results do not depend on it. */
int trmc_fuse_steps(trmc_ctx* ctx, int on);

/* Admission budget for serving: the device memory (workspace plus particle
 * arrays, as trmc_workspace_size and the descriptor give it) that the active
 * instances of the context may occupy together; 0 (the default) for none.
 * trmc_admit fails with TRMC_EBUSY beyond it; trmc_retire gives an instance's
 * memory back at once (the caller keeps its buffers alive until the stream has
 * passed the instance's last step).  Lowering it retires nothing. */
int trmc_set_budget(trmc_ctx* ctx, uint64_t bytes);

/* Launch order (a scheduling choice, not a passage of the paper).  on != 0 (the
 * default): before each launch of the whole-cell kernels a device kernel sorts
 * their work lists (up to 8192 cells each) by the measured wall-clock duration
 * of every cell's last step, longest first, so that the costliest cells start
 * first and the launch ends on short ones; cells not yet stepped keep the
 * order of expected size.  on == 0: the order of expected size.  Results do not
 * depend on it (every draw is keyed by its cell, not by its position). */
int trmc_order_by_cost(trmc_ctx* ctx, int on);

/* Allocation-free stepping, for callers that cannot allocate (code under stream
 * capture, allocation-free serving loops): n_steps collision steps of ONE
 * space-homogeneous instance, in place on the caller's device arrays b->vx,
 * b->vy, b->vz (b->x unused), enqueued on hip_stream with no host wait, the
 * same as trmc_init + trmc_step(n_steps) on a context holding only this
 * instance (same kernels and kernel path: one wave below 1024 particles when
 * m_cap <= 256, one workgroup otherwise), starting from m_init (adaptive
 * depth) and step0.  Every working buffer (instance record, cell tables,
 * per-cell scratch) lives in a static device array of 64 MiB per device, held
 * until the process ends; no device or pinned memory is allocated.  Calls on
 * one device share that array: calls that overlap on a device (other streams or
 * host threads) race; a call reads nothing that an earlier call left there.
 * No counters or moments are kept: use a context for those.
 * Errors: TRMC_EINVAL for a bad descriptor or buffers, a slab, per-cell eps,
 * saved depths, tree-shape truncation or TRMC_ADAPTIVE_REUSE; TRMC_ENOMEM when
 * the instance's working memory exceeds the static array (about 300,000 FP32
 * or 170,000 FP64 particles); TRMC_EIO for a HIP error.  A cell whose trees
 * exceed its scratch is left unchanged, as in trmc_step. */
int trmc_step_static(const trmc_desc* desc, const trmc_particles* b, uint32_t n_steps, void* hip_stream);

/* Wait for the stream and report any asynchronous error. */
int trmc_sync(trmc_ctx* ctx);

/* Destroy the context (never frees caller memory). */
int trmc_destroy(trmc_ctx* ctx);

const char* trmc_strerror(int status);

/* ABI version compiled into the library. */
int trmc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
