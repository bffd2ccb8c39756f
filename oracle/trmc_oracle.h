/*
 * trmc_oracle.h -- interface of the FP64 CPU oracle (test infrastructure only).
 * Private to oracle/: the GPU library neither includes nor links this file.
 */
#ifndef TRMC_ORACLE_H
#define TRMC_ORACLE_H
#include <stdint.h>

enum { ORC_HOMOG = 1, ORC_SLAB = 2 };
enum { ORC_NATURAL = 0, ORC_FIXED = 1, ORC_ADAPTIVE = 2, ORC_ADAPTIVE_REUSE = 3 };
enum { ORC_WB_OFF = 0, ORC_WB_MIN = 1, ORC_WB_MEAN = 2 }; /* tree-shape truncation, Sec. 4.4 */
enum { ORC_BC_SPECULAR = 0, ORC_BC_INFLOW = 1 };          /* slab ends: walls or reservoirs */
enum { ORC_MAJ_STEP = 0, ORC_MAJ_LEVEL = 1 };             /* VHS majorant: per step, or raised per level */

typedef struct {
    uint32_t seed, uid;
    uint32_t geometry;   /* ORC_HOMOG: one cell; ORC_SLAB: [0, length] split in n_cells */
    uint32_t n_cells;
    double length;       /* slab length, or the volume of a homogeneous instance */
    double dt;
    double weight;       /* mass carried by one particle: rho_c = n_c * weight / V_c */
    double eps;          /* Knudsen number when eps_cells is NULL */
    const double* eps_cells;
    double alpha;        /* VHS exponent: 0 Maxwell molecules, 1 hard spheres */
    uint32_t trunc, m_init, m_cap;
    double delta1, delta2;
    uint32_t wb;         /* ORC_WB_OFF, or thermalize finals longer than wb_mmax under def:2 / def:3 */
    uint32_t wb_mmax;
    uint32_t bc;         /* ORC_BC_SPECULAR, or ORC_BC_INFLOW: reservoirs at both ends of a slab */
    double in_left[3], in_right[3]; /* reservoir states (rho, u, T); u along +x */
    uint32_t majorant;   /* ORC_MAJ_STEP, or ORC_MAJ_LEVEL (Remark 4.1; not with reuse or tree shape) */
} orc_desc;

typedef struct {
    uint32_t n, N0, m_eff, m_used, attempts, R0, n_th, borrowed, folds, m_state_after;
    uint32_t wb_th;      /* finals thermalized by tree shape (included in n_th) */
    uint64_t collisions, dummies, violations, work_collisions;
    double q, g, E1;
} orc_cell_record;

/* Integer outline of one attempt of a cell's step (after its folds), recorded
 * while a log is set on the calling thread: what a kernel's index arithmetic
 * has to hold.  sum_R = sum of the requests over levels 1..me; max_C = most
 * collisions of one level; coff_max = largest draw offset of a level after the
 * attempt (reuse). */
typedef struct {
    uint32_t n, N0, m, me, mprev, folds;
    uint64_t R0prev, R0, ncoll, sum_R, max_C, coff_max, borrowed, n_th;
} orc_attempt;

/* Record the attempts of the cell steps this thread runs into buf (at most cap;
 * NULL stops recording); returns the number recorded since the last call. */
uint64_t orc_attempt_log(orc_attempt* buf, uint64_t cap);

void orc_philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]);
double orc_exp_neg(double x);
double orc_grid_up(double g);
uint32_t orc_perm(uint32_t i, uint32_t n, const uint32_t k[4]);
uint32_t orc_transport(double* x, double* vx, double dt, double L, uint32_t n_cells);
double orc_flux_inverse(double a, double u);
double orc_inflow_mean(double rho, double u_in, double T, double weight, double dt);
int orc_run(const orc_desc* d, uint64_t* n_io, uint64_t cap, double* x, double* vx, double* vy, double* vz,
            uint32_t* m_state, uint32_t step0, uint32_t n_steps, orc_cell_record* rec,
            uint32_t* cell_counts);
void orc_moments(uint64_t n, const double* vx, const double* vy, const double* vz, double rho_factor,
                 double out[9]);
int orc_split(uint32_t seed, uint32_t uid, uint32_t cell, uint32_t step, uint32_t n, double q, uint32_t m,
              uint64_t* N_out, uint32_t* m_eff_out);
int64_t orc_tree(uint32_t seed, uint32_t uid, uint32_t cell, uint32_t step, uint32_t n, double q, uint32_t m,
                 uint32_t kind, uint64_t* R, uint64_t* C, uint64_t* first, uint32_t* jch, uint64_t* rA,
                 uint64_t* rB, uint64_t cap_coll, double* finlen, uint32_t* me_out, uint64_t* R0_out);
double orc_wb_len(double a, double b, uint32_t kind);
int orc_collide(const double a[3], const double b[3], double xi1, double xi2, double xacc, double alpha,
                double g, double oa[3], double ob[3]);

#endif
