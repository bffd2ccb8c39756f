/*
 * trmc_oracle.c -- plain, serial, FP64 CPU oracle of the recursive time-relaxed
 * Monte Carlo (TRMC-R) step of Trazzi, Pareschi and Wennberg, "Adaptive and
 * Recursive Time Relaxed Monte Carlo methods for rarefied gas dynamics".
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  The GPU library shares no code,
 * header, table or constant with this file; the two sides implement the same
 * written conventions independently.
 *
 * It is written for a reader checking it against the paper, not for speed:
 *   - every floating-point value is a double, contraction is off (-ffp-contract=off);
 *   - one cell at a time, one particle at a time, no blocking and no fusion;
 *   - the steps follow the paper's order: splitting of transport and collision
 *     (Sec. 3.1), the Wild-sum split into collision sets (Alg. 4.2), the recursive
 *     collision trees with the twin store (Alg. 4.3), dummy collisions for VHS
 *     (Alg. 4.4), the Maxwellian remainder (Alg. 4.3 point 5), and the adaptive
 *     choice of the truncation depth (Sec. 4.3).
 *
 * Readings of the paper taken here (each one is also listed in the design notes):
 *   R1  post-collision velocities from eq. (Maxwell_coll-r): v' = c + |q|s/2,
 *       v'_* = c - |q|s/2 (the Sec. 2 display repeats the '+' sign by mistake);
 *   R2  the direction is sigma of eq. (n3d-r), with cos(theta) = 2 xi1 - 1 used
 *       directly instead of acos (same law);
 *   R3  tau = 1 - exp(-mu dt/eps), q = 1 - tau = exp(-mu dt/eps) is used directly;
 *       omega_n / lambda_n of Alg. 4.2 equals q exactly, so N_n = Iround(q * rem);
 *       the loop of Alg. 4.2 is read as "while rem > 0 and n < m";
 *   R4  K = 1/(4 pi) in B = K|q|^alpha, so mu = rho_c * (2 dv)^alpha and the
 *       acceptance test of Alg. 4.4 is xi * g < |q|^alpha with g = (2 dv)^alpha
 *       rounded up to 20 significant bits;
 *   R5  the depth-first recursion of Alg. 4.3 is evaluated in level order: all
 *       requests to a level are known before its own loop runs, consecutive
 *       requests to a level share the two outputs of one collision (the twin
 *       store holds at most one particle), an odd request count leaves one stored
 *       twin that is a final sample, and the level's own loop runs while its
 *       remaining count is positive, two samples per collision;
 *   R6  roles (unchanged, leaf, thermalized) are assigned by a keyed random
 *       permutation; missing leaves are borrowed from the unchanged block in
 *       reverse order, and if even that is not enough the deepest level is folded
 *       into the remainder;
 *   R7  the Maxwellian remainder is sampled by Box-Muller, the sample of a
 *       thermalized particle keyed by its slot, and then affinely rescaled to
 *       the removed particles' momentum and energy (exact conservation); a
 *       remainder of at most one particle is left unchanged,
 *       and a normal sample with zero spread (not reachable in practice) puts
 *       the remainder at the removed mean;
 *   R8  adaptive depth (Sec. 4.3) uses S = P_xx per unit mass, the analytic
 *       Maxwellian estimate for the thermalized part, halving (at least 1) below
 *       delta1, keeping between delta1 and delta2, and recomputing from the
 *       pre-step velocities at twice the depth above delta2 (same keyed draws);
 *       no recompute when it cannot change the result: at m_cap, when the
 *       split left no remainder, or when continuing the split from the
 *       remainder would put no particle in any level up to m_cap (the deeper
 *       trees are then those of depth m);
 *   R9  transport (1-D slab, specular walls) then a stable counting sort by cell,
 *       then the collision step (first-order splitting of Sec. 3.1);
 *   R15 tree-shape truncation (Sec. 4.4, TRMC-WB of Alg. 4.6): a leaf has length
 *       0 and both outputs of a collision whose inputs have lengths a and b have
 *       length 1 + min(a, b) (definition def:2) or 1 + (a + b)/2 (def:3), the
 *       latter in double as fl(fl(a + b) * 0.5) + 1; the lengths depend on the
 *       tree schedule only, so they are known before any collision.  A final
 *       sample whose length exceeds m_max is thermalized: its slot joins the
 *       Maxwellian remainder of R7.  Every scheduled collision is still
 *       evaluated (twins make trees share collisions), and the dropped final
 *       joins the removed set whose momentum and energy the rescale keeps, so
 *       the step stays conservative.  Twin outputs share a length, so they are
 *       thermalized together.  Not combined with the adaptive depth (the
 *       paper leaves that combination open);
 *   R16 adaptive depth with reuse (ORC_ADAPTIVE_REUSE, the efficient form of
 *       Sec. 4.3): a rejected attempt at depth m is kept, with its collisions,
 *       leaves and finals; the attempt at 2m splits with the same draws, takes
 *       the levels 1..m as done (no own samples), and builds the trees of the
 *       levels m+1..2m in level order on top: their requests to levels <= m are
 *       served by new collisions whose draw indices continue after the earlier
 *       ones, their leaves are the next roles of the pool, and their finals
 *       continue the leaf ranks.  An odd request count at a done level leaves
 *       one more final of that level.  Leaves running out fold only the new
 *       levels.  Counters add up over the attempts; nothing is discarded;
 *   R17 open slab for the stationary shock (Sec. 5.2): each end is a reservoir
 *       with a Maxwellian state (rho, u, T).  Per step, before transport, each
 *       end injects floor(lambda + U) particles, lambda the expected number that
 *       cross inward in dt, (rho / weight) sigma (phi(a) + a Phi(a)) dt with a the
 *       inward drift over sigma = sqrt(T); the inward normal speed is drawn from
 *       the flux-weighted half-range law by inverting its distribution function,
 *       the tangential ones from the Maxwellian, and the particle is placed
 *       outside by the part of the step it has not yet flown.  Particles beyond
 *       either end after transport are removed.  The left end enters along +x:
 *       the sign of the paper's inflow velocity only chooses the side.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) with
 * key {seed, uid} and counter {index, tag<<24 | aux, cell, step}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "trmc_oracle.h"

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from its published definition.                              */
/* ------------------------------------------------------------------------- */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void orc_philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * c0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * c2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { TAG_SPLIT = 1, TAG_PERM = 2, TAG_TREE = 3, TAG_COLL = 4, TAG_MAXW = 5, TAG_INJ = 6 };

typedef struct {
    uint32_t seed, uid, cell, step;
} stream_key;

static void draw(const stream_key* s, uint32_t index, uint32_t tag, uint32_t aux, uint32_t out[4])
{
    uint32_t ctr[4] = {index, (tag << 24) | (aux & 0xFFFFFFu), s->cell, s->step};
    orc_philox(ctr, s->seed, s->uid, out);
}

/* Uniform in [0,1) from 53 bits: the high word gives the top 21 bits. */
static double unif53(uint32_t hi, uint32_t lo)
{
    uint64_t bits = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return (double)bits * 0x1.0p-53;
}

/* ------------------------------------------------------------------------- */
/* exp(-x) by a fixed written algorithm so that both implementations of the   */
/* method obtain the same bits for q = exp(-mu dt / eps):                     */
/* Cody-Waite reduction x = k ln2 + r with ln2 split into a 21-bit head and a */
/* tail, then the degree-13 Taylor polynomial of e^r by Horner, then 2^k.     */
/* ------------------------------------------------------------------------- */
double orc_exp_neg(double x)
{
    const double ln2_head = 0x1.62e42p-1;          /* 0.6931467056274414 */
    const double ln2_tail = 0x1.fdf473de6af28p-22; /* ln 2 - ln2_head */
    const double inv_ln2 = 0x1.71547652b82fep+0;
    if (!(x >= 0.0)) return x != x ? x : 1.0; /* NaN stays NaN; negative input is not used */
    if (x > 746.0) return 0.0;
    double y = -x;
    double k = floor(y * inv_ln2 + 0.5);
    double r = (y - k * ln2_head) - k * ln2_tail;
    double p = 1.0 / 6227020800.0; /* 1/13! */
    p = p * r + 1.0 / 479001600.0; /* 1/12! */
    p = p * r + 1.0 / 39916800.0;  /* 1/11! */
    p = p * r + 1.0 / 3628800.0;   /* 1/10! */
    p = p * r + 1.0 / 362880.0;    /* 1/9!  */
    p = p * r + 1.0 / 40320.0;     /* 1/8!  */
    p = p * r + 1.0 / 5040.0;      /* 1/7!  */
    p = p * r + 1.0 / 720.0;       /* 1/6!  */
    p = p * r + 1.0 / 120.0;       /* 1/5!  */
    p = p * r + 1.0 / 24.0;        /* 1/4!  */
    p = p * r + 1.0 / 6.0;         /* 1/3!  */
    p = p * r + 0.5;               /* 1/2!  */
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

/* Round a positive double up to 20 significant bits (majorant grid). */
double orc_grid_up(double g)
{
    uint64_t bits;
    memcpy(&bits, &g, sizeof bits);
    const uint64_t low = (1ull << 33) - 1ull;
    if (bits & low) bits = (bits | low) + 1ull;
    memcpy(&g, &bits, sizeof g);
    return g;
}

/* Iround of Alg. 4.2: floor(y) + 1 with probability y - floor(y). */
static uint64_t iround(double y, double u)
{
    double f = floor(y);
    return (uint64_t)f + (u < y - f ? 1u : 0u);
}

/* Whether the split of Alg. 4.2, continued past level m with the remainder rem,
 * would leave levels m+1..m_cap all empty (then a deeper attempt builds the same
 * trees as depth m).  The draws are those the split at a deeper depth uses. */
static int split_extension_empty(const stream_key* key, double q, uint64_t rem, uint32_t m, uint32_t m_cap)
{
    for (uint32_t k = m + 1; k <= m_cap; ++k) {
        uint32_t w[4];
        draw(key, k, TAG_SPLIT, 0, w);
        if (iround(q * (double)rem, unif53(w[0], w[1])) != 0) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Keyed permutation of [0, n): a 6-round alternating Feistel network on b    */
/* bits, b = max(8, ceil(log2 n)), with cycle walking.  A value is split into */
/* a high part of ceil(b/2) bits and a low part of floor(b/2) bits; round i   */
/* xors F(low) into the high part when i is even and F(high) into the low     */
/* part when i is odd.  Round i uses the key word k[i mod 4] xor              */
/* (i * 0x9E3779B9); F(x) = mix24(x xor key), where mix24 multiplies the low  */
/* 24 bits by 0xEBCA6B (keeping the low 32 bits of the product), xors in its  */
/* value shifted right by 15, multiplies the low 24 bits by 0xB2AE35 and      */
/* xors in its value shifted right by 13.                                     */
/* ------------------------------------------------------------------------- */
static uint32_t mul24(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu)) & 0xFFFFFFFFull);
}

static uint32_t mix24(uint32_t x)
{
    uint32_t h = mul24(x, 0xEBCA6Bu);
    h ^= h >> 15;
    h = mul24(h, 0xB2AE35u);
    h ^= h >> 13;
    return h;
}

static uint32_t perm_bits(uint32_t n)
{
    uint32_t b = 0;
    while (b < 32 && ((uint64_t)1 << b) < (uint64_t)n) ++b;
    return b < 8 ? 8 : b;
}

static uint32_t feistel_once(uint32_t x, uint32_t b, const uint32_t k[4])
{
    uint32_t lo = b / 2, hi = b - lo;
    uint32_t mlo = (uint32_t)(((uint64_t)1 << lo) - 1u), mhi = (uint32_t)(((uint64_t)1 << hi) - 1u);
    uint32_t H = x >> lo, W = x & mlo;
    for (uint32_t i = 0; i < 6; ++i) {
        uint32_t rk = k[i & 3u] ^ (i * 0x9E3779B9u);
        if ((i & 1u) == 0) H ^= mix24(W ^ rk) & mhi;
        else W ^= mix24(H ^ rk) & mlo;
    }
    return (H << lo) | W;
}

uint32_t orc_perm(uint32_t i, uint32_t n, const uint32_t k[4])
{
    uint32_t b = perm_bits(n);
    uint32_t x = feistel_once(i, b, k);
    while (x >= n) x = feistel_once(x, b, k);
    return x;
}

/* ------------------------------------------------------------------------- */
/* Per-cell collision step                                                    */
/* ------------------------------------------------------------------------- */
typedef struct { double x, y, z; } vec3;

typedef struct {
    /* per level l = 0..me (arrays sized cap_levels) */
    uint64_t* N;     /* collision-set sizes N_0..N_{me+1} */
    uint64_t* R;     /* requests received by level l */
    uint64_t* C;     /* collisions at level l */
    uint64_t* first; /* index of level l's first collision in the lists below */
    uint64_t* F;     /* finals of level l */
    /* per collision */
    uint32_t* jch;   /* sub-level choice j of the collision */
    uint64_t* rA;    /* rank of request A at level j */
    uint64_t* rB;    /* rank of request B at level l-1-j */
    uint64_t ncoll, cap_coll;
    uint32_t me;
    uint64_t R0;
} tree_t;

static void* xrealloc(void* p, size_t bytes)
{
    void* q = realloc(p, bytes ? bytes : 1);
    if (!q) abort();
    return q;
}

static void tree_push(tree_t* t, uint32_t j, uint64_t ra, uint64_t rb)
{
    if (t->ncoll == t->cap_coll) {
        t->cap_coll = t->cap_coll ? 2 * t->cap_coll : 1024;
        t->jch = xrealloc(t->jch, t->cap_coll * sizeof *t->jch);
        t->rA = xrealloc(t->rA, t->cap_coll * sizeof *t->rA);
        t->rB = xrealloc(t->rB, t->cap_coll * sizeof *t->rB);
    }
    t->jch[t->ncoll] = j;
    t->rA[t->ncoll] = ra;
    t->rB[t->ncoll] = rb;
    t->ncoll++;
}

/* Sub-level choice for collision c of level l: k uniform in {0..l-1}
 * (Alg. 4.1 / 4.3: "choose k with equal probability"). */
static uint32_t tree_choice(const stream_key* s, uint32_t l, uint64_t c)
{
    uint32_t w[4];
    draw(s, (uint32_t)(c >> 2), TAG_TREE, l, w);
    return (uint32_t)(((uint64_t)w[c & 3u] * (uint64_t)l) >> 32);
}

/* Level-order evaluation of the recursive sampler (reading R5).  Levels are
 * visited from the deepest down.  Requests to a level come only from deeper
 * levels, so when level l is visited its request count R_l is final:
 *   - ceil(R_l/2) collisions serve the requests (consecutive requests take the
 *     two outputs of one collision: the second takes the stored twin);
 *   - if R_l is odd the last stored twin is a final sample of level l, which
 *     counts against N_l; the level's own loop then runs while the remaining
 *     count is positive, producing two samples per collision;
 *   - each collision chooses j uniformly in {0..l-1} and asks level j and level
 *     l-1-j for one input each, in that order.
 * Returns R_0, the number of leaves (initial-density samples) needed. */
static void tree_build(tree_t* t, const stream_key* s, const uint64_t* coff)
{
    uint32_t me = t->me;
    for (uint32_t l = 0; l <= me; ++l) { t->R[l] = 0; t->C[l] = 0; t->F[l] = 0; t->first[l] = 0; }
    t->ncoll = 0;
    for (uint32_t l = me; l >= 1; --l) {
        uint64_t Rl = t->R[l];
        uint64_t odd = Rl & 1u;
        uint64_t Nl = t->N[l];
        uint64_t own = (Nl > odd) ? (Nl - odd + 1) / 2 : 0; /* loop "while N_l > 0", 2 per collision */
        uint64_t Cl = (Rl + 1) / 2 + own;
        t->C[l] = Cl;
        t->first[l] = t->ncoll;
        for (uint64_t c = 0; c < Cl; ++c) {
            /* coff: collisions of level l in earlier attempts (reuse, reading R16) */
            uint32_t j = tree_choice(s, l, (coff ? coff[l] : 0) + c);
            uint64_t ra = t->R[j]++;
            uint64_t rb = t->R[l - 1 - j]++;
            tree_push(t, j, ra, rb);
        }
        t->F[l] = 2 * Cl - Rl;
    }
    t->R0 = t->R[0];
}

/* Collision of eq. (Maxwell_coll-r) with sigma of eq. (n3d-r); for alpha > 0 a
 * dummy collision (Alg. 4.4) unless xi_acc * g < |q|^alpha. */
static int collide(vec3 a, vec3 b, double xi1, double xi2, double xacc, double alpha, double g,
                   vec3* oa, vec3* ob, uint64_t* violations)
{
    vec3 q = {a.x - b.x, a.y - b.y, a.z - b.z};
    double qn = sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
    if (alpha != 0.0) {
        double s = (alpha == 1.0) ? qn : pow(qn, alpha);
        if (s > g) (*violations)++;
        if (!(xacc * g < s)) {
            *oa = a;
            *ob = b;
            return 0;
        }
    }
    double ct = 2.0 * xi1 - 1.0;
    double st2 = 1.0 - ct * ct;
    double st = sqrt(st2 > 0.0 ? st2 : 0.0);
    double phi = 6.283185307179586 * xi2;
    double sx = cos(phi) * st, sy = sin(phi) * st, sz = ct;
    double h = 0.5 * qn;
    vec3 c = {0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z)};
    oa->x = c.x + h * sx; oa->y = c.y + h * sy; oa->z = c.z + h * sz;
    ob->x = c.x - h * sx; ob->y = c.y - h * sy; ob->z = c.z - h * sz;
    return 1;
}

/* Three standard normals for the thermalized particle in slot t (Box-Muller). */
static vec3 maxw_normals(const stream_key* s, uint64_t t)
{
    uint32_t b0[4], b1[4];
    draw(s, (uint32_t)t, TAG_MAXW, 0, b0);
    draw(s, (uint32_t)t, TAG_MAXW, 1, b1);
    double u0 = unif53(b0[0], b1[0]), u1 = unif53(b0[1], b1[1]);
    double u2 = unif53(b0[2], b1[2]), u3 = unif53(b0[3], b1[3]);
    double r1 = sqrt(-2.0 * log(1.0 - u0));
    double r2 = sqrt(-2.0 * log(1.0 - u2));
    double a1 = 6.283185307179586 * u1, a2 = 6.283185307179586 * u3;
    vec3 z = {r1 * cos(a1), r1 * sin(a1), r2 * cos(a2)};
    return z;
}

typedef struct {
    uint32_t N0, half;
    uint64_t n, P, R0, borrowed, n_th;
    uint32_t pk[4];
} roles_t;

/* Slot of leaf r (reading R6). */
static uint32_t leaf_slot(const roles_t* ro, uint64_t r)
{
    if (r < ro->P) return orc_perm((uint32_t)(ro->N0 + r), (uint32_t)ro->n, ro->pk);
    return orc_perm((uint32_t)(ro->N0 - 1 - (r - ro->P)), (uint32_t)ro->n, ro->pk);
}

static uint32_t therm_slot(const roles_t* ro, uint64_t t)
{
    return orc_perm((uint32_t)(ro->N0 + ro->R0 + t), (uint32_t)ro->n, ro->pk);
}

static uint32_t kept_slot(const roles_t* ro, uint64_t i)
{
    return orc_perm((uint32_t)i, (uint32_t)ro->n, ro->pk);
}

typedef struct {
    const stream_key* key;
    double rho_factor; /* rho_c = n * rho_factor */
    double dt, eps, alpha;
    int trunc;
    uint32_t m_init, m_cap;
    double delta1, delta2;
    uint32_t wb, wb_mmax; /* tree-shape truncation (reading R15): ORC_WB_* and m_max */
    uint32_t majorant;    /* ORC_MAJ_STEP, or ORC_MAJ_LEVEL: the bound raised level by level (Remark 4.1) */
} cell_params;

/* One collision step of one cell, in place on v[0..n). */
/* Length of a sample made by one collision from inputs of lengths a and b
 * (Sec. 4.4): definition def:2 (ORC_WB_MIN) or def:3 (ORC_WB_MEAN). */
static double wb_len(double a, double b, uint32_t kind)
{
    if (kind == ORC_WB_MIN) return 1.0 + (a < b ? a : b);
    return (a + b) * 0.5 + 1.0;
}

/* Lengths of the final samples of a built tree (reading R15), in the order in
 * which the collision loop below lists the finals: level 1 first, within a
 * level by output rank.  lens[l] holds the lengths of level l's outputs. */
static void tree_lengths(const tree_t* t, uint32_t kind, double** lens, double* finlen)
{
    uint64_t nf = 0;
    for (uint32_t l = 1; l <= t->me; ++l) {
        lens[l] = xrealloc(lens[l], sizeof(double) * (size_t)(2 * t->C[l] + 1));
        for (uint64_t c = 0; c < t->C[l]; ++c) {
            uint64_t id = t->first[l] + c;
            uint32_t j = t->jch[id], h = l - 1 - j;
            double a = (j == 0) ? 0.0 : lens[j][t->rA[id]];
            double b = (h == 0) ? 0.0 : lens[h][t->rB[id]];
            double L = wb_len(a, b, kind);
            lens[l][2 * c] = L;
            lens[l][2 * c + 1] = L;
        }
        for (uint64_t o = t->R[l]; o < 2 * t->C[l]; ++o) finlen[nf++] = lens[l][o];
    }
}

static __thread orc_attempt* g_alog;
static __thread uint64_t g_alog_cap, g_alog_n;

uint64_t orc_attempt_log(orc_attempt* buf, uint64_t cap)
{
    const uint64_t n = g_alog_n;
    g_alog = buf;
    g_alog_cap = buf ? cap : 0;
    g_alog_n = 0;
    return n;
}

static void cell_step(const cell_params* cp, uint32_t n, vec3* v, uint32_t* m_state, orc_cell_record* rec)
{
    memset(rec, 0, sizeof *rec);
    rec->n = n;
    rec->m_state_after = *m_state;
    if (n < 2) return;
    const stream_key* key = cp->key;

    /* Moments of the cell before the step: mean, dv = max |v_i - mean|, S = P_xx. */
    vec3 mean = {0, 0, 0};
    for (uint32_t i = 0; i < n; ++i) { mean.x += v[i].x; mean.y += v[i].y; mean.z += v[i].z; }
    mean.x /= n; mean.y /= n; mean.z /= n;
    double dv2 = 0.0, Sn = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        double dx = v[i].x - mean.x, dy = v[i].y - mean.y, dz = v[i].z - mean.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 > dv2) dv2 = d2;
        Sn += dx * dx;
    }
    Sn /= n;

    /* Majorant and relaxation parameter (Sec. 4.2; tau of Sec. 3.2). */
    double g = 1.0;
    if (cp->alpha != 0.0) {
        double two_dv = 2.0 * sqrt(dv2);
        g = orc_grid_up(cp->alpha == 1.0 ? two_dv : pow(two_dv, cp->alpha));
    }
    double rho = (double)n * cp->rho_factor;
    double mu = rho * g;
    double xarg = mu * cp->dt / cp->eps;
    double q = orc_exp_neg(xarg);
    rec->q = q;
    rec->g = g;

    uint32_t m;
    const int reuse = cp->trunc == ORC_ADAPTIVE_REUSE;
    const int adaptive = cp->trunc == ORC_ADAPTIVE || reuse;
    if (cp->trunc == ORC_FIXED) m = cp->m_init;
    else if (adaptive) m = *m_state;
    else m = cp->m_cap;
    if (m < 1) m = 1;
    if (m > cp->m_cap) m = cp->m_cap;

    uint32_t pk[4];
    draw(key, 0, TAG_PERM, 0, pk);

    size_t cap_levels = (size_t)cp->m_cap + 2;
    tree_t T;
    memset(&T, 0, sizeof T);
    T.N = calloc(cap_levels, sizeof *T.N);
    T.R = calloc(cap_levels, sizeof *T.R);
    T.C = calloc(cap_levels, sizeof *T.C);
    T.first = calloc(cap_levels, sizeof *T.first);
    T.F = calloc(cap_levels, sizeof *T.F);
    vec3* leaf = malloc(sizeof(vec3) * n);
    vec3* fin = malloc(sizeof(vec3) * n);
    vec3* wth = malloc(sizeof(vec3) * n);
    vec3** out = calloc(cap_levels, sizeof *out);
    double** lens = calloc(cap_levels, sizeof *lens);
    double* finlen = malloc(sizeof(double) * n);
    uint8_t* wbth = malloc(n);
    uint32_t* thslot = malloc(sizeof(uint32_t) * n);
    vec3* thv = malloc(sizeof(vec3) * n);
    if (!T.N || !T.R || !T.C || !T.first || !T.F || !leaf || !fin || !wth || !out || !lens || !finlen || !wbth ||
        !thslot || !thv)
        abort();

    uint64_t work_coll = 0;
    uint64_t nth_acc = 0; /* thermalized slots of the accepted attempt */
    /* Reuse of rejected attempts (reading R16): levels 1..mprev are done, their
     * collisions kept; cprev[l] counts level l's collisions so far (draw offset);
     * leaf and final ranks continue from R0prev. */
    uint64_t* cprev = calloc(cap_levels, sizeof *cprev);
    if (!cprev) abort();
    uint64_t R0prev = 0, coll_acc = 0;
    uint32_t mprev = 0, folds_acc = 0;
    uint32_t attempts = 0;
    roles_t ro;
    uint64_t dummies = 0, viol = 0;
    for (;;) {
        attempts++;
        /* Split into collision sets (Alg. 4.2, reading R3). */
        uint32_t w[4];
        draw(key, 0, TAG_SPLIT, 0, w);
        uint64_t N0 = iround(q * (double)n, unif53(w[0], w[1]));
        uint64_t rem = (uint64_t)n - N0;
        uint32_t k = 0;
        T.N[0] = N0;
        while (rem > 0 && k < m) {
            ++k;
            draw(key, k, TAG_SPLIT, 0, w);
            uint64_t Nk = iround(q * (double)rem, unif53(w[0], w[1]));
            T.N[k] = Nk;
            rem -= Nk;
        }
        uint64_t split_rem = rem;
        T.me = k;
        T.N[k + 1] = rem;
        /* Reuse: the samples of levels 1..mprev were made by earlier attempts. */
        if (reuse)
            for (uint32_t l = 1; l <= mprev && l <= T.me; ++l) T.N[l] = 0;

        /* Collision trees (Alg. 4.3, reading R5); fold if the leaves run out. */
        uint32_t folds = 0;
        for (;;) {
            tree_build(&T, key, reuse ? cprev : NULL);
            if (R0prev + T.R0 <= n || T.me <= mprev) break;
            T.N[T.me] += T.N[T.me + 1];
            T.me -= 1;
            folds++;
        }

        ro.n = n;
        ro.N0 = (uint32_t)N0;
        ro.P = (uint64_t)n - N0;
        ro.R0 = R0prev + T.R0;
        ro.borrowed = ro.R0 > ro.P ? ro.R0 - ro.P : 0;
        ro.n_th = ro.R0 < ro.P ? ro.P - ro.R0 : 0;
        memcpy(ro.pk, pk, sizeof pk);
        if (g_alog && g_alog_n < g_alog_cap) {
            orc_attempt* a = &g_alog[g_alog_n++];
            a->n = n;
            a->N0 = (uint32_t)N0;
            a->m = m;
            a->me = T.me;
            a->mprev = mprev;
            a->folds = folds;
            a->R0prev = R0prev;
            a->R0 = T.R0;
            a->ncoll = T.ncoll;
            a->sum_R = 0;
            a->max_C = 0;
            a->coff_max = 0;
            for (uint32_t l = 1; l <= T.me; ++l) {
                a->sum_R += T.R[l];
                if (T.C[l] > a->max_C) a->max_C = T.C[l];
                const uint64_t co = (reuse ? cprev[l] : 0) + T.C[l];
                if (co > a->coff_max) a->coff_max = co;
            }
            a->borrowed = ro.borrowed;
            a->n_th = ro.n_th;
        }

        /* Tree-shape truncation (reading R15): finals whose tree is longer than
         * m_max are thermalized; the decision needs the schedule only. */
        uint64_t n_wb = 0;
        memset(wbth, 0, n);
        if (cp->wb != ORC_WB_OFF) {
            tree_lengths(&T, cp->wb, lens, finlen);
            for (uint64_t r = 0; r < T.R0; ++r)
                if (finlen[r] > (double)cp->wb_mmax) { wbth[r] = 1; n_wb++; }
        }

        /* Leaves: initial-density samples, i.e. the particles' current velocities. */
        for (uint64_t r = R0prev; r < ro.R0; ++r) leaf[r] = v[leaf_slot(&ro, r)];

        /* Collisions, shallowest level first; outputs of level l are out[l][0..2C_l). */
        if (!reuse) {
            dummies = 0;
            viol = 0;
        }
        uint64_t nf = 0;
        /* Majorant of the collisions (reading R18).  ORC_MAJ_STEP: the step's bound
         * sigma(2 dv) for every level.  ORC_MAJ_LEVEL (Remark 4.1: the bound
         * updated as the collisions change the velocities): the bound of level l
         * is sigma(2 dv_l), dv_l the largest distance from the cell mean among
         * the pre-step velocities and the outputs of levels 1..l-1, from which
         * level l takes its inputs; no pair can then exceed it. */
        double gl = g, d2seen = dv2;
        for (uint32_t l = 1; l <= T.me; ++l) {
            if (cp->majorant == ORC_MAJ_LEVEL && l > 1 && cp->alpha != 0.0) {
                double two_dv = 2.0 * sqrt(d2seen);
                gl = orc_grid_up(cp->alpha == 1.0 ? two_dv : pow(two_dv, cp->alpha));
            }
            out[l] = xrealloc(out[l], sizeof(vec3) * (size_t)(2 * T.C[l] + 1));
            for (uint64_t c = 0; c < T.C[l]; ++c) {
                uint64_t id = T.first[l] + c;
                uint32_t j = T.jch[id], h = l - 1 - j;
                vec3 a = (j == 0) ? leaf[R0prev + T.rA[id]] : out[j][T.rA[id]];
                vec3 b = (h == 0) ? leaf[R0prev + T.rB[id]] : out[h][T.rB[id]];
                uint32_t b0[4], b1[4];
                uint32_t cg = (uint32_t)((reuse ? cprev[l] : 0) + c);
                draw(key, cg, TAG_COLL, l | (0u << 20), b0);
                draw(key, cg, TAG_COLL, l | (1u << 20), b1);
                double xi1 = unif53(b0[0], b1[0]);
                double xi2 = unif53(b0[1], b1[1]);
                double xacc = unif53(b0[2], b1[2]);
                if (!collide(a, b, xi1, xi2, xacc, cp->alpha, gl, &out[l][2 * c], &out[l][2 * c + 1], &viol))
                    dummies++;
            }
            if (cp->majorant == ORC_MAJ_LEVEL) {
                for (uint64_t o = 0; o < 2 * T.C[l]; ++o) {
                    double dx = out[l][o].x - mean.x, dy = out[l][o].y - mean.y, dz = out[l][o].z - mean.z;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 > d2seen) d2seen = d2;
                }
            }
            /* Finals of level l: the outputs no deeper request took. */
            for (uint64_t o = T.R[l]; o < 2 * T.C[l]; ++o) fin[R0prev + nf++] = out[l][o];
        }
        /* nf == R0 by construction: every output is either taken or final. */
        if (nf != T.R0) abort();
        work_coll += T.ncoll;

        /* Maxwellian remainder (reading R7) over the thermalized slots: the
         * split's remainder, then the finals thermalized by tree shape (R15).
         * The removed velocities are the remainder's pre-step ones and the
         * dropped finals, so the rescale keeps the cell's momentum and energy. */
        uint64_t nth = 0;
        for (uint64_t t = 0; t < ro.n_th; ++t) {
            thslot[nth] = therm_slot(&ro, t);
            thv[nth++] = v[therm_slot(&ro, t)];
        }
        for (uint64_t r = 0; r < T.R0; ++r)
            if (wbth[r]) {
                thslot[nth] = leaf_slot(&ro, r);
                thv[nth++] = fin[r];
            }
        vec3 ur = {0, 0, 0};
        double Eth = 0.0;
        if (nth >= 2) {
            for (uint64_t t = 0; t < nth; ++t) {
                vec3 a = thv[t];
                ur.x += a.x; ur.y += a.y; ur.z += a.z;
            }
            ur.x /= (double)nth; ur.y /= (double)nth; ur.z /= (double)nth;
            for (uint64_t t = 0; t < nth; ++t) {
                vec3 a = thv[t];
                double dx = a.x - ur.x, dy = a.y - ur.y, dz = a.z - ur.z;
                Eth += dx * dx + dy * dy + dz * dz;
            }
            vec3 zm = {0, 0, 0};
            for (uint64_t t = 0; t < nth; ++t) {
                wth[t] = maxw_normals(key, thslot[t]);
                zm.x += wth[t].x; zm.y += wth[t].y; zm.z += wth[t].z;
            }
            zm.x /= (double)nth; zm.y /= (double)nth; zm.z /= (double)nth;
            double Z = 0.0;
            for (uint64_t t = 0; t < nth; ++t) {
                double dx = wth[t].x - zm.x, dy = wth[t].y - zm.y, dz = wth[t].z - zm.z;
                Z += dx * dx + dy * dy + dz * dz;
            }
            double a = Z > 0.0 ? sqrt(Eth / Z) : 0.0;
            for (uint64_t t = 0; t < nth; ++t) {
                if (Z > 0.0) {
                    wth[t].x = ur.x + a * (wth[t].x - zm.x);
                    wth[t].y = ur.y + a * (wth[t].y - zm.y);
                    wth[t].z = ur.z + a * (wth[t].z - zm.z);
                } else {
                    wth[t] = ur; /* degenerate normal sample: the removed mean (momentum kept) */
                }
            }
        } else {
            for (uint64_t t = 0; t < nth; ++t) wth[t] = thv[t];
        }

        rec->N0 = (uint32_t)N0;
        rec->m_eff = T.me;
        rec->m_used = m;
        rec->R0 = (uint32_t)ro.R0;
        nth_acc = nth;
        rec->n_th = (uint32_t)nth;
        rec->wb_th = (uint32_t)n_wb;
        rec->borrowed = (uint32_t)ro.borrowed;
        rec->folds = folds_acc + folds;
        rec->collisions = coll_acc + T.ncoll;
        rec->dummies = dummies;
        rec->violations = viol;
        rec->g = gl; /* the bound of the last level */

        if (!adaptive) break;

        /* Adaptive depth (Sec. 4.3, reading R8). */
        double Snew = 0.0;
        uint64_t kept = (uint64_t)N0 - ro.borrowed;
        for (uint64_t i = 0; i < kept; ++i) {
            double d = v[kept_slot(&ro, i)].x - mean.x;
            Snew += d * d;
        }
        for (uint64_t r = 0; r < ro.R0; ++r) {
            double d = fin[r].x - mean.x;
            Snew += d * d;
        }
        if (ro.n_th >= 2) {
            double d = ur.x - mean.x;
            Snew += Eth / 3.0 + (double)ro.n_th * d * d;
        } else {
            for (uint64_t t = 0; t < ro.n_th; ++t) {
                double d = wth[t].x - mean.x;
                Snew += d * d;
            }
        }
        Snew /= n;
        if (Sn == 0.0) { *m_state = m; break; }
        double E1 = fabs(Snew - Sn) / fabs(Sn);
        rec->E1 = E1;
        if (E1 < cp->delta1) { *m_state = m / 2 > 1 ? m / 2 : 1; break; }
        if (E1 <= cp->delta2) { *m_state = m; break; }
        if (m >= cp->m_cap || split_rem == 0 || split_extension_empty(key, q, split_rem, m, cp->m_cap)) {
            *m_state = m;
            break;
        }
        if (reuse) {
            for (uint32_t l = 1; l <= T.me; ++l) cprev[l] += T.C[l];
            R0prev = ro.R0;
            mprev = m;
            coll_acc += T.ncoll;
            folds_acc += folds;
        }
        m = 2 * m < cp->m_cap ? 2 * m : cp->m_cap;
    }
    free(cprev);

    /* Write the accepted result: leaf slots take the finals, thermalized slots
     * take the rescaled Maxwellian samples, the rest are unchanged. */
    for (uint64_t r = 0; r < ro.R0; ++r)
        if (!wbth[r]) v[leaf_slot(&ro, r)] = fin[r];
    for (uint64_t t = 0; t < nth_acc; ++t) v[thslot[t]] = wth[t];

    rec->attempts = attempts;
    rec->work_collisions = work_coll;
    rec->m_state_after = *m_state;

    for (size_t l = 0; l < cap_levels; ++l) { free(out[l]); free(lens[l]); }
    free(out); free(lens); free(finlen); free(wbth); free(thslot); free(thv); free(leaf); free(fin); free(wth);
    free(T.N); free(T.R); free(T.C); free(T.first); free(T.F);
    free(T.jch); free(T.rA); free(T.rB);
}

/* ------------------------------------------------------------------------- */
/* Free flight in the slab [0, L] with specular walls (reading R9).           */
/* ------------------------------------------------------------------------- */
uint32_t orc_transport(double* x, double* vx, double dt, double L, uint32_t n_cells)
{
    double xn = fma(*vx, dt, *x);
    double u = *vx;
    for (int it = 0; (xn < 0.0 || xn > L) && it < 64; ++it) {
        if (xn < 0.0) xn = -xn;
        else xn = 2.0 * L - xn;
        u = -u;
    }
    if (xn < 0.0) xn = 0.0; /* at most 64 wall crossings per step; only non-finite input gets here */
    if (xn > L) xn = L;
    *x = xn;
    *vx = u;
    double inv_dx = (double)n_cells / L;
    double cf = floor(xn * inv_dx);
    uint32_t c = cf < 0.0 ? 0u : (cf >= (double)n_cells ? n_cells - 1u : (uint32_t)cf);
    return c;
}

/* ------------------------------------------------------------------------- */
/* Driver                                                                     */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* Open slab (reading R17): reservoirs at both ends.                          */
/* ------------------------------------------------------------------------- */
static double std_phi(double t) { return exp(-0.5 * t * t) * 0.3989422804014327; /* 1/sqrt(2 pi) */ }
static double std_Phi(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }

/* Distribution of w = v_n / sigma for the particles of a Maxwellian of drift
 * a sigma (along the inward normal) that cross a wall inward in unit time: the
 * density is proportional to w phi(w - a) on w > 0.  F is its integral from 0
 * to w; Z = F(infinity) = phi(a) + a Phi(a). */
static double flux_cdf(double w, double a)
{
    return (std_phi(a) - std_phi(w - a)) + a * (std_Phi(w - a) - std_Phi(-a));
}
static double flux_norm(double a) { return std_phi(a) + a * std_Phi(a); }

/* Inverse of F at u Z, by 64 bisection steps on [0, max(a, 0) + 12]. */
double orc_flux_inverse(double a, double u)
{
    double target = u * flux_norm(a);
    double lo = 0.0, hi = (a > 0.0 ? a : 0.0) + 12.0;
    for (int it = 0; it < 64; ++it) {
        double mid = 0.5 * (lo + hi);
        if (flux_cdf(mid, a) < target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Expected number of simulation particles entering through one end in one
 * step: (rho / weight) * sigma * Z(a) * dt, a = u_in / sigma. */
double orc_inflow_mean(double rho, double u_in, double T, double weight, double dt)
{
    double sigma = sqrt(T);
    return rho / weight * sigma * flux_norm(u_in / sigma) * dt;
}

/* Particles entering in one step, appended after the n live ones: left end
 * first, then right end.  Each enters at a uniform time of the step, so it is
 * placed outside the slab by the part of the step it has not yet flown.
 * Returns -2 if the arrays are full (nothing injected). */
static int inject(const orc_desc* d, uint32_t step, uint64_t* n, uint64_t cap, double* x, double* vx, double* vy,
                  double* vz)
{
    uint64_t k[2];
    double sig[2], a[2];
    for (int side = 0; side < 2; ++side) {
        const double* st = side == 0 ? d->in_left : d->in_right;
        stream_key key = {d->seed, d->uid, 0xFFFFFFF0u + (uint32_t)side, step};
        sig[side] = sqrt(st[2]);
        double u_in = side == 0 ? st[1] : -st[1]; /* drift along the inward normal */
        a[side] = u_in / sig[side];
        double lam = orc_inflow_mean(st[0], u_in, st[2], d->weight, d->dt);
        uint32_t w[4];
        draw(&key, 0, TAG_INJ, 2, w);
        k[side] = (uint64_t)floor(lam + unif53(w[0], w[1]));
    }
    if (*n + k[0] + k[1] > cap) return -2;
    uint64_t at = *n;
    for (int side = 0; side < 2; ++side) {
        stream_key key = {d->seed, d->uid, 0xFFFFFFF0u + (uint32_t)side, step};
        for (uint64_t i = 0; i < k[side]; ++i) {
            uint32_t b0[4], b1[4];
            draw(&key, (uint32_t)i, TAG_INJ, 0, b0);
            draw(&key, (uint32_t)i, TAG_INJ, 1, b1);
            double u0 = unif53(b0[0], b1[0]), u1 = unif53(b0[1], b1[1]);
            double u2 = unif53(b0[2], b1[2]), u3 = unif53(b0[3], b1[3]);
            double vn = sig[side] * orc_flux_inverse(a[side], u0);
            double v = side == 0 ? vn : -vn;
            double r = sqrt(-2.0 * log(1.0 - u2));
            double ph = 6.283185307179586 * u3;
            x[at] = side == 0 ? -v * d->dt * u1 : d->length - v * d->dt * u1;
            vx[at] = v;
            vy[at] = sig[side] * (r * cos(ph));
            vz[at] = sig[side] * (r * sin(ph));
            at++;
        }
    }
    *n = at;
    return 0;
}

/* Free flight out of an open slab: a particle beyond either end has left. */
static uint32_t transport_open(double* x, double vx, double dt, double L, uint32_t n_cells)
{
    double xn = fma(vx, dt, *x);
    *x = xn;
    if (xn < 0.0 || xn > L) return n_cells; /* gone */
    double cf = floor(xn * ((double)n_cells / L));
    return cf >= (double)n_cells ? n_cells - 1u : (uint32_t)cf;
}

int orc_run(const orc_desc* d, uint64_t* n_io, uint64_t cap, double* x, double* vx, double* vy, double* vz,
            uint32_t* m_state, uint32_t step0, uint32_t n_steps, orc_cell_record* rec,
            uint32_t* cell_counts)
{
    if (!d || !n_io || !vx || !vy || !vz || !m_state) return -1;
    uint64_t n = *n_io;
    uint32_t nc = d->geometry == ORC_SLAB ? d->n_cells : 1u;
    if (nc == 0) return -1;
    if (d->geometry == ORC_SLAB && !x) return -1;
    if (d->bc > ORC_BC_INFLOW || (d->bc == ORC_BC_INFLOW && d->geometry != ORC_SLAB)) return -1;
    if (d->bc == ORC_BC_INFLOW) {
        for (int side = 0; side < 2; ++side) {
            const double* st = side == 0 ? d->in_left : d->in_right;
            if (!(st[0] > 0.0) || !(st[2] > 0.0) || !isfinite(st[1])) return -1;
        }
    } else if (cap != n) {
        return -1;
    }
    if (n > cap) return -1;
    if (d->trunc > ORC_ADAPTIVE_REUSE) return -1;
    if (d->wb > ORC_WB_MEAN || (d->wb != ORC_WB_OFF && (d->trunc >= ORC_ADAPTIVE || d->wb_mmax < 1))) return -1;
    if (d->majorant > ORC_MAJ_LEVEL ||
        (d->majorant == ORC_MAJ_LEVEL && (d->wb != ORC_WB_OFF || d->trunc == ORC_ADAPTIVE_REUSE)))
        return -1;
    double volume = d->geometry == ORC_SLAB ? d->length / (double)nc : d->length;
    double rho_factor = d->weight / volume;

    uint32_t* cell = malloc(sizeof(uint32_t) * (cap ? cap : 1));
    uint64_t* count = calloc((size_t)nc + 2, sizeof(uint64_t));
    double* tmp = malloc(sizeof(double) * (cap ? cap : 1));
    vec3* cv = malloc(sizeof(vec3) * (cap ? cap : 1));
    if (!cell || !count || !tmp || !cv) abort();
    const int open = d->bc == ORC_BC_INFLOW;

    for (uint32_t s = 0; s < n_steps; ++s) {
        uint32_t step = step0 + s;
        uint64_t* start = count;
        if (d->geometry == ORC_SLAB) {
            /* Open ends: the reservoirs' particles enter first (reading R17). */
            if (open && inject(d, step, &n, cap, x, vx, vy, vz) != 0) {
                free(cell); free(count); free(tmp); free(cv);
                return -2;
            }
            /* Transport, then a stable counting sort by cell; with open ends the
             * particles that left go to bucket nc and are dropped. */
            for (uint64_t i = 0; i < n; ++i)
                cell[i] = open ? transport_open(&x[i], vx[i], d->dt, d->length, nc)
                               : orc_transport(&x[i], &vx[i], d->dt, d->length, nc);
            memset(count, 0, sizeof(uint64_t) * ((size_t)nc + 2));
            for (uint64_t i = 0; i < n; ++i) count[cell[i] + 1]++;
            for (uint32_t c = 0; c < nc + (uint32_t)open; ++c) count[c + 1] += count[c];
            uint64_t* pos = malloc(sizeof(uint64_t) * (nc + 1));
            if (!pos) abort();
            double* arrs[4] = {x, vx, vy, vz};
            for (int a = 0; a < 4; ++a) {
                memcpy(pos, count, sizeof(uint64_t) * (nc + 1));
                for (uint64_t i = 0; i < n; ++i) tmp[pos[cell[i]]++] = arrs[a][i];
                memcpy(arrs[a], tmp, sizeof(double) * n);
            }
            free(pos);
            n = count[nc]; /* particles still in the slab */
        } else {
            count[0] = 0;
            count[1] = n;
        }
        for (uint32_t c = 0; c < nc; ++c) {
            uint64_t off = start[c], cnt = start[c + 1] - start[c];
            stream_key key = {d->seed, d->uid, c, step};
            cell_params cp = {&key, rho_factor, d->dt, d->eps_cells ? d->eps_cells[c] : d->eps,
                              d->alpha, d->trunc, d->m_init, d->m_cap, d->delta1, d->delta2,
                              d->wb, d->wb_mmax, d->majorant};
            for (uint64_t i = 0; i < cnt; ++i) {
                cv[i].x = vx[off + i]; cv[i].y = vy[off + i]; cv[i].z = vz[off + i];
            }
            orc_cell_record r;
            cell_step(&cp, (uint32_t)cnt, cv, &m_state[c], &r);
            for (uint64_t i = 0; i < cnt; ++i) {
                vx[off + i] = cv[i].x; vy[off + i] = cv[i].y; vz[off + i] = cv[i].z;
            }
            if (rec) rec[c] = r;
            if (cell_counts) cell_counts[c] = (uint32_t)cnt;
        }
    }
    free(cell); free(count); free(tmp); free(cv);
    *n_io = n;
    return 0;
}

/* Per-cell moments (Sec. 2: rho, u, T; Sec. 5.1: P_ii and M4), per unit mass
 * except rho. */
void orc_moments(uint64_t n, const double* vx, const double* vy, const double* vz, double rho_factor,
                 double out[9])
{
    double u[3] = {0, 0, 0};
    for (uint64_t i = 0; i < n; ++i) { u[0] += vx[i]; u[1] += vy[i]; u[2] += vz[i]; }
    double P[3] = {0, 0, 0}, m4 = 0.0;
    if (n > 0) { u[0] /= n; u[1] /= n; u[2] /= n; }
    for (uint64_t i = 0; i < n; ++i) {
        double dx = vx[i] - u[0], dy = vy[i] - u[1], dz = vz[i] - u[2];
        P[0] += dx * dx; P[1] += dy * dy; P[2] += dz * dz;
        double s = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        m4 += s * s;
    }
    double inv = n > 0 ? 1.0 / (double)n : 0.0;
    out[0] = (double)n * rho_factor;
    out[1] = u[0]; out[2] = u[1]; out[3] = u[2];
    out[4] = (P[0] + P[1] + P[2]) * inv / 3.0;
    out[5] = P[0] * inv; out[6] = P[1] * inv; out[7] = P[2] * inv;
    out[8] = m4 * inv;
}

/* Test hooks: the split and the tree counts of one cell for given n, q, m. */
int orc_split(uint32_t seed, uint32_t uid, uint32_t cell, uint32_t step, uint32_t n, double q, uint32_t m,
              uint64_t* N_out /* m+2 */, uint32_t* m_eff_out)
{
    stream_key key = {seed, uid, cell, step};
    uint32_t w[4];
    draw(&key, 0, TAG_SPLIT, 0, w);
    uint64_t N0 = iround(q * (double)n, unif53(w[0], w[1]));
    uint64_t rem = (uint64_t)n - N0;
    uint32_t k = 0;
    N_out[0] = N0;
    while (rem > 0 && k < m) {
        ++k;
        draw(&key, k, TAG_SPLIT, 0, w);
        uint64_t Nk = iround(q * (double)rem, unif53(w[0], w[1]));
        N_out[k] = Nk;
        rem -= Nk;
    }
    for (uint32_t i = k + 1; i <= m + 1; ++i) N_out[i] = 0;
    N_out[k + 1] = rem;
    *m_eff_out = k;
    return 0;
}

/* Collision hook: outputs of one collision for given inputs and uniforms. */
int orc_collide(const double a[3], const double b[3], double xi1, double xi2, double xacc, double alpha,
                double g, double oa[3], double ob[3])
{
    vec3 A = {a[0], a[1], a[2]}, B = {b[0], b[1], b[2]}, OA, OB;
    uint64_t viol = 0;
    int acc = collide(A, B, xi1, xi2, xacc, alpha, g, &OA, &OB, &viol);
    oa[0] = OA.x; oa[1] = OA.y; oa[2] = OA.z;
    ob[0] = OB.x; ob[1] = OB.y; ob[2] = OB.z;
    return acc;
}

/* Test hook: the tree schedule of one cell for given n, q, m (reading R5) and
 * the lengths of its finals (reading R15; kind ORC_WB_MIN or ORC_WB_MEAN).
 * Arrays: R, C, first [m+2]; jch, rA, rB [cap_coll]; finlen [n].  Returns the
 * number of collisions, or -1 if cap_coll is too small. */
int64_t orc_tree(uint32_t seed, uint32_t uid, uint32_t cell, uint32_t step, uint32_t n, double q, uint32_t m,
                 uint32_t kind, uint64_t* R, uint64_t* C, uint64_t* first, uint32_t* jch, uint64_t* rA,
                 uint64_t* rB, uint64_t cap_coll, double* finlen, uint32_t* me_out, uint64_t* R0_out)
{
    stream_key key = {seed, uid, cell, step};
    size_t cap_levels = (size_t)m + 2;
    tree_t T;
    memset(&T, 0, sizeof T);
    T.N = calloc(cap_levels, sizeof *T.N);
    T.R = calloc(cap_levels, sizeof *T.R);
    T.C = calloc(cap_levels, sizeof *T.C);
    T.first = calloc(cap_levels, sizeof *T.first);
    T.F = calloc(cap_levels, sizeof *T.F);
    double** lens = calloc(cap_levels, sizeof *lens);
    if (!T.N || !T.R || !T.C || !T.first || !T.F || !lens) abort();
    uint32_t me = 0;
    orc_split(seed, uid, cell, step, n, q, m, T.N, &me);
    T.me = me;
    for (;;) {
        tree_build(&T, &key, NULL);
        if (T.R0 <= n) break;
        T.N[T.me] += T.N[T.me + 1];
        T.me -= 1;
    }
    int64_t rc = (int64_t)T.ncoll;
    if (T.ncoll > cap_coll) {
        rc = -1;
    } else {
        for (uint32_t l = 0; l <= T.me; ++l) { R[l] = T.R[l]; C[l] = T.C[l]; first[l] = T.first[l]; }
        memcpy(jch, T.jch, sizeof(uint32_t) * T.ncoll);
        memcpy(rA, T.rA, sizeof(uint64_t) * T.ncoll);
        memcpy(rB, T.rB, sizeof(uint64_t) * T.ncoll);
        if (kind != ORC_WB_OFF) tree_lengths(&T, kind, lens, finlen);
        *me_out = T.me;
        *R0_out = T.R0;
    }
    for (size_t l = 0; l < cap_levels; ++l) free(lens[l]);
    free(lens); free(T.N); free(T.R); free(T.C); free(T.first); free(T.F);
    free(T.jch); free(T.rA); free(T.rB);
    return rc;
}

/* Test hook: the length rule of Sec. 4.4 for one collision. */
double orc_wb_len(double a, double b, uint32_t kind)
{
    return wb_len(a, b, kind);
}
