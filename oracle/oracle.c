/*
 * oracle.c -- plain CPU FP64 oracle for the operator-split multicellular
 * stochastic simulation (Coulier & Hellander, "Orchestral").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU library.
 *
 * What it computes, and the passage each part follows:
 *   - one splitting interval = internal dynamics chi for every cell
 *     independently, then the pairwise signalling operator S
 *     (Algorithm section, "A parallel framework", the splitting assumption;
 *     Fig. 1 caption: chi first, then S, every timestep);
 *   - chi: per-cell stochastic reaction-diffusion over the cell's voxels
 *     (Introduction: Gillespie's SSA and the RDME as admissible
 *     single-cell modules; "Internal cell dynamics module");
 *   - S: molecules of two adjacent cells near their common face react
 *     pairwise, each pair independently ("Cell signaling module";
 *     "Translation scripts": T_chi->S gathers the molecules near the shared
 *     boundary, T_S->chi reports products back to the target cell);
 *   - each face-near molecule is handed to exactly one face's signalling
 *     model (Results, Setup, Model: coupling through a single face);
 *   - cells are arranged in a 2D layer with at most four neighbours on the
 *     square lattice (Results, Setup, Model).
 * The paper leaves the SSA's summation order, random stream, log and
 * tie rules open; this file follows the numerical contract written out in
 * the design notes (geometry conventions, Philox counter layout, plog,
 * sum tree, selection rules).  Every step is done the plain way: leaves are
 * recomputed from the counts and the whole internal tree is rebuilt after
 * every event; the S channels are all recomputed after every event.
 *
 * Built with: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction;
 * fma() only where plog says so).
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11, the Philox family).  N=4 words of W=32 bits,
 * R=10 rounds.  Each round: two 32x32->64 products of words 0 and 2 with
 * the multipliers, the high halves xored with the other two words and the
 * round key, the words permuted; the key is bumped by the Weyl constants
 * between rounds.
 * ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u /* floor(2^32 * (golden ratio - 1)) */
#define PHILOX_W1 0xBB67AE85u /* floor(2^32 * (sqrt(3) - 1)) */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Two uniforms from one Philox output block:
 * m1 = (w0:w1) >> 11, m2 = (w2:w3) >> 11 (53-bit integers);
 * U1 = (m1 + 1) * 2^-53 in (0, 1], U2 = m2 * 2^-53 in [0, 1). */
void oracle_uniforms(const uint32_t w[4], double *u1, double *u2)
{
    uint64_t m1 = ((((uint64_t)w[0]) << 32) | (uint64_t)w[1]) >> 11;
    uint64_t m2 = ((((uint64_t)w[2]) << 32) | (uint64_t)w[3]) >> 11;
    const double two_m53 = 1.0 / 9007199254740992.0; /* 2^-53, exact */
    *u1 = (double)(m1 + 1u) * two_m53;
    *u2 = (double)m2 * two_m53;
}

/* One draw of unit `unit` (cell or edge) at draw ordinal j of global step n.
 * Counter = (j, n, unit, sim_id << 2 | tag); key = (lo32 seed, hi32 seed). */
static void draw_pair(uint64_t seed, uint32_t sim_id, uint32_t tag,
                      uint32_t unit, uint32_t step, uint32_t j,
                      double *u1, double *u2)
{
    uint32_t ctr[4] = { j, step, unit, (sim_id << 2) | tag };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    oracle_uniforms(w, u1, u2);
}

/* ------------------------------------------------------------------------
 * plog(x), x in [2^-53, 1]: natural log from the identity
 * log m = 2 atanh((m-1)/(m+1)) = 2 (s + s^3/3 + s^5/5 + ...),
 * with x = m 2^k, m folded into (sqrt2/2, sqrt2], and the result
 * reconstructed as k ln2 + log m with ln2 split in a head and a tail
 * (argument reduction as in J.-M. Muller, "Elementary Functions").
 * Series kept to l = 11: 2/(2l+3) z^l, l = 0..11, so the truncation error
 * is below 2^-60 relative on the reduced range.
 * ------------------------------------------------------------------------ */
double oracle_plog(double x)
{
    /* decompose x = m * 2^k, m in [1, 2) */
    int e;
    double fr = frexp(x, &e);        /* fr in [0.5, 1), x = fr * 2^e, exact */
    double m = fr * 2.0;             /* exact */
    int k = e - 1;
    const double sqrt2 = 1.4142135623730951; /* RN(sqrt(2)) */
    if (m > sqrt2) {
        m = m * 0.5;                 /* exact */
        k = k + 1;
    }
    double f = m - 1.0;              /* exact (Sterbenz) */
    double s = f / (2.0 + f);
    double z = s * s;
    /* coefficients 2/(2l+3), each the correctly rounded quotient */
    static const double c[12] = {
        2.0 / 3.0,  2.0 / 5.0,  2.0 / 7.0,  2.0 / 9.0,
        2.0 / 11.0, 2.0 / 13.0, 2.0 / 15.0, 2.0 / 17.0,
        2.0 / 19.0, 2.0 / 21.0, 2.0 / 23.0, 2.0 / 25.0 };
    double p = c[11];
    for (int l = 10; l >= 0; --l)
        p = fma(p, z, c[l]);
    double q = fma(s * z, p, 2.0 * s);
    const double ln2_hi = 0x1.62e42fefa39efp-1;  /* RN(ln 2) */
    const double ln2_lo = 0x1.abc9e3b39803fp-56; /* RN(ln 2 - ln2_hi) */
    double dk = (double)k;
    return fma(dk, ln2_hi, fma(dk, ln2_lo, q));
}

/* ------------------------------------------------------------------------
 * Geometry (conventions; the paper only fixes "2D layer, at most four
 * neighbours" and "a single face per molecule").
 * ------------------------------------------------------------------------ */

/* Voxel neighbours of v = y*w + x in the order (-x, +x, -y, +y), present
 * ones only.  Returns the degree. */
int oracle_voxel_neighbours(int w, int h, int v, int *nb)
{
    int x = v % w, y = v / w, deg = 0;
    if (x > 0)     nb[deg++] = v - 1;
    if (x < w - 1) nb[deg++] = v + 1;
    if (y > 0)     nb[deg++] = v - w;
    if (y < h - 1) nb[deg++] = v + w;
    return deg;
}

/* Membrane ring: clockwise (y pointing down) from the top-right corner:
 * right column downwards, bottom row leftwards, left column upwards,
 * top row rightwards; a voxel already on the ring is skipped. */
int oracle_ring(int w, int h, int *ring)
{
    int seen[64];
    int n = 0;
    memset(seen, 0, sizeof(seen));
#define RING_ADD(xx, yy) do { int vv = (yy) * w + (xx); \
        if (!seen[vv]) { seen[vv] = 1; ring[n++] = vv; } } while (0)
    for (int y = 0; y <= h - 1; ++y) RING_ADD(w - 1, y);
    for (int x = w - 2; x >= 0; --x) RING_ADD(x, h - 1);
    for (int y = h - 2; y >= 0; --y) RING_ADD(0, y);
    for (int x = 1; x <= w - 2; ++x) RING_ADD(x, 0);
#undef RING_ADD
    return n;
}

/* Face group of lattice direction d among nd directions: a contiguous
 * slice ring[floor(d M / nd) : floor((d+1) M / nd)]; when that slice is
 * empty, the single voxel ring[floor(d M / nd) mod M]. */
int oracle_face_group(int w, int h, int nd, int d, int *g)
{
    int ring[64];
    int M = oracle_ring(w, h, ring);
    int lo = (d * M) / nd, hi = ((d + 1) * M) / nd;
    int m = 0;
    if (hi > lo) {
        for (int t = lo; t < hi; ++t) g[m++] = ring[t];
    } else {
        g[m++] = ring[lo % M];
    }
    return m;
}

/* Lattice neighbour of cell (x, y) in direction d, or -1 (open boundary).
 * Square: 0 +x, 1 +y, 2 -x, 3 -y.
 * Hex (axial rhombus q = x, r = y): 0 E(+1,0), 1 SE(0,+1), 2 SW(-1,+1),
 *   3 W(-1,0), 4 NW(0,-1), 5 NE(+1,-1). */
int oracle_lattice_neighbour(int lattice, int nx, int ny, int cell, int d)
{
    static const int sq[4][2] = { {1, 0}, {0, 1}, {-1, 0}, {0, -1} };
    static const int hx[6][2] = { {1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1} };
    int x = cell % nx, y = cell / nx;
    int dx = lattice == 0 ? sq[d][0] : hx[d][0];
    int dy = lattice == 0 ? sq[d][1] : hx[d][1];
    int X = x + dx, Y = y + dy;
    if (X < 0 || X >= nx || Y < 0 || Y >= ny) return -1;
    return Y * nx + X;
}

/* Edges: one per adjacent pair, taken in a forward direction d
 * (square {0,1}, hex {0,1,2}) so that j > i.  Colour = 2 d + parity, the
 * parity being x mod 2 for d = 0 and y mod 2 for the other forward
 * directions; each colour class is a matching.  Edges are ranked by
 * (colour, i).  Returns the number of edges; arrays may be NULL to count. */
int oracle_lattice_edges(int lattice, int nx, int ny,
                         int32_t *ei, int32_t *ej, int32_t *ed, int32_t *ecol)
{
    int nfwd = lattice == 0 ? 2 : 3;
    int ncol = 2 * nfwd;
    int E = 0;
    for (int col = 0; col < ncol; ++col) {
        int d = col / 2, par = col % 2;
        for (int i = 0; i < nx * ny; ++i) {
            int x = i % nx, y = i / nx;
            int p = (d == 0) ? (x % 2) : (y % 2);
            if (p != par) continue;
            int j = oracle_lattice_neighbour(lattice, nx, ny, i, d);
            if (j < 0) continue;
            if (ei) { ei[E] = i; ej[E] = j; ed[E] = d; ecol[E] = col; }
            ++E;
        }
    }
    return E;
}

/* ------------------------------------------------------------------------
 * Problem description and run
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t lattice;          /* 0 square, 1 hex */
    int32_t nx, ny;
    const int32_t *mesh_w;    /* [n_cells] */
    const int32_t *mesh_h;    /* [n_cells] */
    int32_t n_species;
    int32_t n_reactions;
    const int32_t *reactants; /* [R][2], species or -1 */
    const int32_t *stoich;    /* [R][S] */
    const double *rates;      /* [R] */
    const double *diffusion;  /* [S] */
    int32_t trans_n, trans_d, trans_i; /* see signal_order */
    int32_t signal_order;     /* 2: N_i + D_j -> I_i (no S when trans_n < 0);
                                 1: D_i -> I_j into the facing voxel (no S when
                                 trans_d < 0) */
    double trans_rate;
    uint64_t seed;
    uint32_t sim_id;
    uint32_t start_step;
    uint32_t event_cap;       /* events per unit-step before the unit stops */
    uint32_t scheme;          /* 0 Lie: S o chi; 1 Strang: chi/2 o S o chi/2 */
    /* Per-cell networks (several models updating different cells, the
     * multi-fidelity use the paper's Discussion describes): n_models > 1
     * and cell_model[c] in [0, n_models).  Model m's tables, padded to 16
     * reactions: m_n_reactions[m], m_reactants[m][16][2], m_stoich[m][16][S],
     * m_rates[m][16], m_diffusion[m][S]; model 0 equals the fields above.
     * The S reaction's species are the same for every cell; under
     * first-order signalling each molecule signals at its own cell's
     * model's rate, m_signal_rate[m] (m_signal_rate[0] = trans_rate). */
    int32_t n_models;
    int32_t pad2;
    const int32_t *cell_model;
    const int32_t *m_n_reactions;
    const int32_t *m_reactants;
    const int32_t *m_stoich;
    const double *m_rates;
    const double *m_diffusion;
    const double *m_signal_rate;
} oracle_problem;

/* First-order signalling rate of cell c's molecules. */
static double cell_signal_rate(const oracle_problem *p, int c)
{
    return p->n_models > 1 ? p->m_signal_rate[p->cell_model[c]] : p->trans_rate;
}

/* The problem as seen by cell c: its own model's network. */
static oracle_problem cell_view(const oracle_problem *p, int c)
{
    oracle_problem v = *p;
    if (p->n_models > 1) {
        const int m = p->cell_model[c], S = p->n_species;
        v.n_reactions = p->m_n_reactions[m];
        v.reactants = p->m_reactants + (size_t)m * 16 * 2;
        v.stoich = p->m_stoich + (size_t)m * 16 * S;
        v.rates = p->m_rates + (size_t)m * 16;
        v.diffusion = p->m_diffusion + (size_t)m * S;
    }
    return v;
}

typedef struct {
    uint64_t chi_events, s_events, draws;
    uint32_t overflow;        /* a count left [0, 2^26) */
    uint32_t capped;          /* a unit-step reached event_cap */
} oracle_stats;

#define COUNT_LIMIT (1 << 26)

/* mass-action propensity of reaction r in voxel counts x[] */
static double reaction_propensity(const oracle_problem *p, int r, const int32_t *x)
{
    int a = p->reactants[2 * r], b = p->reactants[2 * r + 1];
    double c = p->rates[r];
    if (a < 0 && b < 0) return c;
    if (a < 0 || b < 0) {
        int s = a < 0 ? b : a;
        return c * (double)(int64_t)x[s];
    }
    if (a == b) {
        int64_t xa = x[a];
        return c * (double)(xa * (xa - 1) / 2);
    }
    return c * (double)((int64_t)x[a] * (int64_t)x[b]);
}

/* Channels of voxel v: the reactions in order, then one aggregated
 * diffusion channel per species with D_s > 0 (only when the voxel has a
 * neighbour), propensity D_s * (x_s * deg). */
static int voxel_channels(const oracle_problem *p, const int32_t *x, int deg,
                          double *a, int *kind, int *spec)
{
    int K = 0;
    for (int r = 0; r < p->n_reactions; ++r) {
        a[K] = reaction_propensity(p, r, x);
        kind[K] = 0; spec[K] = r; ++K;
    }
    if (deg > 0) {
        for (int s = 0; s < p->n_species; ++s) {
            if (!(p->diffusion[s] > 0.0)) continue;
            a[K] = p->diffusion[s] * (double)((int64_t)x[s] * (int64_t)deg);
            kind[K] = 1; spec[K] = s; ++K;
        }
    }
    return K;
}

/* voxel propensity: left fold over the channels, from 0.0 */
static double voxel_propensity(const oracle_problem *p, const int32_t *x, int deg)
{
    double a[64]; int kind[64], spec[64];
    int K = voxel_channels(p, x, deg, a, kind, spec);
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc = acc + a[k];
    return acc;
}

/* Selection within a list of channel propensities given residual r:
 * the first channel with a_k > 0 and r < (prefix through k); if none,
 * the last channel with a_k > 0.  Returns the channel and its residual. */
static int select_channel(const double *a, int K, double r, double *resid)
{
    double prefix = 0.0;
    int last = -1;
    double last_prefix = 0.0;
    for (int k = 0; k < K; ++k) {
        double next = prefix + a[k];
        if (a[k] > 0.0) {
            if (r < next) { *resid = r - prefix; return k; }
            last = k; last_prefix = prefix;
        }
        prefix = next;
    }
    *resid = r - last_prefix;
    return last;
}

static int next_pow2(int v)
{
    int P = 1;
    while (P < v) P *= 2;
    return P;
}

static void set_flag(uint32_t *flag)
{
#ifdef _OPENMP
#pragma omp atomic write
#endif
    *flag = 1u;
}

static void check_count(int32_t v, uint32_t *flag)
{
    if (v < 0 || v >= COUNT_LIMIT) set_flag(flag);
}

/* One chi step of one cell: direct method over the cell's voxels, over the
 * interval [0, dt), clock restarted at 0 every step. */
static void chi_cell_step(const oracle_problem *p, int cell, int w, int h,
                          int32_t *cnt, double dt, uint32_t step, uint32_t tag,
                          uint64_t *events_out, uint64_t *draws_out,
                          double *last_t_out, uint32_t *overflow, uint32_t *capped)
{
    const int S = p->n_species;
    const int V = w * h;
    const int P = next_pow2(V);
    double tree[2 * 64];
    int nb[4];

    double t = 0.0;
    uint32_t j = 0;           /* draw ordinal */
    uint64_t events = 0;
    for (;;) {
        /* rebuild the tree: leaves from the counts, internal nodes as the
         * pairwise sums tree[n] = tree[2n] + tree[2n+1] */
        for (int v = 0; v < P; ++v) {
            if (v < V) {
                int deg = oracle_voxel_neighbours(w, h, v, nb);
                tree[P + v] = voxel_propensity(p, cnt + v * S, deg);
            } else {
                tree[P + v] = 0.0;
            }
        }
        for (int n = P - 1; n >= 1; --n) tree[n] = tree[2 * n] + tree[2 * n + 1];
        double a0 = tree[1];
        if (a0 == 0.0) break;
        if (events >= p->event_cap) { set_flag(capped); break; }

        double u1, u2;
        draw_pair(p->seed, p->sim_id, tag, (uint32_t)cell, step, j, &u1, &u2);
        ++j;
        double tau = (-oracle_plog(u1)) / a0;
        double tn = t + tau;
        if (tn >= dt) break;
        t = tn;
        double r = u2 * a0;

        /* descend the sum tree */
        int n = 1;
        while (n < P) {
            double L = tree[2 * n], R = tree[2 * n + 1];
            if (r < L || R == 0.0) {
                n = 2 * n;
            } else {
                r = r - L;
                n = 2 * n + 1;
            }
        }
        int v = n - P;

        /* channel within the voxel */
        int deg = oracle_voxel_neighbours(w, h, v, nb);
        double a[64]; int kind[64], spec[64];
        int K = voxel_channels(p, cnt + v * S, deg, a, kind, spec);
        double resid;
        int k = select_channel(a, K, r, &resid);

        if (kind[k] == 0) {
            int rr = spec[k];
            for (int s = 0; s < S; ++s) {
                int dlt = p->stoich[rr * S + s];
                if (dlt != 0) {
                    cnt[v * S + s] += dlt;
                    check_count(cnt[v * S + s], overflow);
                }
            }
        } else {
            int s = spec[k];
            double a1 = p->diffusion[s] * (double)(int64_t)cnt[v * S + s];
            int kdir = 0;
            for (int l = 1; l <= deg - 1; ++l)
                if (resid >= (double)l * a1) ++kdir;
            int dst = nb[kdir];
            cnt[v * S + s] -= 1;
            cnt[dst * S + s] += 1;
            check_count(cnt[v * S + s], overflow);
            check_count(cnt[dst * S + s], overflow);
        }
        ++events;
    }
    *events_out = events;
    *draws_out = j;
    *last_t_out = t;
}

/* S channels of one edge: first N_i(v) D_j(w) for v in A, w in B, then the
 * mirror N_j(w) D_i(v) for w in B, v in A; propensity trans_rate * N * D. */
/* Whether the problem has an S operator at all. */
static int has_signal(const oracle_problem *p)
{
    return p->signal_order == 1 ? p->trans_d >= 0 : p->trans_n >= 0;
}

/* First-order signalling: the voxel of the receiving face group that a
 * sending face voxel k of a group of m_from voxels faces.  Both groups are
 * slices of their cells' membrane rings, traversed the same way round, so
 * along the shared face they run in opposite directions: the k-th of m_from
 * faces the (m_to - 1 - floor(k m_to / m_from))-th of m_to (the mirror
 * image when the groups are equal). */
static int facing_voxel(int k, int m_from, int m_to)
{
    return m_to - 1 - (k * m_to) / m_from;
}

/* The edge's S channels in order.  Bimolecular (order 2): c N_i(a) D_j(b)
 * for a in A, b in B, then c N_j(b) D_i(a) for b in B, a in A.  First order
 * (order 1, the paper's Delta turning into the neighbour's NICD at k_N,
 * Results, Model): c D_i(a) for a in A, then c D_j(b) for b in B. */
static int edge_channels(const oracle_problem *p, const int32_t *ci, const int32_t *cj,
                         const int *A, int mA, const int *B, int mB, double ki, double kj,
                         double *a)
{
    const int S = p->n_species;
    int K = 0;
    if (p->signal_order == 1) {  /* ki, kj: the rates of cell i's and cell j's molecules */
        for (int ia = 0; ia < mA; ++ia) a[K++] = ki * (double)ci[A[ia] * S + p->trans_d];
        for (int ib = 0; ib < mB; ++ib) a[K++] = kj * (double)cj[B[ib] * S + p->trans_d];
        return K;
    }
    for (int ia = 0; ia < mA; ++ia)
        for (int ib = 0; ib < mB; ++ib) {
            int64_t nn = ci[A[ia] * S + p->trans_n], dd = cj[B[ib] * S + p->trans_d];
            a[K++] = p->trans_rate * (double)(nn * dd);
        }
    for (int ib = 0; ib < mB; ++ib)
        for (int ia = 0; ia < mA; ++ia) {
            int64_t nn = cj[B[ib] * S + p->trans_n], dd = ci[A[ia] * S + p->trans_d];
            a[K++] = p->trans_rate * (double)(nn * dd);
        }
    return K;
}

/* One S step of one edge (i, j) over [0, dt). */
static void s_edge_step(const oracle_problem *p, int e, int32_t *ci, int32_t *cj,
                        const int *A, int mA, const int *B, int mB, double ki, double kj,
                        double dt, uint32_t step,
                        uint64_t *events_out, uint64_t *draws_out, double *last_t_out,
                        uint32_t *overflow, uint32_t *capped)
{
    const int S = p->n_species;
    double t = 0.0;
    uint32_t j = 0;
    uint64_t events = 0;
    for (;;) {
        double a[2 * 64];
        int K = edge_channels(p, ci, cj, A, mA, B, mB, ki, kj, a);
        double a0 = 0.0;
        for (int k = 0; k < K; ++k) a0 = a0 + a[k];
        if (a0 == 0.0) break;
        if (events >= p->event_cap) { set_flag(capped); break; }
        double u1, u2;
        draw_pair(p->seed, p->sim_id, 1u, (uint32_t)e, step, j, &u1, &u2);
        ++j;
        double tau = (-oracle_plog(u1)) / a0;
        double tn = t + tau;
        if (tn >= dt) break;
        t = tn;
        double r = u2 * a0;
        double resid;
        int k = select_channel(a, K, r, &resid);
        if (p->signal_order == 1) {
            int32_t *from, *to;
            int vf, vt;
            if (k < mA) {           /* a Delta of cell i becomes NICD in cell j */
                from = ci; to = cj; vf = A[k]; vt = B[facing_voxel(k, mA, mB)];
            } else {                /* and the mirror */
                from = cj; to = ci; vf = B[k - mA]; vt = A[facing_voxel(k - mA, mB, mA)];
            }
            from[vf * S + p->trans_d] -= 1;
            to[vt * S + p->trans_i] += 1;
            check_count(from[vf * S + p->trans_d], overflow);
            check_count(to[vt * S + p->trans_i], overflow);
            ++events;
            continue;
        }
        int32_t *recv, *send;
        int vr, vs;
        if (k < mA * mB) {          /* into cell i */
            recv = ci; send = cj; vr = A[k / mB]; vs = B[k % mB];
        } else {                    /* mirror, into cell j */
            int kk = k - mA * mB;
            recv = cj; send = ci; vr = B[kk / mA]; vs = A[kk % mA];
        }
        recv[vr * S + p->trans_n] -= 1;
        send[vs * S + p->trans_d] -= 1;
        recv[vr * S + p->trans_i] += 1;
        check_count(recv[vr * S + p->trans_n], overflow);
        check_count(send[vs * S + p->trans_d], overflow);
        check_count(recv[vr * S + p->trans_i], overflow);
        ++events;
    }
    *events_out = events;
    *draws_out = j;
    *last_t_out = t;
}

static uint64_t dbits(double d)
{
    uint64_t u;
    memcpy(&u, &d, sizeof(u));
    return u;
}

/* Number of edges of the problem's lattice. */
int oracle_num_edges(const oracle_problem *p)
{
    return oracle_lattice_edges(p->lattice, p->nx, p->ny, NULL, NULL, NULL, NULL);
}

/* Run n_steps splitting steps with global step indices start_step + k.
 * Lie (scheme 0): Phi = S_{C-1} o ... o S_0 o chi, the modules one after the
 * other over dt (the splitting the paper's framework rests on: section "A
 * parallel framework for multiscale simulation of cells", design
 * assumptions).  Strang (scheme 1, G. Strang 1968, symmetric splitting):
 * chi over dt/2 with counter tag 0, S over dt, chi over dt/2 with tag 2.
 * counts: [cell][voxel][species], updated in place.  Trace arrays are
 * optional (NULL): chi_ev/chi_t are [n_steps][n_cells], s_ev/s_t are
 * [n_steps][n_edges]; *_t hold the bits of the clock after the last accepted
 * event of the unit-step (0.0 if none); under Strang chi_ev sums the two
 * halves and chi_t is the second half's clock. */
int oracle_run(const oracle_problem *p, double dt, int32_t n_steps, int32_t *counts,
               oracle_stats *st, uint32_t *chi_ev, uint64_t *chi_t,
               uint32_t *s_ev, uint64_t *s_t, int32_t n_threads)
{
    const int S = p->n_species;
    const int ncell = p->nx * p->ny;
    const int nd = p->lattice == 0 ? 4 : 6;
    const int ncol = p->lattice == 0 ? 4 : 6;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (ncell + 1));
    off[0] = 0;
    for (int c = 0; c < ncell; ++c) off[c + 1] = off[c] + (int64_t)p->mesh_w[c] * p->mesh_h[c] * S;
    int E = oracle_num_edges(p);
    int32_t *ei = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    int32_t *ej = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    int32_t *ed = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    int32_t *ec = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    oracle_lattice_edges(p->lattice, p->nx, p->ny, ei, ej, ed, ec);
    int *cstart = (int *)calloc(ncol + 1, sizeof(int));
    for (int e = 0; e < E; ++e) cstart[ec[e] + 1]++;
    for (int c = 0; c < ncol; ++c) cstart[c + 1] += cstart[c];
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    memset(st, 0, sizeof(*st));
    uint64_t chi_events = 0, s_events = 0, draws = 0;

    for (int k = 0; k < n_steps; ++k) {
        uint32_t step = p->start_step + (uint32_t)k;
        /* chi: every cell independently (first half under Strang) */
        const double dchi = p->scheme == 1 ? dt * 0.5 : dt;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(+:chi_events, draws)
#endif
        for (int c = 0; c < ncell; ++c) {
            uint64_t ev, dr;
            double lt;
            const oracle_problem pc = cell_view(p, c);
            chi_cell_step(&pc, c, p->mesh_w[c], p->mesh_h[c], counts + off[c], dchi, step, 0u,
                          &ev, &dr, &lt, &st->overflow, &st->capped);
            chi_events += ev;
            draws += dr;
            if (chi_ev) chi_ev[(int64_t)k * ncell + c] = (uint32_t)ev;
            if (chi_t) chi_t[(int64_t)k * ncell + c] = dbits(lt);
        }
        /* S: colour classes in order, edges of one class independently */
        if (has_signal(p)) {
            for (int col = 0; col < ncol; ++col) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(+:s_events, draws)
#endif
                for (int e = cstart[col]; e < cstart[col + 1]; ++e) {
                    int i = ei[e], jj = ej[e], d = ed[e];
                    int A[64], B[64];
                    int mA = oracle_face_group(p->mesh_w[i], p->mesh_h[i], nd, d, A);
                    int mB = oracle_face_group(p->mesh_w[jj], p->mesh_h[jj], nd,
                                               (d + nd / 2) % nd, B);
                    uint64_t ev, dr;
                    double lt;
                    s_edge_step(p, e, counts + off[i], counts + off[jj], A, mA, B, mB,
                                cell_signal_rate(p, i), cell_signal_rate(p, jj),
                                dt, step, &ev, &dr, &lt, &st->overflow, &st->capped);
                    s_events += ev;
                    draws += dr;
                    if (s_ev) s_ev[(int64_t)k * E + e] = (uint32_t)ev;
                    if (s_t) s_t[(int64_t)k * E + e] = dbits(lt);
                }
            }
        }
        /* Strang: the second half of chi */
        if (p->scheme == 1) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(+:chi_events, draws)
#endif
            for (int c = 0; c < ncell; ++c) {
                uint64_t ev, dr;
                double lt;
                const oracle_problem pc = cell_view(p, c);
                chi_cell_step(&pc, c, p->mesh_w[c], p->mesh_h[c], counts + off[c], dchi, step, 2u,
                              &ev, &dr, &lt, &st->overflow, &st->capped);
                chi_events += ev;
                draws += dr;
                if (chi_ev) chi_ev[(int64_t)k * ncell + c] += (uint32_t)ev;
                if (chi_t) chi_t[(int64_t)k * ncell + c] = dbits(lt);
            }
        }
    }
    st->chi_events = chi_events;
    st->s_events = s_events;
    st->draws = draws;
    free(off); free(ei); free(ej); free(ed); free(ec); free(cstart);
    return 0;
}

/* Threads the OpenMP runtime would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
