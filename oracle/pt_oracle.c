/*
 * pt_oracle.c -- CPU reference ("oracle") for the replica-exchange Metropolis
 * simulation of an elastic bead-spring homopolymer described by Gross, Janke
 * and Bachmann, "Massively parallelized replica-exchange simulations of
 * polymers on GPUs" (Comput. Phys. Commun.; arXiv:1107.3490).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, FP64 implementation that
 * the HIP library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it.  It shares no code, no
 * header and no constant table with the HIP library; both are written from
 * the paper and from the canonical operation order spelt out below.
 *
 * What is computed, and where the paper defines it:
 *   - truncated, shifted Lennard-Jones pair energy ............ Sec. 3.1, Eqs. (1)-(2)
 *   - FENE bond energy ......................................... Sec. 3.1, Eq. (3)
 *   - total energy E(C) (all pairs i<j, bonded pairs included) . Sec. 3.1, Eq. (4)
 *   - local move: random monomer, uniform cube displacement .... Sec. 3.2
 *   - Metropolis acceptance ..................................... Sec. 3.2, Eq. (5)
 *   - neighbour-temperature replica exchange ................... Sec. 3.3, Eq. (6)
 *   - per-sweep energy, end-to-end distance, radius of gyration  Sec. 3.4 (kernel
 *     description) and Sec. 4.1, Eq. (8)
 *
 * Where the paper leaves the arithmetic open, this file fixes it (the same
 * fixed order is the contract the GPU library implements independently):
 *   - Pair distance: r2 = fma(dz, dz, fma(dy, dy, dx*dx)), dx = difference of
 *     the two FP64 coordinates (sign irrelevant: squares are sign-blind).
 *   - LJ term e(r2): 0 if !(r2 < rc2); else s2 = sig2/r2, s6 = (s2*s2)*s2,
 *     g = s6*(s6-1), e = fma(4 eps, g, -E_LJ(rc)).  Coincident beads give +inf.
 *   - FENE term F(r2): r = sqrt(r2), x = (r - r0)/R, y = fma(-x, x, 1);
 *     +inf if !(y > 0), else (-(K/2) R^2) * plog(y).
 *   - plog: a deterministic natural logarithm built from IEEE +,-,*,/ and fma
 *     only (argument reduction to [sqrt(1/2), sqrt(2)), s = f/(2+f), the odd
 *     atanh series in s through the z^9 term by Horner, e*ln2 split hi/lo).
 *     libm's log is not used: the GPU must reproduce every bit.
 *   - Sums: zero-padded pairwise trees over a power-of-two index range,
 *     sum[lo,hi) = sum[lo,mid) + sum[mid,hi).
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (seed low 32 bits, seed high 32 bits).  Move m of sweep t in global
 *     slot g uses counters (m, t, g, 0) -> w0..w3 and (m, t, g, 1) -> v0;
 *     bead k = floor(w0 * N / 2^32); displacement component a =
 *     (((w_a + 0.5) 2^-32) - 0.5) * edge; u = (v0 + 0.5) 2^-32.
 *     Exchange of slots (i, i+1) of chain c at exchange step e uses counter
 *     (i, e, c, 2), u from word 0.
 *   - Metropolis (Eq. 5): accept iff dE <= 0 or beta*dE < -plog(u).
 *   - Exchange (Eq. 6): D = (beta_i - beta_{i+1}) * (E_i - E_{i+1}); accept
 *     iff D >= 0 or plog(u) < D, with E the canonical energy of the
 *     conformation held by the slot.  At exchange step e, pairs (i, i+1) with
 *     i = e mod 2, e mod 2 + 2, ... are attempted; slots keep their beta and
 *     their random stream, conformations are permuted.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off (see build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Model (Sec. 3.1).                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double epsilon, sigma, r_cut, fene_k, fene_R, fene_r0, step_edge;
} orc_model;

/* Derived constants, each a fixed IEEE expression of the model parameters. */
typedef struct {
    double sig2;      /* sigma * sigma                                        */
    double rc2;       /* r_cut * r_cut                                        */
    double four_eps;  /* 4 * epsilon                                          */
    double e_rc;      /* E_LJ(r_c), Eq. (2) evaluated at r_c                  */
    double fene_cf;   /* ((-0.5 * K) * R) * R                                 */
    double r0, R, edge;
} orc_consts;

ORC_API void orc_consts_init(const orc_model *m, orc_consts *c)
{
    c->sig2 = m->sigma * m->sigma;
    c->rc2 = m->r_cut * m->r_cut;
    c->four_eps = 4.0 * m->epsilon;
    double s2 = c->sig2 / c->rc2;
    double s6 = (s2 * s2) * s2;
    c->e_rc = c->four_eps * (s6 * (s6 - 1.0));
    c->fene_cf = ((-0.5 * m->fene_k) * m->fene_R) * m->fene_R;
    c->r0 = m->fene_r0;
    c->R = m->fene_R;
    c->edge = m->step_edge;
}

/* ------------------------------------------------------------------------ */
/* Deterministic logarithm.                                                   */
/* ------------------------------------------------------------------------ */

static const double ORC_LN2_HI = 0x1.62e42fee00000p-1;   /* ln 2 to 32 bits   */
static const double ORC_LN2_LO = 0x1.a39ef35793c76p-33;  /* ln 2 - ORC_LN2_HI */
static const double ORC_SQRT2 = 0x1.6a09e667f3bcdp+0;    /* nearest to sqrt 2 */

/* Natural logarithm: x = 2^e m, m in [sqrt(1/2), sqrt(2)); with f = m - 1 and
 * s = f / (2 + f), log m = 2 atanh s = 2s + sum_{k>=1} 2 s^(2k+1) / (2k+1).
 * |s| <= 0.1716, so ten series terms leave a truncation below 2^-56 |2s|. */
ORC_API double orc_plog(double x)
{
    if (x != x || x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return INFINITY;
    uint64_t ix;
    int e = 0;
    memcpy(&ix, &x, sizeof ix);
    if ((ix >> 52) == 0) {               /* subnormal: scale into the normal range */
        x = x * 0x1p54;
        memcpy(&ix, &x, sizeof ix);
        e = -54;
    }
    e += (int)(ix >> 52) - 1023;
    ix = (ix & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &ix, sizeof m);           /* m in [1, 2) */
    if (m >= ORC_SQRT2) {
        m = m * 0.5;
        e += 1;
    }
    double f = m - 1.0;                  /* exact */
    double s = f / (2.0 + f);
    double z = s * s;
    double q = 2.0 / 21.0;
    q = fma(q, z, 2.0 / 19.0);
    q = fma(q, z, 2.0 / 17.0);
    q = fma(q, z, 2.0 / 15.0);
    q = fma(q, z, 2.0 / 13.0);
    q = fma(q, z, 2.0 / 11.0);
    q = fma(q, z, 2.0 / 9.0);
    q = fma(q, z, 2.0 / 7.0);
    q = fma(q, z, 2.0 / 5.0);
    q = fma(q, z, 2.0 / 3.0);
    double L = fma(s * z, q, 2.0 * s);
    double de = (double)e;
    return de * ORC_LN2_HI + fma(de, ORC_LN2_LO, L);
}

/* ------------------------------------------------------------------------ */
/* Pair and bond terms (Eqs. 1-3).                                            */
/* ------------------------------------------------------------------------ */

static inline double orc_r2(const double *a, const double *b)
{
    double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* E_LJ^mod of Eq. (1): E_LJ(min(r, r_c)) - E_LJ(r_c), E_LJ from Eq. (2). */
ORC_API double orc_lj(const orc_consts *c, double r2)
{
    if (!(r2 < c->rc2)) return 0.0;
    double s2 = c->sig2 / r2;
    double s6 = (s2 * s2) * s2;
    double g = s6 * (s6 - 1.0);
    return fma(c->four_eps, g, -c->e_rc);
}

/* E_FENE of Eq. (3); +inf where the bond is at or beyond r0 +- R. */
ORC_API double orc_fene(const orc_consts *c, double r2)
{
    double r = sqrt(r2);
    double x = (r - c->r0) / c->R;
    double y = fma(-x, x, 1.0);
    if (!(y > 0.0)) return INFINITY;
    return c->fene_cf * orc_plog(y);
}

/* ------------------------------------------------------------------------ */
/* Pairwise trees.                                                            */
/* ------------------------------------------------------------------------ */

static int orc_pow2_at_least(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

/* sum of a[lo, hi), hi - lo a power of two, split at the middle. */
static double orc_tree(const double *a, int lo, int hi)
{
    if (hi - lo == 1) return a[lo];
    int mid = lo + (hi - lo) / 2;
    return orc_tree(a, lo, mid) + orc_tree(a, mid, hi);
}

/* ------------------------------------------------------------------------ */
/* Energies (Eq. 4) and the local energy difference of a move.               */
/* ------------------------------------------------------------------------ */

/* E(C) = sum_{i<j} E_LJ^mod(r_ij) + sum_{i<N-1} E_FENE(r_{i,i+1}).  The
 * factor 1/2 over ordered pairs of Eq. (4) is the sum over unordered pairs.
 * Row i is the tree over j of [i < j < N] e(r2_ij); the LJ part is the tree
 * over rows; the FENE part is the tree over bonds; E = LJ + FENE.
 * xyz: N beads, AoS.  scratch: 2 * pow2(N) doubles. */
static double orc_energy_s(const orc_consts *c, int n, const double *xyz, double *scratch)
{
    int np = orc_pow2_at_least(n);
    double *row = scratch, *acc = scratch + np;
    for (int i = 0; i < np; ++i) {
        if (i < n) {
            for (int j = 0; j < np; ++j)
                row[j] = (j > i && j < n) ? orc_lj(c, orc_r2(xyz + 3 * i, xyz + 3 * j)) : 0.0;
            acc[i] = orc_tree(row, 0, np);
        } else {
            acc[i] = 0.0;
        }
    }
    double e_lj = orc_tree(acc, 0, np);
    for (int i = 0; i < np; ++i)
        row[i] = (i < n - 1) ? orc_fene(c, orc_r2(xyz + 3 * i, xyz + 3 * (i + 1))) : 0.0;
    double e_fene = orc_tree(row, 0, np);
    return e_lj + e_fene;
}

ORC_API double orc_energy(const orc_consts *c, int n, const double *xyz)
{
    double *s = (double *)malloc(sizeof(double) * 2 * (size_t)orc_pow2_at_least(n));
    double e = orc_energy_s(c, n, xyz, s);
    free(s);
    return e;
}

/* E(C') - E(C) restricted to the terms that involve the moved bead k (the
 * other terms cancel exactly in real arithmetic):
 *   S  = tree over j of t_j, t_j = e(|r_j - r'_k|^2) - e(|r_j - r_k|^2) for
 *        j < N, j != k, and t_j = 0 otherwise (pow2(N) leaves);
 *   dF = (F(r'_k, r_{k-1}) - F(r_k, r_{k-1})) + (F(r_{k+1}, r'_k) - F(r_{k+1}, r_k)),
 *        a missing neighbour contributing 0;
 *   dE = S + dF.                                            (Eqs. 4 and 5) */
static double orc_delta_e_s(const orc_consts *c, int n, const double *xyz, int k,
                            const double *rn, double *scratch)
{
    int np = orc_pow2_at_least(n);
    const double *ro = xyz + 3 * k;
    for (int j = 0; j < np; ++j) {
        if (j < n && j != k) {
            const double *rj = xyz + 3 * j;
            scratch[j] = orc_lj(c, orc_r2(rj, rn)) - orc_lj(c, orc_r2(rj, ro));
        } else {
            scratch[j] = 0.0;
        }
    }
    double s = orc_tree(scratch, 0, np);
    double dfl = 0.0, dfr = 0.0;
    if (k > 0) {
        const double *rl = xyz + 3 * (k - 1);
        dfl = orc_fene(c, orc_r2(rl, rn)) - orc_fene(c, orc_r2(rl, ro));
    }
    if (k < n - 1) {
        const double *rr = xyz + 3 * (k + 1);
        dfr = orc_fene(c, orc_r2(rr, rn)) - orc_fene(c, orc_r2(rr, ro));
    }
    return s + (dfl + dfr);
}

ORC_API double orc_delta_e(const orc_consts *c, int n, const double *xyz, int k, const double *rn)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)orc_pow2_at_least(n));
    double d = orc_delta_e_s(c, n, xyz, k, rn, s);
    free(s);
    return d;
}

/* End-to-end distance squared and squared radius of gyration (Eq. 8), with
 * the centre of mass as the plain mean: m_a = tree(a_k) / N;
 * Rg2 = tree(fma(dz,dz,fma(dy,dy,dx*dx))) / N with d = r_k - m. */
static void orc_shape_s(int n, const double *xyz, double *ree2, double *rg2, double *scratch)
{
    int np = orc_pow2_at_least(n);
    double mean[3];
    *ree2 = orc_r2(xyz, xyz + 3 * (n - 1));
    for (int a = 0; a < 3; ++a) {
        for (int k = 0; k < np; ++k) scratch[k] = (k < n) ? xyz[3 * k + a] : 0.0;
        mean[a] = orc_tree(scratch, 0, np) / (double)n;
    }
    for (int k = 0; k < np; ++k) scratch[k] = (k < n) ? orc_r2(mean, xyz + 3 * k) : 0.0;
    *rg2 = orc_tree(scratch, 0, np) / (double)n;
}

ORC_API void orc_shape(int n, const double *xyz, double *ree2, double *rg2)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)orc_pow2_at_least(n));
    orc_shape_s(n, xyz, ree2, rg2, s);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11) and the draws of one move.           */
/* ------------------------------------------------------------------------ */

ORC_API void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double orc_unit(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Sec. 3.2: a random monomer k and a displacement uniform in the cube of the
 * given edge; u drives the acceptance test. */
ORC_API void orc_move_draws(uint64_t seed, uint32_t m, uint32_t t, uint32_t gid, int n, double edge,
                            int *k, double d[3], double *u)
{
    uint32_t ctr[4] = {m, t, gid, 0u}, w[4], v[4];
    orc_philox(ctr, seed, w);
    ctr[3] = 1u;
    orc_philox(ctr, seed, v);
    *k = (int)(((uint64_t)w[0] * (uint64_t)(uint32_t)n) >> 32);
    for (int a = 0; a < 3; ++a) d[a] = (orc_unit(w[a + 1]) - 0.5) * edge;
    *u = orc_unit(v[0]);
}

/* Eq. (5): p = min(1, exp(-beta dE)); accept iff u < p, taken in the log domain. */
ORC_API int orc_metropolis(double beta, double de, double u)
{
    if (de <= 0.0) return 1;
    return (beta * de < -orc_plog(u)) ? 1 : 0;
}

/* Eq. (6): p = min(1, exp((E_i - E_{i+1})(beta_i - beta_{i+1}))). */
ORC_API int orc_exchange_accept(double beta_i, double beta_j, double e_i, double e_j, double u)
{
    double d = (beta_i - beta_j) * (e_i - e_j);
    if (d >= 0.0) return 1;
    return (orc_plog(u) < d) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Whole simulation.                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_chains;
    const int32_t *n_beads;        /* [n_chains]                                  */
    const int32_t *n_slots;        /* [n_chains]                                  */
    const double *beta;            /* [sum R_c] per chain, slot 0 first           */
    const uint32_t *stream_chain;  /* [n_chains] chain id in exchange counters    */
    const uint32_t *stream_slot0;  /* [n_chains] global slot id of slot 0         */
    uint64_t seed;
    int32_t exchange_every;        /* exchange step after sweeps t with (t+1)%k==0; 0 = never */
    int32_t n_threads;             /* 0 = OpenMP default                          */
} orc_config;

/* State and outputs.  Conformation q of chain c occupies N_c beads (AoS) at
 * conf_off[q]; perm[g] is the conformation held by global slot g.
 * Optional outputs (NULL to skip):
 *   accept_log [sweep][word]  ceil(N/64) words per slot, slots in order;
 *   exch_log   [step][slot]   1 accepted / 0 rejected for the lower slot of an
 *                             attempted pair, 0xFF otherwise;
 *   series     [sweep][slot][3] = (E, Ree2, Rg2) after the sweep, before exchange. */
typedef struct {
    double *coords;
    int32_t *perm;
    double *energy;         /* [slots] canonical E of the held conformation */
    int64_t *accepts;       /* [slots] accepted moves                       */
    int64_t *exch_tries;    /* [slots] attempts of pair (g, g+1)            */
    int64_t *exch_accepts;  /* [slots]                                      */
    uint64_t *accept_log;
    uint8_t *exch_log;
    double *series;
} orc_state;

static void orc_layout(const orc_config *cfg, int32_t *chain_of, int32_t *slot_in_chain,
                       int64_t *conf_off, int64_t *word_off, int64_t *words_total)
{
    int64_t off = 0, woff = 0;
    int g = 0;
    for (int c = 0; c < cfg->n_chains; ++c) {
        for (int s = 0; s < cfg->n_slots[c]; ++s, ++g) {
            chain_of[g] = c;
            slot_in_chain[g] = s;
            conf_off[g] = off;
            word_off[g] = woff;
            off += 3 * (int64_t)cfg->n_beads[c];
            woff += (cfg->n_beads[c] + 63) / 64;
        }
    }
    *words_total = woff;
}

/* One exchange step with index e over all chains (Sec. 3.3). */
static void orc_exchange_step(const orc_config *cfg, orc_state *st, const int32_t *slot0,
                              uint32_t e, uint8_t *log_row)
{
    int total = 0;
    for (int c = 0; c < cfg->n_chains; ++c) total += cfg->n_slots[c];
    if (log_row) memset(log_row, 0xFF, (size_t)total);
    for (int c = 0; c < cfg->n_chains; ++c) {
        int base = slot0[c];
        uint32_t cid = cfg->stream_chain ? cfg->stream_chain[c] : (uint32_t)c;
        for (int i = (int)(e & 1u); i + 1 < cfg->n_slots[c]; i += 2) {
            int g = base + i;
            uint32_t ctr[4] = {(uint32_t)i, e, cid, 2u}, w[4];
            orc_philox(ctr, cfg->seed, w);
            int acc = orc_exchange_accept(cfg->beta[g], cfg->beta[g + 1], st->energy[g],
                                          st->energy[g + 1], orc_unit(w[0]));
            st->exch_tries[g] += 1;
            if (acc) {
                int32_t tp = st->perm[g];
                st->perm[g] = st->perm[g + 1];
                st->perm[g + 1] = tp;
                double te = st->energy[g];
                st->energy[g] = st->energy[g + 1];
                st->energy[g + 1] = te;
                st->exch_accepts[g] += 1;
            }
            if (log_row) log_row[g] = (uint8_t)acc;
        }
    }
}

/* Run sweeps t0 .. t0+n_sweeps-1 (exchange steps numbered from e0).
 * One sweep of a slot is N attempted moves (Sec. 3.2).  After each sweep the
 * canonical energy and the shape observables of every slot are recorded;
 * then, if due, one exchange step runs.  Returns the next exchange index. */
ORC_API int64_t orc_run(const orc_model *model, const orc_config *cfg, orc_state *st,
                        int64_t t0, int64_t e0, int64_t n_sweeps)
{
    orc_consts cst;
    orc_consts_init(model, &cst);
    int total = 0, nmax = 1;
    for (int c = 0; c < cfg->n_chains; ++c) {
        total += cfg->n_slots[c];
        if (cfg->n_beads[c] > nmax) nmax = cfg->n_beads[c];
    }
    int32_t *chain_of = (int32_t *)malloc(sizeof(int32_t) * total);
    int32_t *slot_in = (int32_t *)malloc(sizeof(int32_t) * total);
    int64_t *conf_off = (int64_t *)malloc(sizeof(int64_t) * total);
    int64_t *word_off = (int64_t *)malloc(sizeof(int64_t) * total);
    int32_t *slot0 = (int32_t *)malloc(sizeof(int32_t) * (cfg->n_chains + 1));
    int64_t words_total = 0;
    orc_layout(cfg, chain_of, slot_in, conf_off, word_off, &words_total);
    for (int c = 0, g = 0; c < cfg->n_chains; g += cfg->n_slots[c], ++c) slot0[c] = g;
    int npmax = orc_pow2_at_least(nmax);
    int nthreads = cfg->n_threads;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int64_t e = e0;
    for (int64_t ts = 0; ts < n_sweeps; ++ts) {
        uint32_t t = (uint32_t)(t0 + ts);
#pragma omp parallel num_threads(nthreads)
        {
            double *scratch = (double *)malloc(sizeof(double) * 2 * (size_t)npmax);
#pragma omp for schedule(dynamic, 1)
            for (int g = 0; g < total; ++g) {
                int c = chain_of[g];
                int n = cfg->n_beads[c];
                double beta = cfg->beta[g];
                uint32_t gid = cfg->stream_slot0 ? cfg->stream_slot0[c] + (uint32_t)slot_in[g]
                                                 : (uint32_t)g;
                double *xyz = st->coords + conf_off[st->perm[g]];
                uint64_t *bits = st->accept_log ? st->accept_log + ts * words_total + word_off[g] : NULL;
                if (bits) memset(bits, 0, sizeof(uint64_t) * (size_t)((n + 63) / 64));
                for (int m = 0; m < n; ++m) {
                    int k;
                    double d[3], u, rn[3];
                    orc_move_draws(cfg->seed, (uint32_t)m, t, gid, n, cst.edge, &k, d, &u);
                    for (int a = 0; a < 3; ++a) rn[a] = xyz[3 * k + a] + d[a];
                    double de = orc_delta_e_s(&cst, n, xyz, k, rn, scratch);
                    if (orc_metropolis(beta, de, u)) {
                        for (int a = 0; a < 3; ++a) xyz[3 * k + a] = rn[a];
                        st->accepts[g] += 1;
                        if (bits) bits[m >> 6] |= 1ull << (m & 63);
                    }
                }
                double en = orc_energy_s(&cst, n, xyz, scratch);
                st->energy[g] = en;
                if (st->series) {
                    double ree2, rg2;
                    orc_shape_s(n, xyz, &ree2, &rg2, scratch);
                    double *row = st->series + ((size_t)ts * total + g) * 3;
                    row[0] = en;
                    row[1] = ree2;
                    row[2] = rg2;
                }
            }
            free(scratch);
        }
        if (cfg->exchange_every > 0 && ((int64_t)t + 1) % cfg->exchange_every == 0) {
            uint8_t *row = st->exch_log ? st->exch_log + (e - e0) * total : NULL;
            orc_exchange_step(cfg, st, slot0, (uint32_t)e, row);
            e += 1;
        }
    }
    free(chain_of);
    free(slot_in);
    free(conf_off);
    free(word_off);
    free(slot0);
    return e;
}

/* One explicit exchange step (index e) on the current state; energies must
 * hold the canonical energy of each slot's conformation. */
ORC_API void orc_exchange(const orc_config *cfg, orc_state *st, uint32_t e, uint8_t *log_row)
{
    int32_t *slot0 = (int32_t *)malloc(sizeof(int32_t) * (cfg->n_chains + 1));
    for (int c = 0, g = 0; c < cfg->n_chains; g += cfg->n_slots[c], ++c) slot0[c] = g;
    orc_exchange_step(cfg, st, slot0, e, log_row);
    free(slot0);
}
