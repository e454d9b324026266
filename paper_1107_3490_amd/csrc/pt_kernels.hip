// pt_kernels.hip -- gfx950 kernels of libpt.so: Metropolis sweeps of single-
// monomer moves, the FP64-order energy, and neighbour-temperature replica
// exchange for a bead-spring homopolymer (Gross, Janke, Bachmann,
// arXiv:1107.3490, Secs. 3.1-3.4).
//
// Mapping.  One 64-lane wavefront owns one replica for a whole sweep.  The
// replica's FP64 coordinates live in LDS in a swizzled SoA layout: bead j of a
// chain whose class has B beads per lane sits at (j mod B) * 64 + j / B, so
// lane l owns the contiguous bead block [l B, (l+1) B) and, for a fixed b, the
// 64 lanes touch 64 consecutive doubles (no bank conflicts).  The same layout
// is kept in HBM, so loading and storing a replica are straight coalesced
// copies.  Beads past the chain end hold a far-away sentinel x coordinate, and
// the moved bead's slot holds it during its own pair loop, so every pair term
// of a padded or excluded bead is an exact zero without a per-pair mask.
//
// The pair sum of a move is the pairwise tree over the lane's contiguous block
// followed by the butterfly over lanes: the FP64-order sum of the public header
// for every beads-per-lane choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_device.hpp"
#include "pt_internal.hpp"

namespace pt {

namespace {

constexpr double SENTINEL = 1.0e30;

template <int B>
struct Geo {
    static constexpr int NP = 64 * B;
    static constexpr int LOG = (B == 1) ? 0 : (B == 2) ? 1 : (B == 4) ? 2 : (B == 8) ? 3 : (B == 16) ? 4 : 5;
    static constexpr int LOG_NP = 6 + LOG;
    __device__ static __forceinline__ int pos(int j) { return ((j & (B - 1)) << 6) | (j >> LOG); }
};

struct Leaf64 {
    double t, a;
    __device__ Leaf64 operator+(const Leaf64 &o) const { return Leaf64{t + o.t, a + o.a}; }
};

struct LeafMx {
    double t;
    float b;
    __device__ LeafMx operator+(const LeafMx &o) const { return LeafMx{t + o.t, b + o.b}; }
};

__device__ __forceinline__ double dabs(double v) { return __builtin_fabs(v); }
__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Bound on |E_run - exact sum of the FP64-order terms| added by one accepted
// move scored in the FP64 order: the leaf differences (u each), the tree over
// the leaves (depth log2 NP, u |partial| each), the two bond differences, their
// sum and the final addition, all with a factor-two margin (2^-52 for u).
__device__ __forceinline__ double bound64(int log_np, double abs_leaves, double dfl, double dfr,
                                          double de) {
    return 0x1p-52 * ((double)(log_np + 2) * abs_leaves + 2.0 * (dabs(dfl) + dabs(dfr)) + dabs(de));
}

// Bound on |E_FP64(C) - exact sum of the FP64-order terms| for a conformation
// whose running energy is e with bound b: the two trees of Eq. (4) have depth
// <= 2 log2 NP + 1 and their summands are bounded in absolute value by
// (E + 2 P neg_floor), P = N(N-1)/2, since every negative term is >= -neg_floor
// and the positive ones sum to E plus the negative ones.
__device__ __forceinline__ double bound_energy(const Consts &k, int log_np, int n, double e, double b) {
    const double pairs = 0.5 * (double)n * (double)(n - 1);
    return 0x1p-51 * (double)(2 * log_np + 4) * (dabs(e) + b + 2.0 * pairs * k.neg_floor);
}

// Pushes value v as leaf number `idx` (0, 1, 2, ... in order) of a pairwise
// tree kept as a binary counter: stk[l] holds the pending left sibling of
// size 2^l.  idx is uniform across the wavefront; after leaf 2^L - 1 the
// complete tree over 2^L leaves sits in stk[L].
template <int LEVELS>
__device__ __forceinline__ void tree_push(double (&stk)[LEVELS + 1], int idx, double v) {
    double carry = v;
    bool placed = false;
#pragma unroll
    for (int l = 0; l <= LEVELS; ++l) {
        if (!placed) {
            if ((idx >> l) & 1) {
                carry = stk[l] + carry;
            } else {
                stk[l] = carry;
                placed = true;
            }
        }
    }
}

// Pairwise tree over 64 consecutive leaves j = j0 + jj of row i (zero unless
// i < j < n), the leaves computed in registers from LDS broadcasts.
template <int B, int LO, int HI>
__device__ __forceinline__ double row_chunk(const double *X, const double *Y, const double *Z,
                                            const Consts &k, int i, int n, int j0, double xi,
                                            double yi, double zi) {
    if constexpr (HI - LO == 1) {
        const int j = j0 + LO;
        const int a = Geo<B>::pos(j);
        const double v = lj64(k, sq3(X[a] - xi, Y[a] - yi, Z[a] - zi));
        return (j > i && j < n) ? v : 0.0;
    } else {
        constexpr int MID = (LO + HI) / 2;
        const double l = row_chunk<B, LO, MID>(X, Y, Z, k, i, n, j0, xi, yi, zi);
        const double r = row_chunk<B, MID, HI>(X, Y, Z, k, i, n, j0, xi, yi, zi);
        return l + r;
    }
}

// FP64-order energy E(C) of Eq. (4) for the replica in LDS.  Lane l computes
// the rows i of its own contiguous block [l B, (l+1) B): each row is the tree
// over j in chunks of 64 (static trees, chained by a binary counter), the
// lane's rows feed a binary counter over its block, and the butterfly over
// lanes completes the tree over all NP rows.
template <int B>
__device__ double energy_wave(const double *X, const double *Y, const double *Z, int n,
                              const Consts &k) {
    using G = Geo<B>;
    constexpr int CH = G::NP / 64;  // chunks of 64 leaves per row (= B)
    constexpr int LC = G::LOG;      // levels of the chunk counter
    const int lane = threadIdx.x;
    double blk[LC + 1];
#pragma unroll
    for (int l = 0; l <= LC; ++l) blk[l] = 0.0;
    for (int b = 0; b < B; ++b) {
        const int i = lane * B + b;
        const int a = b * 64 + lane;
        const double xi = X[a], yi = Y[a], zi = Z[a];
        double row[LC + 1];
#pragma unroll
        for (int l = 0; l <= LC; ++l) row[l] = 0.0;
        for (int c = 0; c < CH; ++c) {
            const double v = row_chunk<B, 0, 64>(X, Y, Z, k, i, n, c * 64, xi, yi, zi);
            tree_push<LC>(row, c, v);
        }
        tree_push<LC>(blk, b, (CH == 1) ? row[0] : row[LC]);
    }
    const double e_lj = wave_tree((B == 1) ? blk[0] : blk[LC]);
    // FENE part: bonds (i, i+1), i < n - 1, lane blocks, then the butterfly.
    const double fb = lane_tree<0, B>([&](int b) {
        const int i = lane * B + b;
        const int i0 = (i < n - 1) ? i : 0;
        const int a0 = G::pos(i0), a1 = G::pos(i0 + 1);
        const double v = fene64(k, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
        return (i < n - 1) ? v : 0.0;
    });
    return e_lj + wave_tree(fb);
}

template <int B>
__device__ __forceinline__ void load_replica(double *X, double *Y, double *Z, const double *src) {
    using G = Geo<B>;
    const int lane = threadIdx.x;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        X[b * 64 + lane] = src[b * 64 + lane];
        Y[b * 64 + lane] = src[G::NP + b * 64 + lane];
        Z[b * 64 + lane] = src[2 * G::NP + b * 64 + lane];
    }
    wave_sync();
}

// ------------------------------------------------------------------ sweep --
// One sweep (N attempted moves, Sec. 3.2) of every slot in `list`, then the
// per-sweep record of E, Ree^2 and Rg^2 (Eq. 8).
template <int B, bool MIXED>
__global__ __launch_bounds__(64) void k_sweep(const Tables T, const int32_t *__restrict__ list) {
    using G = Geo<B>;
    __shared__ double X[G::NP], Y[G::NP], Z[G::NP];
    const int lane = threadIdx.x;
    const Consts &K = T.k;
    const int g = list[blockIdx.x];
    const int c = T.slot_chain[g];
    const int n = T.chain_n[c];
    const double beta = T.beta[g];
    const uint32_t gid = T.slot_gid[g];
    const int64_t t64 = T.te[0];
    const uint32_t t = (uint32_t)t64;
    const int q = T.perm[g];
    double *cq = T.coords + T.coord_off[q];
    load_replica<B>(X, Y, Z, cq);

    double E = T.e_run[q], Bd = T.b_run[q];
    int64_t n_acc = 0, n_rescore = 0;
    uint64_t *logrow = (T.accept_log != nullptr && t64 < T.log_cap)
                           ? T.accept_log + t64 * T.words_total + T.word_off[g]
                           : nullptr;

    for (int m0 = 0; m0 < n; m0 += 64) {
        // Draws of move m0 + lane (Philox counters (m, t, g, 0) and (m, t, g, 1)).
        int mk;
        double mdx, mdy, mdz, mth;
        {
            const uint32_t m = (uint32_t)(m0 + lane);
            const U4 w = philox10(U4{m, t, gid, 0u}, T.seed);
            const U4 v = philox10(U4{m, t, gid, 1u}, T.seed);
            mk = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)n) >> 32);
            mdx = (unit_open(w.y) - 0.5) * K.edge;
            mdy = (unit_open(w.z) - 0.5) * K.edge;
            mdz = (unit_open(w.w) - 0.5) * K.edge;
            mth = -det_log(unit_open(v.x));
        }
        const int nb = (n - m0 < 64) ? (n - m0) : 64;
        uint64_t bits = 0;
        for (int i = 0; i < nb; ++i) {
            const int k = read_lane(mk, i);
            const double dx = read_lane(mdx, i), dy = read_lane(mdy, i), dz = read_lane(mdz, i);
            const double th = read_lane(mth, i);
            const int ak = G::pos(k);
            const double xo = X[ak], yo = Y[ak], zo = Z[ak];
            const double xn = xo + dx, yn = yo + dy, zn = zo + dz;

            // Bond terms: lane & 3 picks (k-1,k) new/old, (k,k+1) new/old; the
            // other lanes repeat lanes 0..3.  Straight-line code, so that it
            // overlaps the pair loop.
            const int nbr = (lane & 2) ? k + 1 : k - 1;
            const bool has = nbr >= 0 && nbr < n;
            const int an = G::pos(has ? nbr : k);
            const bool nw = (lane & 1) == 0;
            const double fb = fene64(K, sq3(X[an] - (nw ? xn : xo), Y[an] - (nw ? yn : yo),
                                            Z[an] - (nw ? zn : zo)));
            const double fv = has ? fb : 0.0;

            // The moved bead's own slot holds the sentinel during its pair loop.
            wave_sync();
            if (lane == 0) X[ak] = SENTINEL;
            wave_sync();
            auto leaf64 = [&](int b) {
                const int a = b * 64 + lane;
                const double xj = X[a], yj = Y[a], zj = Z[a];
                const double en = lj64(K, sq3(xj - xn, yj - yn, zj - zn));
                const double eo = lj64(K, sq3(xj - xo, yj - yo, zj - zo));
                const double tt = en - eo;
                return Leaf64{tt, dabs(tt)};
            };
            bool acc = false;
            double de_used = 0.0, bm = 0.0;
            bool exact = !MIXED;
            if constexpr (MIXED) {
                const LeafMx s = lane_tree<0, B>([&](int b) {
                    const int a = b * 64 + lane;
                    const double xj = X[a], yj = Y[a], zj = Z[a];
                    const Lj32 pn = lj32(K, xj - xn, yj - yn, zj - zn);
                    const Lj32 po = lj32(K, xj - xo, yj - yo, zj - zo);
                    return LeafMx{(double)(pn.e - po.e), pn.b + po.b};
                });
                const double sm = wave_tree(s.t);
                const double bs = K.kbound * (double)wave_tree(s.b);
                const double dfl = read_lane(fv, 0) - read_lane(fv, 1);
                const double dfr = read_lane(fv, 2) - read_lane(fv, 3);
                const double df = dfl + dfr;
                const double dem = sm + df;
                const double bt = bs * (1.0 + 0x1p-20) + 0x1p-50 * dabs(dem);
                const double lo = dem - bt, hi = dem + bt;
                const bool sure_acc = (hi <= 0.0) || (beta * hi < th);
                const bool sure_rej = (lo > 0.0) && !(beta * lo < th);
                if (df == __builtin_inf()) {
                    acc = false;  // a broken bond is rejected whatever the pair sum
                } else if (finite(bt) && finite(dem) && (sure_acc || sure_rej)) {
                    acc = sure_acc;
                    de_used = dem;
                    bm = bs * (1.0 + 0x1p-20) + 0x1p-52 * (2.0 * (dabs(dfl) + dabs(dfr)) + dabs(dem));
                } else {
                    exact = true;
                    ++n_rescore;
                }
            }
            if (exact) {
                const Leaf64 s = lane_tree<0, B>(leaf64);
                const double sc = wave_tree(s.t);
                const double ab = wave_tree(s.a);
                const double dfl = read_lane(fv, 0) - read_lane(fv, 1);
                const double dfr = read_lane(fv, 2) - read_lane(fv, 3);
                const double df = dfl + dfr;
                const double de = sc + df;
                acc = (de <= 0.0) || (beta * de < th);
                de_used = de;
                bm = bound64(G::LOG_NP, ab, dfl, dfr, de);
            }
            wave_sync();
            if (lane == 0) {
                X[ak] = acc ? xn : xo;
                if (acc) {
                    Y[ak] = yn;
                    Z[ak] = zn;
                }
            }
            wave_sync();
            if (acc) {
                E = E + de_used;
                Bd = Bd + bm + 0x1p-52 * dabs(E);
                ++n_acc;
                bits |= 1ull << i;
            }
        }
        if (logrow != nullptr && lane == 0) logrow[m0 >> 6] = bits;
    }

    // Write the replica back; record the sweep (before any exchange).
#pragma unroll
    for (int b = 0; b < B; ++b) {
        cq[b * 64 + lane] = X[b * 64 + lane];
        cq[G::NP + b * 64 + lane] = Y[b * 64 + lane];
        cq[2 * G::NP + b * 64 + lane] = Z[b * 64 + lane];
    }
    // Re-synchronise the running energy with the FP64-order energy when its
    // bound has grown past resync_rel of max(1, |E|) (after a start with
    // near-overlapping beads, or after many accepted moves).
    bool resync = false;
    if (!(Bd <= K.resync_rel * (dabs(E) > 1.0 ? dabs(E) : 1.0))) {
        E = energy_wave<B>(X, Y, Z, n, K);
        Bd = bound_energy(K, G::LOG_NP, n, E, 0.0);
        resync = true;
    }
    const int a0 = G::pos(0), a1 = G::pos(n - 1);
    const double ree2 = sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]);
    auto mean = [&](const double *C) {
        double s = lane_tree<0, B>([&](int b) {
            const int j = lane * B + b;
            return (j < n) ? C[b * 64 + lane] : 0.0;
        });
        return wave_tree(s) / (double)n;
    };
    const double mx = mean(X), my = mean(Y), mz = mean(Z);
    double rg = lane_tree<0, B>([&](int b) {
        const int j = lane * B + b;
        const int a = b * 64 + lane;
        const double v = sq3(X[a] - mx, Y[a] - my, Z[a] - mz);
        return (j < n) ? v : 0.0;
    });
    const double rg2 = wave_tree(rg) / (double)n;
    if (lane == 0) {
        T.e_run[q] = E;
        T.b_run[q] = Bd;
        int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
        cnt[0] += n_acc;
        cnt[3] += n_rescore;
        cnt[5] += n;
        cnt[6] += resync ? 1 : 0;
        double *ac = T.acc + (int64_t)g * 5;
        ac[0] += 1.0;
        ac[1] += E;
        ac[2] += E * E;
        ac[3] += rg2;
        ac[4] += ree2;
        if (T.series != nullptr && t64 < T.series_cap) {
            double *row = T.series + (t64 * T.total_slots + g) * 3;
            row[0] = E;
            row[1] = ree2;
            row[2] = rg2;
        }
    }
}

// ----------------------------------------------------------------- energy --
// FP64-order energy of the conformations in `list` (by_slot: list holds slots
// and the conformation is perm[g]); writes out_e / out_b indexed like list.
template <int B>
__global__ __launch_bounds__(64) void k_energy(const Tables T, const int32_t *__restrict__ list,
                                               double *out_e, double *out_b, int by_slot) {
    using G = Geo<B>;
    __shared__ double X[G::NP], Y[G::NP], Z[G::NP];
    const int id = list[blockIdx.x];
    const int q = by_slot ? T.perm[id] : id;
    const int c = T.slot_chain[q];  // conformation q started in slot q: same chain
    const int n = T.chain_n[c];
    load_replica<B>(X, Y, Z, T.coords + T.coord_off[q]);
    const double e = energy_wave<B>(X, Y, Z, n, T.k);
    if (threadIdx.x == 0) {
        out_e[id] = e;
        if (out_b != nullptr) out_b[id] = bound_energy(T.k, G::LOG_NP, n, e, 0.0);
    }
}

// --------------------------------------------------------------- exchange --
// One exchange step (Sec. 3.3, Eq. 6) for the chains in `list`: wave p of a
// chain handles the pair (i, i+1), i = (e mod 2) + 2p.  The decision is taken
// from the running energies when their bounds settle it, otherwise from the
// FP64-order energies of both conformations (which also re-synchronise them).
template <int B>
__global__ __launch_bounds__(64) void k_exchange(const Tables T, const int32_t *__restrict__ list,
                                                 int max_pairs, int force) {
    using G = Geo<B>;
    __shared__ double X[G::NP], Y[G::NP], Z[G::NP];
    const int c = list[blockIdx.x / max_pairs];
    const int p = blockIdx.x % max_pairs;
    const int64_t t = T.te[0], e = T.te[1];
    const bool due = force || (T.exchange_every > 0 && (t + 1) % T.exchange_every == 0);
    if (!due) return;
    const int R = T.chain_slots[c];
    const int i = (int)(e & 1) + 2 * p;
    if (i + 1 >= R) return;
    const int g = T.chain_slot0[c] + i;
    const int n = T.chain_n[c];
    const int q1 = T.perm[g], q2 = T.perm[g + 1];
    const double b1 = T.beta[g], b2 = T.beta[g + 1];
    const U4 w = philox10(U4{(uint32_t)i, (uint32_t)e, T.chain_sid[c], 2u}, T.seed);
    const double pl = det_log(unit_open(w.x));
    const double e1 = T.e_run[q1], e2 = T.e_run[q2];
    const double bb1 = T.b_run[q1], bb2 = T.b_run[q2];
    const double db = b1 - b2;
    const double dd = e1 - e2;
    const double tot = (bb1 + bound_energy(T.k, G::LOG_NP, n, e1, bb1) + bb2 +
                        bound_energy(T.k, G::LOG_NP, n, e2, bb2)) * (1.0 + 0x1p-20) +
                       0x1p-50 * dabs(dd);
    const double d1 = db * (dd - tot), d2 = db * (dd + tot);
    const double dlo = (d1 < d2) ? d1 : d2, dhi = (d1 < d2) ? d2 : d1;
    const bool sure_acc = (dlo >= 0.0) || (pl < dlo);
    const bool sure_rej = (dhi < 0.0) && !(pl < dhi);
    bool acc;
    bool band = false;
    if (finite(tot) && finite(dd) && finite(db) && (sure_acc || sure_rej)) {
        acc = sure_acc;
    } else {
        band = true;
        load_replica<B>(X, Y, Z, T.coords + T.coord_off[q1]);
        const double c1 = energy_wave<B>(X, Y, Z, n, T.k);
        wave_sync();
        load_replica<B>(X, Y, Z, T.coords + T.coord_off[q2]);
        const double c2 = energy_wave<B>(X, Y, Z, n, T.k);
        const double d = db * (c1 - c2);
        acc = (d >= 0.0) || (pl < d);
        if (threadIdx.x == 0) {
            T.e_run[q1] = c1;
            T.b_run[q1] = bound_energy(T.k, G::LOG_NP, n, c1, 0.0);
            T.e_run[q2] = c2;
            T.b_run[q2] = bound_energy(T.k, G::LOG_NP, n, c2, 0.0);
        }
    }
    if (threadIdx.x == 0) {
        int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
        cnt[1] += 1;
        if (band) cnt[4] += 1;
        if (acc) {
            cnt[2] += 1;
            T.perm[g] = q2;
            T.perm[g + 1] = q1;
        }
        if (T.exch_log != nullptr && e < T.log_cap) T.exch_log[e * T.total_slots + g] = acc ? 1 : 0;
    }
}

// Advance the run counters after a sweep (t += 1, and e += 1 when an exchange
// step was due) or after an explicit exchange step (e += 1 only).
__global__ void k_advance(const Tables T, int exchange_only) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t t = T.te[0];
    if (exchange_only) {
        T.te[1] += 1;
        return;
    }
    const bool due = T.exchange_every > 0 && (t + 1) % T.exchange_every == 0;
    T.te[0] = t + 1;
    if (due) T.te[1] += 1;
}

// --------------------------------------------------------------- selftest --
__global__ void k_selftest(const Consts k, int op, const double *x, const double *y, double *out,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (op == 7 || op == 8) {
        // Whole wavefronts: n is a multiple of 64 (checked by the host).
        if (i - (int64_t)(threadIdx.x & 63) >= n) return;
        out[i] = (op == 7) ? wave_tree(x[i]) : (double)wave_tree((float)x[i]);
        return;
    }
    if (i >= n) return;
    switch (op) {
        case 0: out[i] = __builtin_sqrt(x[i]); break;
        case 1: out[i] = x[i] / y[i]; break;
        case 2: out[i] = det_log(x[i]); break;
        case 3: out[i] = fene64(k, x[i]); break;
        case 4: out[i] = lj64(k, x[i]); break;
        case 5: {
            const Lj32 r = lj32(k, x[i], y[i], 0.0);
            out[2 * i] = (double)r.e;
            out[2 * i + 1] = k.kbound * (double)r.b;
            break;
        }
        case 6: {
            const uint64_t seed = ((uint64_t)(uint32_t)y[1] << 32) | (uint64_t)(uint32_t)y[0];
            const U4 w = philox10(U4{(uint32_t)x[4 * i], (uint32_t)x[4 * i + 1],
                                     (uint32_t)x[4 * i + 2], (uint32_t)x[4 * i + 3]}, seed);
            out[4 * i] = w.x;
            out[4 * i + 1] = w.y;
            out[4 * i + 2] = w.z;
            out[4 * i + 3] = w.w;
            break;
        }
        default: break;
    }
}

template <int B>
hipError_t sweep_b(bool mixed, const Tables &T, const int32_t *list, int n, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL((k_sweep<B, true>), dim3(n), dim3(64), 0, s, T, list);
    else
        hipLaunchKernelGGL((k_sweep<B, false>), dim3(n), dim3(64), 0, s, T, list);
    return hipGetLastError();
}

template <int B>
hipError_t energy_b(const Tables &T, const int32_t *list, int n, double *oe, double *ob, int by_slot,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_energy<B>), dim3(n), dim3(64), 0, s, T, list, oe, ob, by_slot);
    return hipGetLastError();
}

template <int B>
hipError_t exchange_b(const Tables &T, const int32_t *list, int nc, int mp, int force, hipStream_t s) {
    hipLaunchKernelGGL((k_exchange<B>), dim3(nc * mp), dim3(64), 0, s, T, list, mp, force);
    return hipGetLastError();
}

}  // namespace

#define PT_DISPATCH_B(bpl, CALL)             \
    switch (bpl) {                           \
        case 1: return CALL(1);              \
        case 2: return CALL(2);              \
        case 4: return CALL(4);              \
        case 8: return CALL(8);              \
        case 16: return CALL(16);            \
        case 32: return CALL(32);            \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_sweep(int bpl, bool mixed, const Tables &T, const int32_t *list, int n,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define PT_SW(B) sweep_b<B>(mixed, T, list, n, s)
    PT_DISPATCH_B(bpl, PT_SW)
#undef PT_SW
}

hipError_t launch_energy(int bpl, const Tables &T, const int32_t *list, int n, double *out_e,
                         double *out_b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int by_slot = (out_b == nullptr) ? 1 : 0;
#define PT_EN(B) energy_b<B>(T, list, n, out_e, out_b, by_slot, s)
    PT_DISPATCH_B(bpl, PT_EN)
#undef PT_EN
}

hipError_t launch_exchange(int bpl, const Tables &T, const int32_t *list, int n_chains,
                           int max_pairs, int force, hipStream_t s) {
    if (n_chains <= 0 || max_pairs <= 0) return hipSuccess;
#define PT_EX(B) exchange_b<B>(T, list, n_chains, max_pairs, force, s)
    PT_DISPATCH_B(bpl, PT_EX)
#undef PT_EX
}

hipError_t launch_advance(const Tables &T, int exchange_only, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, T, exchange_only);
    return hipGetLastError();
}

hipError_t launch_selftest(const Consts &k, int op, const double *x, const double *y, double *out,
                           int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_selftest, dim3((unsigned)blocks), dim3(256), 0, s, k, op, x, y, out, n);
    return hipGetLastError();
}

}  // namespace pt
