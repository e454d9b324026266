// pt_kernels.hip -- gfx950 kernels of libpt.so: Metropolis sweeps of single-
// monomer moves, the FP64-order energy, and neighbour-temperature replica
// exchange for a bead-spring homopolymer (Gross, Janke, Bachmann,
// arXiv:1107.3490, Secs. 3.1-3.4).
//
// Mapping.  A replica is owned by W wavefronts (W = 1, 2 or 4; 64 W lanes),
// each lane holding the contiguous bead block [t B, (t+1) B) of the padded
// range of NP = 64 W B beads (t = thread index in the block, B <= 8), in
// registers.  LDS mirrors the replica's FP64 coordinates in a swizzled SoA
// layout -- bead j at (j mod B) 64 W + j / B -- so that block-wide copies and
// the per-bead accesses of the 64 W lanes touch consecutive doubles; HBM keeps
// the same layout.  Beads past the chain end hold a far-away sentinel x
// coordinate, so their pair terms are exact zeros.
//
// The pair sum of a move is the pairwise tree over each lane's block, the
// register butterfly over the 64 lanes of a wavefront, and the pairwise tree
// over the W wavefront sums: the FP64-order sum of the public header for
// every (B, W).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_device.hpp"
#include "pt_internal.hpp"

namespace pt {

namespace {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int B, int W>
struct Geo {
    static constexpr int NT = 64 * W;  // lanes owning the replica in a sweep
    static constexpr int NP = NT * B;  // padded bead range
    static constexpr int LOGB = ilog2(B);
    static constexpr int LOGW = ilog2(W);
    static constexpr int LOG_NP = 6 + LOGW + LOGB;
    __device__ static __forceinline__ int pos(int j) {
        return ((j & (B - 1)) << (6 + LOGW)) | (j >> LOGB);
    }
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

// Pushes v as leaf number idx (0, 1, 2, ... in order) of a pairwise tree kept
// as a binary counter: stk[l] holds the pending left sibling of size 2^l.
// idx is uniform across the wavefront; after leaf 2^L - 1 the complete tree
// over 2^L leaves sits in stk[L].
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

// Pairwise tree over the 64 leaves j = j0 .. j0+63 of row i (zero unless
// i < j < n), computed in registers from LDS broadcasts.
template <int B, int W, int LO, int HI>
__device__ __forceinline__ double row_chunk(const double *X, const double *Y, const double *Z,
                                            const Consts &k, int i, int n, int j0, double xi,
                                            double yi, double zi) {
    if constexpr (HI - LO == 1) {
        const int j = j0 + LO;
        const int a = Geo<B, W>::pos(j);
        const double v = lj64(k, sq3(X[a] - xi, Y[a] - yi, Z[a] - zi));
        return (j > i && j < n) ? v : 0.0;
    } else {
        constexpr int MID = (LO + HI) / 2;
        const double l = row_chunk<B, W, LO, MID>(X, Y, Z, k, i, n, j0, xi, yi, zi);
        const double r = row_chunk<B, W, MID, HI>(X, Y, Z, k, i, n, j0, xi, yi, zi);
        return l + r;
    }
}

// FP64-order energy E(C) of Eq. (4) for the replica in LDS, on one wavefront
// (lanes 0..63 of the calling block).  The rows are taken in aligned blocks of
// 64: lane l computes row 64 r + l, each row being the tree over j in chunks
// of 64 (static trees chained by a binary counter; chunks left of the block
// or past the chain end are exact zeros and are skipped); the butterfly over
// lanes gives the tree over the block's 64 rows, and a binary counter over r
// the tree over all NP rows.  Bonds: contiguous lane blocks and the butterfly.
template <int B, int W>
__device__ double energy_wave(const double *X, const double *Y, const double *Z, int n,
                              const Consts &k) {
    using G = Geo<B, W>;
    constexpr int BP = B * W;  // 64-row blocks = 64-leaf chunks per row
    constexpr int LC = ilog2(BP);
    const int lane = threadIdx.x & 63;
    double blk[LC + 1];
#pragma unroll
    for (int l = 0; l <= LC; ++l) blk[l] = 0.0;
    for (int r = 0; r < BP; ++r) {
        double bv = 0.0;
        if (r * 64 < n) {
            const int i = r * 64 + lane;
            const int ai = G::pos(i);
            const double xi = X[ai], yi = Y[ai], zi = Z[ai];
            double row[LC + 1];
#pragma unroll
            for (int l = 0; l <= LC; ++l) row[l] = 0.0;
            for (int c = 0; c < BP; ++c) {
                double v = 0.0;
                if (c >= r && c * 64 < n) v = row_chunk<B, W, 0, 64>(X, Y, Z, k, i, n, c * 64, xi, yi, zi);
                tree_push<LC>(row, c, v);
            }
            bv = wave_tree(row[LC]);
        }
        tree_push<LC>(blk, r, bv);
    }
    const double e_lj = blk[LC];
    const double fb = lane_tree<0, BP>([&](int b) {
        const int i = lane * BP + b;
        const int i0 = (i < n - 1) ? i : 0;
        const int a0 = G::pos(i0), a1 = G::pos(i0 + 1);
        const double v = fene64(k, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
        return (i < n - 1) ? v : 0.0;
    });
    return e_lj + wave_tree(fb);
}

// Squared end-to-end distance and squared radius of gyration (Eq. 8) of the
// replica in LDS, one wavefront: means and the sum of squares as lane-block
// trees plus the butterfly.
template <int B, int W>
__device__ void shape_wave(const double *X, const double *Y, const double *Z, int n,
                           double &ree2, double &rg2) {
    using G = Geo<B, W>;
    constexpr int BP = B * W;
    const int lane = threadIdx.x & 63;
    const int a0 = G::pos(0), a1 = G::pos(n - 1);
    ree2 = sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]);
    auto mean = [&](const double *C) {
        const double s = lane_tree<0, BP>([&](int b) {
            const int j = lane * BP + b;
            return (j < n) ? C[G::pos(j)] : 0.0;
        });
        return wave_tree(s) / (double)n;
    };
    const double mx = mean(X), my = mean(Y), mz = mean(Z);
    const double s = lane_tree<0, BP>([&](int b) {
        const int j = lane * BP + b;
        const int a = G::pos(j);
        const double v = sq3(X[a] - mx, Y[a] - my, Z[a] - mz);
        return (j < n) ? v : 0.0;
    });
    rg2 = wave_tree(s) / (double)n;
}

// Copy a replica (x, y, z arrays back to back) with NTH threads of the block.
template <int B, int W, int NTH>
__device__ __forceinline__ void copy_replica(double *dst, const double *src) {
    constexpr int TOT = 3 * Geo<B, W>::NP;
    for (int i = threadIdx.x; i < TOT; i += NTH) dst[i] = src[i];
}

// ------------------------------------------------------------------ sweep --
// What the batch prologue knows about one move: its draws, and, at the start
// of the batch, r_k and the two bond differences.  These stay valid unless an
// earlier move of the same batch that touched k-1, k or k+1 was accepted;
// `conflict` lists the earlier moves of the batch with |k' - k| <= 1.
struct MoveRec {
    double dx, dy, dz, th;
    double xo, yo, zo;
    double dfl, dfr;
    uint64_t conflict;
    int k;
    int pad;
};

// Sum of the W per-wavefront values v[0..W) as a pairwise tree.
template <int W>
__device__ __forceinline__ double tree_w(const double *v) {
    if constexpr (W == 1) return v[0];
    else if constexpr (W == 2) return v[0] + v[1];
    else return (v[0] + v[1]) + (v[2] + v[3]);
}

// One sweep (N attempted moves, Sec. 3.2) of every slot in `list`, then the
// per-sweep record of E, Ree^2 and Rg^2 (Eq. 8).
//
// Moves are processed in batches.  A vector prologue (wavefront 0, one move
// per lane) computes the Philox draws, -log u, the gather of r_k and of its
// bond neighbours, the four bond terms and the conflict mask.  The serial part
// of a move is then the pair loop over the lane's beads in registers, the
// butterflies, one barrier to combine the W wavefront sums (W > 1), and the
// decision, taken identically by every wavefront.
template <int B, int W, bool MIXED>
__global__ __launch_bounds__(64 * W) void k_sweep(const Tables T, const int32_t *__restrict__ list) {
    using G = Geo<B, W>;
    constexpr int NT = G::NT;
    constexpr int MB = (W >= 4) ? 32 : 64;  // moves per batch (LDS budget at W = 4)
    __shared__ double XYZ[3 * G::NP];
    double *const X = XYZ, *const Y = XYZ + G::NP, *const Z = XYZ + 2 * G::NP;
    __shared__ MoveRec rec[MB];
    __shared__ double part[2][2][W];
    __shared__ double partx[2][W];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
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
    copy_replica<B, W, NT>(XYZ, cq);
    __syncthreads();
    double rx[B], ry[B], rz[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        rx[b] = X[b * NT + tid];
        ry[b] = Y[b * NT + tid];
        rz[b] = Z[b * NT + tid];
    }

    double E = T.e_run[q], Bd = T.b_run[q];
    int64_t n_acc = 0, n_rescore = 0;
    uint64_t *logrow = (T.accept_log != nullptr && t64 < T.log_cap)
                           ? T.accept_log + t64 * T.words_total + T.word_off[g]
                           : nullptr;
    uint64_t logword = 0;

    for (int m0 = 0; m0 < n; m0 += MB) {
        __syncthreads();  // commits of the previous batch visible, rec[] free
        if (wv == 0) {
            // ---- prologue: move m0 + lane (Philox counters (m, t, g, 0), (m, t, g, 1))
            const uint32_t m = (uint32_t)(m0 + lane);
            const U4 w = philox10(U4{m, t, gid, 0u}, T.seed);
            const U4 v = philox10(U4{m, t, gid, 1u}, T.seed);
            MoveRec r;
            r.k = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)n) >> 32);
            r.dx = (unit_open(w.y) - 0.5) * K.edge;
            r.dy = (unit_open(w.z) - 0.5) * K.edge;
            r.dz = (unit_open(w.w) - 0.5) * K.edge;
            r.th = -det_log(unit_open(v.x));
            const int k = r.k;
            const int ak = G::pos(k);
            r.xo = X[ak];
            r.yo = Y[ak];
            r.zo = Z[ak];
            const double xn = r.xo + r.dx, yn = r.yo + r.dy, zn = r.zo + r.dz;
            const bool hl = k > 0, hr = k + 1 < n;
            const int al = G::pos(hl ? k - 1 : k), ar = G::pos(hr ? k + 1 : k);
            const double xl = X[al], yl = Y[al], zl = Z[al];
            const double xr = X[ar], yr = Y[ar], zr = Z[ar];
            const double fln = fene64(K, sq3(xl - xn, yl - yn, zl - zn));
            const double flo = fene64(K, sq3(xl - r.xo, yl - r.yo, zl - r.zo));
            const double frn = fene64(K, sq3(xr - xn, yr - yn, zr - zn));
            const double fro = fene64(K, sq3(xr - r.xo, yr - r.yo, zr - r.zo));
            r.dfl = hl ? fln - flo : 0.0;
            r.dfr = hr ? frn - fro : 0.0;
            uint64_t cm = 0;
            for (int j = 0; j < MB; ++j) {
                const int dd = read_lane(k, j) - k;
                cm |= (j < lane && dd >= -1 && dd <= 1) ? (1ull << j) : 0ull;
            }
            r.conflict = cm;
            r.pad = 0;
            if (lane < MB) rec[lane] = r;
        }
        __syncthreads();
        const int nb = (n - m0 < MB) ? (n - m0) : MB;
        uint64_t bits = 0;
        // The last committed move: earlier commits are visible in LDS to every
        // wavefront, this one possibly not yet to the other wavefronts.
        int last_k = -1;
        double lx = 0.0, ly = 0.0, lz = 0.0;
        for (int i = 0; i < nb; ++i) {
            const MoveRec r = rec[i];
            const int k = __builtin_amdgcn_readfirstlane(r.k);
            const uint64_t cf =
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)r.conflict)) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(r.conflict >> 32)) << 32);
            const double th = r.th;
            double xo = r.xo, yo = r.yo, zo = r.zo, dfl = r.dfl, dfr = r.dfr;
            if ((cf & bits) != 0) {
                // An accepted move of this batch touched k-1, k or k+1: redo the
                // gather and the bond terms from the current replica (lanes 0..3
                // of each wavefront evaluate (k-1,k) new/old, (k,k+1) new/old).
                auto fetch = [&](int a, double &x, double &y, double &z) {
                    const int p = G::pos(a);
                    x = X[p];
                    y = Y[p];
                    z = Z[p];
                    if (W > 1 && a == last_k) {
                        x = lx;
                        y = ly;
                        z = lz;
                    }
                };
                fetch(k, xo, yo, zo);
                const double xq = xo + r.dx, yq = yo + r.dy, zq = zo + r.dz;
                const int nbr = (lane & 2) ? k + 1 : k - 1;
                const bool has = nbr >= 0 && nbr < n;
                double xa, ya, za;
                fetch(has ? nbr : k, xa, ya, za);
                const bool nw = (lane & 1) == 0;
                const double fb = fene64(K, sq3(xa - (nw ? xq : xo), ya - (nw ? yq : yo),
                                                za - (nw ? zq : zo)));
                const double fv = has ? fb : 0.0;
                dfl = read_lane(fv, 0) - read_lane(fv, 1);
                dfr = read_lane(fv, 2) - read_lane(fv, 3);
            }
            const double xn = xo + r.dx, yn = yo + r.dy, zn = zo + r.dz;
            const double df = dfl + dfr;
            const int owner = k >> G::LOGB, slot = k & (B - 1);
            const bool mine = (tid == owner);

            auto leaf64 = [&](int b) {
                const double en = lj64(K, sq3(rx[b] - xn, ry[b] - yn, rz[b] - zn));
                const double eo = lj64(K, sq3(rx[b] - xo, ry[b] - yo, rz[b] - zo));
                const double tt = (mine && b == slot) ? 0.0 : en - eo;
                return Leaf64{tt, dabs(tt)};
            };
            bool acc = false;
            double de_used = 0.0, bm = 0.0;
            bool exact = !MIXED;
            if constexpr (MIXED) {
                const LeafMx s = lane_tree<0, B>([&](int b) {
                    const Lj32 pn = lj32(K, rx[b] - xn, ry[b] - yn, rz[b] - zn);
                    const Lj32 po = lj32(K, rx[b] - xo, ry[b] - yo, rz[b] - zo);
                    const bool self = mine && b == slot;
                    const float tt = self ? 0.0f : pn.e - po.e;
                    const float bb = self ? 0.0f : pn.b + po.b;
                    return LeafMx{(double)tt, bb};
                });
                double sm = wave_tree(s.t);
                double bsum = (double)wave_tree(s.b);
                if constexpr (W > 1) {
                    if (lane == 0) {
                        part[i & 1][0][wv] = sm;
                        part[i & 1][1][wv] = bsum;
                    }
                    __syncthreads();
                    sm = tree_w<W>(part[i & 1][0]);
                    bsum = tree_w<W>(part[i & 1][1]);
                }
                const double bs = K.kbound * bsum;
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
                double sc = wave_tree(s.t);
                double ab = wave_tree(s.a);
                if constexpr (W > 1) {
                    double *pp = MIXED ? partx[0] : part[i & 1][0];
                    double *pa = MIXED ? partx[1] : part[i & 1][1];
                    if (lane == 0) {
                        pp[wv] = sc;
                        pa[wv] = ab;
                    }
                    __syncthreads();
                    sc = tree_w<W>(pp);
                    ab = tree_w<W>(pa);
                }
                const double de = sc + df;
                acc = (de <= 0.0) || (beta * de < th);
                de_used = de;
                bm = bound64(G::LOG_NP, ab, dfl, dfr, de);
            }
            if (acc) {
                if (mine) {
                    const int ak = G::pos(k);
                    X[ak] = xn;
                    Y[ak] = yn;
                    Z[ak] = zn;
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const bool me = mine && b == slot;
                    rx[b] = me ? xn : rx[b];
                    ry[b] = me ? yn : ry[b];
                    rz[b] = me ? zn : rz[b];
                }
                E = E + de_used;
                Bd = Bd + bm + 0x1p-52 * dabs(E);
                ++n_acc;
                bits |= 1ull << i;
                last_k = k;
                lx = xn;
                ly = yn;
                lz = zn;
            } else {
                last_k = -1;
            }
            wave_sync();
        }
        logword |= bits << (m0 & 63);
        if (logrow != nullptr && tid == 0 && (((m0 + MB) & 63) == 0 || m0 + MB >= n))
            logrow[m0 >> 6] = logword;
        if (((m0 + MB) & 63) == 0) logword = 0;
    }

    // Write the replica back; record the sweep (before any exchange); re-sync
    // the running energy with the FP64-order energy when its bound has grown past
    // resync_rel of max(1, |E|) (a start with near-overlapping beads, or many
    // accepted moves).
    __syncthreads();
    copy_replica<B, W, NT>(cq, XYZ);
    if (wv == 0) {
        double ree2, rg2;
        shape_wave<B, W>(X, Y, Z, n, ree2, rg2);
        bool resync = false;
        if (!(Bd <= K.resync_rel * (dabs(E) > 1.0 ? dabs(E) : 1.0))) {
            E = energy_wave<B, W>(X, Y, Z, n, K);
            Bd = bound_energy(K, G::LOG_NP, n, E, 0.0);
            resync = true;
        }
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
}

// ----------------------------------------------------------------- energy --
// FP64-order energy of the conformations in `list` (by_slot: list holds slots
// and the conformation is perm[g]); writes out_e / out_b indexed like list.
template <int B, int W>
__global__ __launch_bounds__(64) void k_energy(const Tables T, const int32_t *__restrict__ list,
                                               double *out_e, double *out_b, int by_slot) {
    using G = Geo<B, W>;
    __shared__ double XYZ[3 * G::NP];
    double *const X = XYZ, *const Y = XYZ + G::NP, *const Z = XYZ + 2 * G::NP;
    const int id = list[blockIdx.x];
    const int q = by_slot ? T.perm[id] : id;
    const int c = T.slot_chain[q];  // conformation q started in slot q: same chain
    const int n = T.chain_n[c];
    copy_replica<B, W, 64>(XYZ, T.coords + T.coord_off[q]);
    wave_sync();
    const double e = energy_wave<B, W>(X, Y, Z, n, T.k);
    if (threadIdx.x == 0) {
        out_e[id] = e;
        if (out_b != nullptr) out_b[id] = bound_energy(T.k, G::LOG_NP, n, e, 0.0);
    }
}

// --------------------------------------------------------------- exchange --
// One exchange step (Sec. 3.3, Eq. 6) for the chains in `list`: wavefront p of
// a chain handles the pair (i, i+1), i = (e mod 2) + 2p.  The decision is
// taken from the running energies when their bounds settle it, otherwise from
// the FP64-order energies of both conformations (which also re-synchronise
// them).
template <int B, int W>
__global__ __launch_bounds__(64) void k_exchange(const Tables T, const int32_t *__restrict__ list,
                                                 int max_pairs, int force) {
    using G = Geo<B, W>;
    __shared__ double XYZ[3 * G::NP];
    double *const X = XYZ, *const Y = XYZ + G::NP, *const Z = XYZ + 2 * G::NP;
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
        copy_replica<B, W, 64>(XYZ, T.coords + T.coord_off[q1]);
        wave_sync();
        const double c1 = energy_wave<B, W>(X, Y, Z, n, T.k);
        wave_sync();
        copy_replica<B, W, 64>(XYZ, T.coords + T.coord_off[q2]);
        wave_sync();
        const double c2 = energy_wave<B, W>(X, Y, Z, n, T.k);
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

template <int B, int W>
hipError_t sweep_bw(bool mixed, const Tables &T, const int32_t *list, int n, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL((k_sweep<B, W, true>), dim3(n), dim3(64 * W), 0, s, T, list);
    else
        hipLaunchKernelGGL((k_sweep<B, W, false>), dim3(n), dim3(64 * W), 0, s, T, list);
    return hipGetLastError();
}

template <int B, int W>
hipError_t energy_bw(const Tables &T, const int32_t *list, int n, double *oe, double *ob, int by_slot,
                     hipStream_t s) {
    hipLaunchKernelGGL((k_energy<B, W>), dim3(n), dim3(64), 0, s, T, list, oe, ob, by_slot);
    return hipGetLastError();
}

template <int B, int W>
hipError_t exchange_bw(const Tables &T, const int32_t *list, int nc, int mp, int force, hipStream_t s) {
    hipLaunchKernelGGL((k_exchange<B, W>), dim3(nc * mp), dim3(64), 0, s, T, list, mp, force);
    return hipGetLastError();
}

}  // namespace

// The (beads per lane, wavefronts per replica) classes the library builds.
#define PT_DISPATCH(bpl, wpr, CALL)           \
    switch ((bpl) * 16 + (wpr)) {             \
        case 1 * 16 + 1: return CALL(1, 1);   \
        case 2 * 16 + 1: return CALL(2, 1);   \
        case 4 * 16 + 1: return CALL(4, 1);   \
        case 8 * 16 + 1: return CALL(8, 1);   \
        case 8 * 16 + 2: return CALL(8, 2);   \
        case 8 * 16 + 4: return CALL(8, 4);   \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_sweep(int bpl, int wpr, bool mixed, const Tables &T, const int32_t *list, int n,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define PT_SW(B, W) sweep_bw<B, W>(mixed, T, list, n, s)
    PT_DISPATCH(bpl, wpr, PT_SW)
#undef PT_SW
}

hipError_t launch_energy(int bpl, int wpr, const Tables &T, const int32_t *list, int n, double *out_e,
                         double *out_b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int by_slot = (out_b == nullptr) ? 1 : 0;
#define PT_EN(B, W) energy_bw<B, W>(T, list, n, out_e, out_b, by_slot, s)
    PT_DISPATCH(bpl, wpr, PT_EN)
#undef PT_EN
}

hipError_t launch_exchange(int bpl, int wpr, const Tables &T, const int32_t *list, int n_chains,
                           int max_pairs, int force, hipStream_t s) {
    if (n_chains <= 0 || max_pairs <= 0) return hipSuccess;
#define PT_EX(B, W) exchange_bw<B, W>(T, list, n_chains, max_pairs, force, s)
    PT_DISPATCH(bpl, wpr, PT_EX)
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
