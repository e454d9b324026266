// pt_kernels.hpp -- device code of the gfx950 kernels of libpt.so: Metropolis
// sweeps of single-monomer moves, the FP64-order energy, and neighbour-
// temperature replica exchange for a bead-spring homopolymer (Gross, Janke,
// Bachmann, arXiv:1107.3490, Secs. 3.1-3.4).  Included by the translation
// units that instantiate and launch the kernels (pt_k_*.hip), so that they
// compile in parallel; everything here has internal linkage.
#pragma once
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
    float t, b;
    __device__ LeafMx operator+(const LeafMx &o) const { return LeafMx{t + o.t, b + o.b}; }
};

// One leaf of the mixed-precision pair sum of a move: bead (x, y, z) against
// the moved bead's new and old positions; the FP32 difference of the two
// Lennard-Jones brackets and the bead's term of the error bound (S^2 + S,
// S = sum of the two s6), both exact zeros when skip (the moved bead itself,
// a padding bead).
__device__ __forceinline__ LeafMx mixed_leaf(const Consts &K, double x, double y, double z, double xn,
                                             double yn, double zn, double xo, double yo, double zo,
                                             bool skip) {
    const Lj32 pn = lj32(K, sq3(x - xn, y - yn, z - zn));
    const Lj32 po = lj32(K, sq3(x - xo, y - yo, z - zo));
    const float sb = pn.s6 + po.s6;
    const float tt = skip ? 0.0f : pn.g - po.g;
    const float bb = skip ? 0.0f : __builtin_fmaf(sb, sb, sb);
    return LeafMx{tt, bb};
}

__device__ __forceinline__ double dabs(double v) { return __builtin_fabs(v); }

// The value of lane l ^ 32 (v_permlane32_swap of two copies leaves the lower
// half's value in the first output and the upper half's in the second, in
// every lane).
__device__ __forceinline__ uint32_t other_half(uint32_t v) {
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? p[0] : p[1];
}
__device__ __forceinline__ double other_half(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = other_half((uint32_t)b), hi = other_half((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Bound on |E_run - exact sum of the FP64-order terms| added by one accepted
// move scored in the FP64 order: the leaf differences (u each), the tree over
// the leaves (depth log2 NP, u |partial| each), the two bond differences, their
// sum and the final addition, all with a factor-two margin (2^-52 for u).
// abs_leaves must be an upper bound on the sum of the leaf magnitudes.
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
template <int LEVELS, class V>
__device__ __forceinline__ void tree_push(V (&stk)[LEVELS + 1], int idx, V v) {
    V carry = v;
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

// Pairwise tree over the leaves j = j0 + LO .. j0 + HI - 1 of row i (zero
// unless i < j < n), computed in registers from broadcast loads.
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

// FP64-order energy E(C) of Eq. (4) of a replica stored in the swizzled layout
// (LDS or HBM).  The rows are taken in aligned blocks of 64: lane l computes
// row 64 r + l, each row being the tree over j in chunks of 16 (static trees
// chained by a binary counter; chunks left of the block or past the chain end
// are exact zeros and are skipped); the butterfly over lanes gives the tree
// over the block's 64 rows, and a binary counter over r the tree over all NP
// rows.  Bonds: contiguous lane blocks and the butterfly.
//
// Sum of the 64-row block r, on one wavefront.
template <int B, int W>
__device__ __forceinline__ double row_block(const double *X, const double *Y, const double *Z, int n,
                                            const Consts &k, int r) {
    using G = Geo<B, W>;
    constexpr int CW = 16;           // leaves per chunk
    constexpr int NC = G::NP / CW;   // chunks per row
    constexpr int LR = ilog2(NC);
    if (r * 64 >= n) return 0.0;
    const int lane = threadIdx.x & 63;
    const int i = r * 64 + lane;
    const int ai = G::pos(i);
    const double xi = X[ai], yi = Y[ai], zi = Z[ai];
    double row[LR + 1];
#pragma unroll
    for (int l = 0; l <= LR; ++l) row[l] = 0.0;
    for (int c = 0; c < NC; ++c) {
        double v = 0.0;
        if (c * CW + CW > r * 64 && c * CW < n)
            v = row_chunk<B, W, 0, CW>(X, Y, Z, k, i, n, c * CW, xi, yi, zi);
        tree_push<LR>(row, c, v);
    }
    return wave_tree(row[LR]);
}

// The bond part, on one wavefront.
template <int B, int W>
__device__ __forceinline__ double bonds_wave(const double *X, const double *Y, const double *Z, int n,
                                             const Consts &k) {
    using G = Geo<B, W>;
    constexpr int BP = B * W;
    const int lane = threadIdx.x & 63;
    const double fb = lane_tree<0, BP>([&](int b) {
        const int i = lane * BP + b;
        const int i0 = (i < n - 1) ? i : 0;
        const int a0 = G::pos(i0), a1 = G::pos(i0 + 1);
        const double v = fene64(k, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
        return (i < n - 1) ? v : 0.0;
    });
    return wave_tree(fb);
}

// The whole energy on one wavefront (lanes 0..63 of the calling block).
template <int B, int W>
__device__ __forceinline__ double energy_wave(const double *X, const double *Y, const double *Z, int n,
                              const Consts &k) {
    constexpr int BP = B * W;        // 64-row blocks
    constexpr int LC = ilog2(BP);
    double blk[LC + 1];
#pragma unroll
    for (int l = 0; l <= LC; ++l) blk[l] = 0.0;
    for (int r = 0; r < BP; ++r) tree_push<LC>(blk, r, row_block<B, W>(X, Y, Z, n, k, r));
    return blk[LC] + bonds_wave<B, W>(X, Y, Z, n, k);
}

// The same energy, bit for bit, with all W wavefronts of the block: wavefront
// w takes the row blocks r = w, w + W, ..., the last one also the bonds; the
// block sums meet in LDS (sh: B W + 1 doubles) and every thread chains them
// with the same binary counter.  Called by every thread of the block; returns
// the energy in every thread.
template <int B, int W>
__device__ __forceinline__ double energy_block(const double *X, const double *Y, const double *Z, int n,
                               const Consts &k, double *sh) {
    if constexpr (W == 1) {
        return energy_wave<B, W>(X, Y, Z, n, k);
    } else {
        constexpr int BP = B * W;
        constexpr int LC = ilog2(BP);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int r = wv; r < BP; r += W) {
            const double bv = row_block<B, W>(X, Y, Z, n, k, r);
            if (lane == 0) sh[r] = bv;
        }
        if (wv == W - 1) {
            const double fb = bonds_wave<B, W>(X, Y, Z, n, k);
            if (lane == 0) sh[BP] = fb;
        }
        __syncthreads();
        double blk[LC + 1];
#pragma unroll
        for (int l = 0; l <= LC; ++l) blk[l] = 0.0;
        for (int r = 0; r < BP; ++r) tree_push<LC>(blk, r, sh[r]);
        const double e = blk[LC] + sh[BP];
        __syncthreads();  // sh free again
        return e;
    }
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
    double thb;  // th / beta: the mixed path's sure tests compare energies with it
    double xo, yo, zo;
    double dfl, dfr;
    uint64_t conflict;
    int k;
    int pad;
};

// Sum of the W per-wavefront values v[0..W) as a pairwise tree, in FP64
// (tree_w) or, for values that are FP32 sums, in FP32 (tree_wf), so that the
// whole sum is the pairwise tree over the padded bead range in one precision
// for every mapping.
template <int W>
__device__ __forceinline__ double tree_w(const double *v) {
    if constexpr (W == 1) return v[0];
    else if constexpr (W == 2) return v[0] + v[1];
    else return (v[0] + v[1]) + (v[2] + v[3]);
}

template <int W>
__device__ __forceinline__ float tree_wf(const float *v) {
    if constexpr (W == 1) return v[0];
    else if constexpr (W == 2) return v[0] + v[1];
    else return (v[0] + v[1]) + (v[2] + v[3]);
}

// ceil(log2 n), n >= 2: the depth of the pairwise tree over n leaves padded
// with zeros to a power of two (levels over padding add exact zeros).
__device__ __forceinline__ int log2c(int n) { return 32 - __builtin_clz((unsigned)(n - 1)); }

// LDS of a sweep block: the replica mirror, the batch's move records and the
// per-wavefront partial sums (double-buffered over consecutive moves).
template <int B, int W>
struct SweepLds {
    // Moves per batch: 32 at the LDS budget of 2048 beads, and for short
    // chains, where an accepted move more often touches a later move's
    // bonds (which then recomputes them); 64 otherwise.
    static constexpr int MB = (Geo<B, W>::NP >= 2048 || Geo<B, W>::NP <= 128) ? 32 : 64;
    double xyz[3 * Geo<B, W>::NP];
    MoveRec rec[MB];
    double part[2][2][W];
    float partf[2][2][W];
    double partx[2][W];
    double bcast[4];
    double eblk[B * W + 1];  // energy_block
    Consts kc;               // model constants for the rare paths of the mixed move (four wavefronts)
};

// The N moves of one sweep of the replica held by the block (Sec. 3.2), on
// slot g at sweep t.  Moves are processed in batches.  A vector prologue
// (wavefront 0, one move per lane) computes the Philox draws, -log u, the
// gather of r_k and of its bond neighbours, the four bond terms and the
// conflict mask.  The serial part of a move is the pair loop over the lane's
// beads in registers, the butterflies, one barrier to combine the W wavefront
// sums (W > 1), and the decision, taken identically by every wavefront.
template <int B, int W, bool MIXED, bool SPLIT_OK = true>
__device__ __forceinline__ void sweep_moves(const Tables &T, SweepLds<B, W> &S, double (&rx)[B],
                                            double (&ry)[B], double (&rz)[B], int g, int n,
                                            uint32_t t, int64_t t64, double &E, double &Bd,
                                            int64_t &n_acc, int64_t &n_rescore) {
    using G = Geo<B, W>;
    constexpr int MB = SweepLds<B, W>::MB;
    double *const X = S.xyz, *const Y = S.xyz + G::NP, *const Z = S.xyz + 2 * G::NP;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const Consts &K = T.k;
    const double beta = T.beta[g];
    const uint32_t gid = T.slot_gid[g];
    const bool fp64_on_accept = MIXED && T.fp64_on_accept != 0;
    const double kb_band = K.kbound * (1.0 + 0x1p-20) * T.guard_scale;
    const double rel_band = 0x1p-50 * T.guard_scale;
    uint64_t *logrow = (T.accept_log != nullptr && t64 < T.log_cap)
                           ? T.accept_log + t64 * T.words_total + T.word_off[g]
                           : nullptr;
    uint64_t logword = 0;
    uint64_t digest = (tid == 0) ? T.dig[2 * g] : 0;
    // At four wavefronts the mixed move's rarely taken paths (the FP64
    // re-score, about one move in 10^4, and the bond terms of a move that
    // conflicts with an earlier accepted one) read the constants from LDS,
    // behind a compiler barrier, so that they do not hold scalar registers
    // across the move loop: the compiler otherwise spills scalar registers into
    // vector lanes and restores 13 of them before every decision (N = 500 x
    // 128: 0.457 -> 0.432 ms per sweep).
    // At one and two wavefronts the same change made the compiler spill more
    // (2.5% and 3.8% slower), and at 8 beads per lane (N = 2000 x 4096) it
    // changed nothing beyond the noise, so there the constants stay where they are.
    constexpr bool lds_consts = MIXED && W == 4 && B <= 4;
    if constexpr (lds_consts)
        if (tid == 0) S.kc = K;

    for (int m0 = 0; m0 < n; m0 += MB) {
        __syncthreads();  // commits of the previous batch visible, rec[] free
        if (wv == 0) {
            // ---- prologue: move m0 + lane (Philox counters (m, t, g, 0), (m, t, g, 1))
            // With 32 moves per batch the two halves of the wavefront share
            // each move's work: lanes 0..31 draw its first Philox block and
            // form the bond (k-1, k), lanes 32..63 the second block and the
            // bond (k, k+1); a row swap hands each half the other's values.
            // Same operations on the same operands as one lane doing both.
            constexpr bool SPLIT = SPLIT_OK && MB == 32;
            const bool hi = SPLIT && lane >= 32;
            const uint32_t m = (uint32_t)(m0 + (SPLIT ? (lane & 31) : lane));
            U4 w, v;
            if constexpr (SPLIT) {
                const U4 p = philox10(U4{m, t, gid, hi ? 1u : 0u}, T.seed);
                const U4 q{other_half(p.x), other_half(p.y), other_half(p.z), other_half(p.w)};
                w = hi ? q : p;
                v = hi ? p : q;
            } else {
                w = philox10(U4{m, t, gid, 0u}, T.seed);
                v = philox10(U4{m, t, gid, 1u}, T.seed);
            }
            MoveRec r;
            r.k = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)n) >> 32);
            r.dx = (unit_open(w.y) - 0.5) * K.edge;
            r.dy = (unit_open(w.z) - 0.5) * K.edge;
            r.dz = (unit_open(w.w) - 0.5) * K.edge;
            r.th = -det_log(unit_open(v.x));
            // th / beta, +inf at beta = 0; NaN where it would be so small
            // (beta beyond 2^1000 th) that its relative rounding is not 2^-53.
            const double thb = r.th / beta;
            r.thb = (thb >= 0x1p-1000) ? thb : __builtin_nan("");
            const int k = r.k;
            const int ak = G::pos(k);
            r.xo = X[ak];
            r.yo = Y[ak];
            r.zo = Z[ak];
            const double xn = r.xo + r.dx, yn = r.yo + r.dy, zn = r.zo + r.dz;
            const bool hl = k > 0, hr = k + 1 < n;
            if constexpr (SPLIT) {
                const bool has = hi ? hr : hl;
                const int ab = G::pos(has ? (hi ? k + 1 : k - 1) : k);
                const double xb = X[ab], yb = Y[ab], zb = Z[ab];
                const double fbn = fene64(K, sq3(xb - xn, yb - yn, zb - zn));
                const double fbo = fene64(K, sq3(xb - r.xo, yb - r.yo, zb - r.zo));
                const double dfb = has ? fbn - fbo : 0.0;
                const double dfo = other_half(dfb);
                r.dfl = hi ? dfo : dfb;
                r.dfr = hi ? dfb : dfo;
            } else {
                const int al = G::pos(hl ? k - 1 : k), ar = G::pos(hr ? k + 1 : k);
                const double xl = X[al], yl = Y[al], zl = Z[al];
                const double xr = X[ar], yr = Y[ar], zr = Z[ar];
                const double fln = fene64(K, sq3(xl - xn, yl - yn, zl - zn));
                const double flo = fene64(K, sq3(xl - r.xo, yl - r.yo, zl - r.zo));
                const double frn = fene64(K, sq3(xr - xn, yr - yn, zr - zn));
                const double fro = fene64(K, sq3(xr - r.xo, yr - r.yo, zr - r.zo));
                r.dfl = hl ? fln - flo : 0.0;
                r.dfr = hr ? frn - fro : 0.0;
            }
            uint64_t cm = 0;
            for (int j = 0; j < MB; ++j) {
                const int dd = read_lane(k, j) - k;
                cm |= (j < lane && dd >= -1 && dd <= 1) ? (1ull << j) : 0ull;
            }
            r.conflict = cm;
            r.pad = 0;
            if (lane < MB) S.rec[lane] = r;
        }
        __syncthreads();
        const int nb = (n - m0 < MB) ? (n - m0) : MB;
        uint64_t bits = 0;
        // The last committed move: earlier commits are visible in LDS to every
        // wavefront, this one possibly not yet to the other wavefronts.
        int last_k = -1;
        double lx = 0.0, ly = 0.0, lz = 0.0;
        auto one_move = [&](const int i, const MoveRec &r) {
            const int k = __builtin_amdgcn_readfirstlane(r.k);
            const uint64_t cf =
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)r.conflict)) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(r.conflict >> 32)) << 32);
            const double th = r.th;
            // The mixed decision's thresholds, formed before the pair sum: read
            // after the W-wavefront barrier, th/beta would put an LDS load on
            // the chain of dependent moves.
            const double thb = MIXED ? r.thb : 0.0;
            const double thb_lo = thb * (1.0 - 0x1p-50), thb_hi = thb * (1.0 + 0x1p-50);
            double xo = r.xo, yo = r.yo, zo = r.zo, dfl = r.dfl, dfr = r.dfr;
            if ((cf & bits) != 0) {
                // An accepted move of this batch touched k-1, k or k+1: redo the
                // gather and the bond terms from the current replica (lanes 0..3
                // of each wavefront evaluate (k-1,k) new/old, (k,k+1) new/old).
                if constexpr (lds_consts) __asm__ volatile("" ::: "memory");
                const Consts &KF = lds_consts ? S.kc : K;
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
                const double fb = fene64(KF, sq3(xa - (nw ? xq : xo), ya - (nw ? yq : yo),
                                                 za - (nw ? zq : zo)));
                const double fv = has ? fb : 0.0;
                dfl = read_lane(fv, 0) - read_lane(fv, 1);
                dfr = read_lane(fv, 2) - read_lane(fv, 3);
            }
            const double xn = xo + r.dx, yn = yo + r.dy, zn = zo + r.dz;
            const double df = dfl + dfr;
            const int owner = k >> G::LOGB, slot = k & (B - 1);
            const bool mine = (tid == owner);

            auto leaf64 = [&](const Consts &KL, int b) {
                const double en = lj64(KL, sq3(rx[b] - xn, ry[b] - yn, rz[b] - zn));
                const double eo = lj64(KL, sq3(rx[b] - xo, ry[b] - yo, rz[b] - zo));
                const double tt = (mine && b == slot) ? 0.0 : en - eo;
                return Leaf64{tt, dabs(tt)};
            };
            bool acc = false;
            double de_used = 0.0, bm = 0.0;
            // The FP32 score's bound term is formed only for an accepted move
            // (in the commit), off the path of a rejected one.
            double bsum_acc = 0.0;
            bool bm_fp32 = false;
            bool exact = !MIXED;
            if constexpr (MIXED) {
                const LeafMx s = lane_tree<0, B>([&](int b) {
                    // The moved bead's own leaf and padding leaves are zeros (a
                    // padding bead's two terms are equal; its bound is dropped so
                    // that the bound does not depend on the padding).
                    const bool skip = (mine && b == slot) || tid * B + b >= n;
                    return mixed_leaf(K, rx[b], ry[b], rz[b], xn, yn, zn, xo, yo, zo, skip);
                });
                float smf = wave_tree(s.t);
                float bsf = wave_tree(s.b);
                if constexpr (W > 1) {
                    if (lane == 0) {
                        S.partf[i & 1][0][wv] = smf;
                        S.partf[i & 1][1][wv] = bsf;
                    }
                    __syncthreads();
                    smf = tree_wf<W>(S.partf[i & 1][0]);
                    bsf = tree_wf<W>(S.partf[i & 1][1]);
                }
                const double bsum = (double)bsf;
                const double dem = K.four_eps * (double)smf + df;  // bracket sum -> energy (Eq. 1)
                // Half-width of the band: the FP32 bound (the factor 1 + 2^-20
                // covering the FP32 sum of its terms) and 2^-50 |dem| for the FP64
                // roundings of dem, both widened by the guard scale.
                const double bt = __builtin_fma(rel_band, dabs(dem), kb_band * bsum);
                const double lo = dem - bt, hi = dem + bt;
                // Straight-line: every outcome is computed, one is kept.  With
                // thb = th / beta > 0: hi < thb (1 - 2^-50) makes every dE <= hi
                // accepted (dE <= 0, or beta dE < th even after rounding), and
                // lo >= thb (1 + 2^-50) makes every dE >= lo rejected; a NaN thb
                // (beta beyond 2^1000 th) decides nothing here.
                const bool sure_acc = hi < thb_lo;
                const bool sure_rej = lo >= thb_hi;
                const bool broken = df == __builtin_inf();  // rejected whatever the pair sum
                // A NaN or infinite dem (FP32 overflow) is never sure; a NaN or
                // infinite bt fails both comparisons.
                const bool sure = broken | (finite(dem) & (sure_acc | sure_rej));
                acc = !broken & sure_acc;
                de_used = dem;
                bsum_acc = bsum;
                bm_fp32 = true;
                // uniform: a scalar branch; with fp64_on_accept every accepted
                // move is re-scored as well, so that the running energy adds
                // FP64-order differences only
                exact = __builtin_amdgcn_ballot_w64(!sure | (fp64_on_accept & acc)) != 0;
                n_rescore += exact ? 1 : 0;
            }
            if (__builtin_expect(exact, 0)) {
                // The FP64 re-score stays behind this (uniform, rarely taken)
                // branch: the empty volatile asm keeps the compiler from
                // computing it speculatively on every move, which it does
                // otherwise at one wavefront per replica.
                __asm__ volatile("" ::: "memory");
                const Consts &KL = lds_consts ? S.kc : K;
                const Leaf64 s = lane_tree<0, B>([&](int b) { return leaf64(KL, b); });
                double sc = wave_tree(s.t);
                double ab = wave_tree(s.a);
                if constexpr (W > 1) {
                    double *pp = MIXED ? S.partx[0] : S.part[i & 1][0];
                    double *pa = MIXED ? S.partx[1] : S.part[i & 1][1];
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
                bm = bound64(log2c(n), ab, dfl, dfr, de);
                bm_fp32 = false;
            }
            if (__builtin_amdgcn_ballot_w64(acc) != 0) {
                // FP32 score: K.kbound sum (S^2 + S), the factor 1 + 2^-20 for
                // the FP32 sum of its terms, and the FP64 roundings of dE.
                if (bm_fp32)
                    bm = (K.kbound * bsum_acc) * (1.0 + 0x1p-20) +
                         0x1p-52 * (2.0 * (dabs(dfl) + dabs(dfr)) + dabs(de_used));
                if (mine) {
                    const int ak = G::pos(k);
                    X[ak] = xn;
                    Y[ak] = yn;
                    Z[ak] = zn;
                }
                // Only the wavefront holding bead k has a register to update.
                if (W == 1 || __builtin_amdgcn_readfirstlane(wv) == (owner >> 6)) {
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const bool me = mine && b == slot;
                        rx[b] = me ? xn : rx[b];
                        ry[b] = me ? yn : ry[b];
                        rz[b] = me ? zn : rz[b];
                    }
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
        };
        if constexpr (W == 1) {
            // One wavefront per replica: the next move's record is read while
            // the current move runs (its LDS latency overlaps the move), in two
            // alternating register sets, each reloaded only after its move is
            // done (no copies between them).  With more wavefronts the
            // registers are worth more than the latency.
            MoveRec ra = S.rec[0];
            for (int i = 0; i < nb; i += 2) {
                const MoveRec rb = S.rec[(i + 1 < MB) ? i + 1 : MB - 1];
                one_move(i, ra);
                if (i + 1 >= nb) break;
                ra = S.rec[(i + 2 < MB) ? i + 2 : MB - 1];
                one_move(i + 1, rb);
            }
        } else {
            for (int i = 0; i < nb; ++i) one_move(i, S.rec[i]);
        }
        logword |= bits << (m0 & 63);
        if (tid == 0 && (((m0 + MB) & 63) == 0 || m0 + MB >= n)) {
            if (logrow != nullptr) logrow[m0 >> 6] = logword;
            digest = mix64(digest ^ logword);
        }
        if (((m0 + MB) & 63) == 0) logword = 0;
    }
    if (tid == 0) T.dig[2 * g] = digest;
    __syncthreads();
}

// The per-sweep record of slot g (before any exchange): E, Ree^2 and Rg^2
// (Eq. 8) into the accumulators and the series; the running energy of
// conformation q.  The running energy is first replaced by the FP64-order
// energy when its bound has grown past resync_rel of max(1, |E|) (a start
// with near-overlapping beads, or many accepted moves), or after every sweep
// when the run recomputes the full energy each sweep, with all wavefronts;
// wavefront 0 does the rest.  E and Bd leave valid in every thread.
template <int B, int W>
__device__ __forceinline__ void sweep_record(const Tables &T, SweepLds<B, W> &S, int g, int q,
                                             int n, int64_t t64, double &E, double &Bd,
                                             int64_t n_acc, int64_t n_rescore) {
    using G = Geo<B, W>;
    const double *X = S.xyz, *Y = S.xyz + G::NP, *Z = S.xyz + 2 * G::NP;
    const Consts &K = T.k;
    const int tid = threadIdx.x;
    // E and Bd are the same in every thread: a block-uniform branch.
    const bool resync = T.full_energy || !(Bd <= K.resync_rel * (dabs(E) > 1.0 ? dabs(E) : 1.0));
    if (resync) {
        E = energy_block<B, W>(X, Y, Z, n, K, S.eblk);
        Bd = bound_energy(K, log2c(n), n, E, 0.0);
    }
    if (tid < 64) {
        double ree2, rg2;
        shape_wave<B, W>(X, Y, Z, n, ree2, rg2);
        if (tid == 0) {
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

template <int B, int W>
__device__ __forceinline__ void load_regs(const SweepLds<B, W> &S, double (&rx)[B], double (&ry)[B],
                                          double (&rz)[B]) {
    using G = Geo<B, W>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        rx[b] = S.xyz[b * G::NT + tid];
        ry[b] = S.xyz[G::NP + b * G::NT + tid];
        rz[b] = S.xyz[2 * G::NP + b * G::NT + tid];
    }
}

// One sweep of every slot in `list` (one block per slot), then its record.
// Classes of 1024 or more lanes' worth of beads (64 W B >= 1024) are built for
// three blocks per CU: more registers at two blocks per CU are slower
// (measured on N = 2000).
template <int B, int W, bool MIXED>
__global__ __launch_bounds__(64 * W, (B * W >= 16) ? 3 : 1) void k_sweep(const Tables T, const int32_t *__restrict__ list) {
    using G = Geo<B, W>;
    __shared__ SweepLds<B, W> S;
    const int g = list[blockIdx.x];
    const int c = T.slot_chain[g];
    const int n = T.chain_n[c];
    const int64_t t64 = T.te[0];
    const int q = T.perm[g];
    double *cq = T.coords + T.coord_off[q];
    copy_replica<B, W, G::NT>(S.xyz, cq);
    __syncthreads();
    double rx[B], ry[B], rz[B];
    load_regs<B, W>(S, rx, ry, rz);
    double E = T.e_run[q], Bd = T.b_run[q];
    int64_t n_acc = 0, n_rescore = 0;
    sweep_moves<B, W, MIXED>(T, S, rx, ry, rz, g, n, (uint32_t)t64, t64, E, Bd, n_acc, n_rescore);
    copy_replica<B, W, G::NT>(cq, S.xyz);
    sweep_record<B, W>(T, S, g, q, n, t64, E, Bd, n_acc, n_rescore);
}

// --------------------------------------------------- one lane per replica --
// The paper's first GPU design (Sec. 4.2: one thread runs the whole sweep of
// a replica), kept as a measured alternative mapping.  Here 64 replicas share
// a wavefront, one per lane, and each lane reads and writes its replica in
// HBM, bead by bead, in the (B, W) layout of its class.  Every sum is the
// pairwise tree of the wavefront kernels taken serially, so decisions,
// coordinates, energies and bounds equal theirs bit for bit.  FP64 order only.

// Pairwise tree over leaf(0) .. leaf(n - 1) padded with zeros to a power of
// two, in one thread: static trees over aligned chunks of 16 leaves chained
// by a binary counter (leaf(j) must be an exact zero for j >= n).  The pending
// subtrees left in the counter are the blocks of the binary expansion of the
// chunk count; adding them from the right gives the tree over the next power
// of two, whose remaining leaves are zeros.
template <int NP, class V, class F>
__device__ __forceinline__ V serial_tree(int n, const F &leaf) {
    constexpr int LV = ilog2(NP / 16);
    V stk[LV + 1];
    const int nc = (n + 15) >> 4;
    for (int c = 0; c < nc; ++c) {
        const V v = lane_tree<0, 16>([&](int b) { return leaf(c * 16 + b); });
        tree_push<LV>(stk, c, v);
    }
    V acc{};
    bool have = false;
#pragma unroll
    for (int l = 0; l <= LV; ++l) {
        if ((nc >> l) & 1) {
            acc = have ? stk[l] + acc : stk[l];
            have = true;
        }
    }
    return acc;
}

// Ree^2, Rg^2 (Eq. 8) and the FP64-order energy (Eq. 4) of a replica in the
// (B, W) layout, in one thread: the trees of shape_wave and energy_wave.
template <int B, int W>
__device__ void shape_serial(const double *X, const double *Y, const double *Z, int n,
                             double &ree2, double &rg2) {
    using G = Geo<B, W>;
    const int a0 = G::pos(0), a1 = G::pos(n - 1);
    ree2 = sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]);
    auto mean = [&](const double *C) {
        return serial_tree<G::NP, double>(n, [&](int j) { return (j < n) ? C[G::pos(j)] : 0.0; }) /
               (double)n;
    };
    const double mx = mean(X), my = mean(Y), mz = mean(Z);
    rg2 = serial_tree<G::NP, double>(n, [&](int j) {
              if (j >= n) return 0.0;
              const int a = G::pos(j);
              return sq3(X[a] - mx, Y[a] - my, Z[a] - mz);
          }) /
          (double)n;
}

template <int B, int W>
__device__ double energy_serial(const double *X, const double *Y, const double *Z, int n,
                                const Consts &k) {
    using G = Geo<B, W>;
    constexpr int LN = G::LOG_NP;
    double rows[LN + 1];
    for (int i = 0; i < n; ++i) {
        const int ai = G::pos(i);
        const double xi = X[ai], yi = Y[ai], zi = Z[ai];
        const double row = serial_tree<G::NP, double>(n, [&](int j) {
            if (!(j > i && j < n)) return 0.0;
            const int a = G::pos(j);
            return lj64(k, sq3(X[a] - xi, Y[a] - yi, Z[a] - zi));
        });
        tree_push<LN>(rows, i, row);
    }
    double e_lj = 0.0;
    bool have = false;
#pragma unroll
    for (int l = 0; l <= LN; ++l) {
        if ((n >> l) & 1) {
            e_lj = have ? rows[l] + e_lj : rows[l];
            have = true;
        }
    }
    const double e_fene = serial_tree<G::NP, double>(n, [&](int i) {
        if (i >= n - 1) return 0.0;
        const int a0 = G::pos(i), a1 = G::pos(i + 1);
        return fene64(k, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
    });
    return e_lj + e_fene;
}

// One sweep and its record for each slot in `list`, one lane per slot.
template <int B, int W>
__global__ __launch_bounds__(64) void k_sweep_lane(const Tables T, const int32_t *__restrict__ list,
                                                   int n_items) {
    using G = Geo<B, W>;
    const int idx = blockIdx.x * 64 + threadIdx.x;
    if (idx >= n_items) return;  // no barriers below
    const int g = list[idx];
    const int n = T.chain_n[T.slot_chain[g]];
    const int64_t t64 = T.te[0];
    const uint32_t t = (uint32_t)t64;
    const int q = T.perm[g];
    double *const X = T.coords + T.coord_off[q];
    double *const Y = X + G::NP, *const Z = X + 2 * G::NP;
    const Consts &K = T.k;
    const double beta = T.beta[g];
    const uint32_t gid = T.slot_gid[g];
    uint64_t *logrow = (T.accept_log != nullptr && t64 < T.log_cap)
                           ? T.accept_log + t64 * T.words_total + T.word_off[g]
                           : nullptr;
    uint64_t word = 0, digest = T.dig[2 * g];
    double E = T.e_run[q], Bd = T.b_run[q];
    int64_t n_acc = 0;
    const int lg = log2c(n);
    for (int m = 0; m < n; ++m) {
        // Draws of move m (Philox counters (m, t, g, 0) and (m, t, g, 1)).
        const U4 w = philox10(U4{(uint32_t)m, t, gid, 0u}, T.seed);
        const U4 v = philox10(U4{(uint32_t)m, t, gid, 1u}, T.seed);
        const int k = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)n) >> 32);
        const double th = -det_log(unit_open(v.x));
        const int ak = G::pos(k);
        const double xo = X[ak], yo = Y[ak], zo = Z[ak];
        const double xn = xo + (unit_open(w.y) - 0.5) * K.edge;
        const double yn = yo + (unit_open(w.z) - 0.5) * K.edge;
        const double zn = zo + (unit_open(w.w) - 0.5) * K.edge;
        // Bond differences (Eq. 3), a missing neighbour giving 0.
        double dfl = 0.0, dfr = 0.0;
        if (k > 0) {
            const int a = G::pos(k - 1);
            const double xl = X[a], yl = Y[a], zl = Z[a];
            dfl = fene64(K, sq3(xl - xn, yl - yn, zl - zn)) - fene64(K, sq3(xl - xo, yl - yo, zl - zo));
        }
        if (k + 1 < n) {
            const int a = G::pos(k + 1);
            const double xr = X[a], yr = Y[a], zr = Z[a];
            dfr = fene64(K, sq3(xr - xn, yr - yn, zr - zn)) - fene64(K, sq3(xr - xo, yr - yo, zr - zo));
        }
        // Pair sum (Eqs. 1, 4): the moved bead's own leaf and j >= n are zeros.
        const Leaf64 s = serial_tree<G::NP, Leaf64>(n, [&](int j) {
            if (j == k || j >= n) return Leaf64{0.0, 0.0};
            const int a = G::pos(j);
            const double en = lj64(K, sq3(X[a] - xn, Y[a] - yn, Z[a] - zn));
            const double eo = lj64(K, sq3(X[a] - xo, Y[a] - yo, Z[a] - zo));
            const double tt = en - eo;
            return Leaf64{tt, dabs(tt)};
        });
        const double de = s.t + (dfl + dfr);
        // Metropolis (Eq. 5) in the log domain.
        if ((de <= 0.0) || (beta * de < th)) {
            X[ak] = xn;
            Y[ak] = yn;
            Z[ak] = zn;
            E = E + de;
            Bd = Bd + bound64(lg, s.a, dfl, dfr, de) + 0x1p-52 * dabs(E);
            ++n_acc;
            word |= 1ull << (m & 63);
        }
        if ((m & 63) == 63 || m == n - 1) {
            if (logrow != nullptr) logrow[m >> 6] = word;
            digest = mix64(digest ^ word);
            word = 0;
        }
    }
    T.dig[2 * g] = digest;
    // Record, as sweep_record.
    double ree2, rg2;
    shape_serial<B, W>(X, Y, Z, n, ree2, rg2);
    bool resync = false;
    if (T.full_energy || !(Bd <= K.resync_rel * (dabs(E) > 1.0 ? dabs(E) : 1.0))) {
        E = energy_serial<B, W>(X, Y, Z, n, K);
        Bd = bound_energy(K, lg, n, E, 0.0);
        resync = true;
    }
    T.e_run[q] = E;
    T.b_run[q] = Bd;
    int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
    cnt[0] += n_acc;
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

// ----------------------------------------------------------------- energy --
// FP64-order energy of the conformations in `list` (by_slot: list holds slots
// and the conformation is perm[g]), one block of W wavefronts each; writes
// out_e / out_b indexed like list.
template <int B, int W>
__global__ __launch_bounds__(64 * W) void k_energy(const Tables T, const int32_t *__restrict__ list,
                                                   double *out_e, double *out_b, int by_slot) {
    using G = Geo<B, W>;
    __shared__ double XYZ[3 * G::NP];
    __shared__ double sh[B * W + 1];
    double *const X = XYZ, *const Y = XYZ + G::NP, *const Z = XYZ + 2 * G::NP;
    const int id = list[blockIdx.x];
    const int q = by_slot ? T.perm[id] : id;
    const int c = T.slot_chain[q];  // conformation q started in slot q: same chain
    const int n = T.chain_n[c];
    copy_replica<B, W, G::NT>(XYZ, T.coords + T.coord_off[q]);
    __syncthreads();
    const double e = energy_block<B, W>(X, Y, Z, n, T.k, sh);
    if (threadIdx.x == 0) {
        out_e[id] = e;
        if (out_b != nullptr) out_b[id] = bound_energy(T.k, log2c(n), n, e, 0.0);
    }
}

// Energy E(C) of Eq. (4) the way of the paper's energy routine (Sec. 3.4):
// the coordinates in LDS, one pair per thread per round.  With N virtual
// threads v (thread tid of the block takes v = tid B + b, b < B), v first
// takes its bond (v, v+1), then in round i = 0 .. floor(N/2) - 1 the pair
// (i, v) when v > i, else (N-2-i, N-1-i+v); rows i and N-2-i together hold
// N pairs.  For even N the last round has i = N-2-i, where the second form
// would repeat the first one's pairs: there only v > i take a pair (the
// printed enumeration drops that whole round instead, and with it row i).
// Each v sums its terms in order; the N sums meet in the pairwise tree over v.
// Not the FP64 order: out_b[g] receives a rigorous bound on |E - exact sum of
// the same FP64 terms|, (m + log2 NP + 3) 2^-52 sum |terms| with m = floor(N/2)
// + 1 terms per v (recursive sums, then the tree, with a factor-two margin);
// out_e, out_b are indexed by slot.
template <int B, int W>
__global__ __launch_bounds__(64 * W) void k_energy_pairs(const Tables T, const int32_t *__restrict__ list,
                                                        double *out_e, double *out_b) {
    using G = Geo<B, W>;
    __shared__ double XYZ[3 * G::NP];
    __shared__ double part[2][W];
    double *const X = XYZ, *const Y = XYZ + G::NP, *const Z = XYZ + 2 * G::NP;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = list[blockIdx.x];
    const int q = T.perm[g];
    const int n = T.chain_n[T.slot_chain[g]];
    const Consts &K = T.k;
    copy_replica<B, W, G::NT>(XYZ, T.coords + T.coord_off[q]);
    __syncthreads();
    double acc[B], ab[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int v = tid * B + b;
        acc[b] = 0.0;
        if (v < n - 1) {
            const int a0 = G::pos(v), a1 = G::pos(v + 1);
            acc[b] = fene64(K, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
        }
        ab[b] = dabs(acc[b]);
    }
    const int rounds = n / 2;
    for (int i = 0; i < rounds; ++i) {
        const bool last_even = (n - 2 - i == i);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int v = tid * B + b;
            const bool upper = v > i;
            const int i1 = upper ? i : n - 2 - i;
            const int i2 = upper ? v : n - 1 - i + v;
            if (v < n && (upper || !last_even)) {
                const int a1 = G::pos(i1), a2 = G::pos(i2);
                const double e = lj64(K, sq3(X[a2] - X[a1], Y[a2] - Y[a1], Z[a2] - Z[a1]));
                acc[b] = acc[b] + e;
                ab[b] = ab[b] + dabs(e);
            }
        }
    }
    const Leaf64 s = lane_tree<0, B>([&](int b) { return Leaf64{acc[b], ab[b]}; });
    double e = wave_tree(s.t), a = wave_tree(s.a);
    if constexpr (W > 1) {
        if (lane == 0) {
            part[0][wv] = e;
            part[1][wv] = a;
        }
        __syncthreads();
        e = tree_w<W>(part[0]);
        a = tree_w<W>(part[1]);
    }
    if (tid == 0) {
        out_e[g] = e;
        out_b[g] = 0x1p-52 * (double)(rounds + 1 + G::LOG_NP + 3) * a;
    }
}

// --------------------------------------------------------------- exchange --
// Decision of one exchange attempt (Sec. 3.3, Eq. 6) between slots (g, g+1)
// of chain c at exchange step e, holding conformations q1, q2 with running
// energies e1, e2 and bounds b1, b2.  The decision is taken from the running
// energies when their bounds settle it; otherwise canon(0), canon(1) give the
// FP64-order energies of q1 and q2, the decision is exact, and e1, b1, e2, b2
// are replaced by those energies and their bounds (band = true).  Block-
// uniform; called by every thread of the block (canon synchronises it).
template <int B, int W, class Canon>
__device__ __forceinline__ bool exch_decide(const Tables &T, int c, int i, int64_t e, int n, int g,
                                            double &e1, double &bb1, double &e2, double &bb2,
                                            bool &band, const Canon &canon) {
    using G = Geo<B, W>;
    const double db = T.beta[g] - T.beta[g + 1];
    const U4 w = philox10(U4{(uint32_t)i, (uint32_t)e, T.chain_sid[c], 2u}, T.seed);
    const double pl = det_log(unit_open(w.x));
    const double dd = e1 - e2;
    const double tot = ((bb1 + bound_energy(T.k, log2c(n), n, e1, bb1) + bb2 +
                         bound_energy(T.k, log2c(n), n, e2, bb2)) * (1.0 + 0x1p-20) +
                        0x1p-50 * dabs(dd)) * T.guard_scale;
    const double d1 = db * (dd - tot), d2 = db * (dd + tot);
    const double dlo = (d1 < d2) ? d1 : d2, dhi = (d1 < d2) ? d2 : d1;
    const bool sure_acc = (dlo >= 0.0) || (pl < dlo);
    const bool sure_rej = (dhi < 0.0) && !(pl < dhi);
    band = false;
    if (finite(tot) && finite(dd) && finite(db) && (sure_acc || sure_rej)) return sure_acc;
    band = true;
    const double c1 = canon(0);
    const double c2 = canon(1);
    const double d = db * (c1 - c2);
    e1 = c1;
    bb1 = bound_energy(T.k, log2c(n), n, c1, 0.0);
    e2 = c2;
    bb2 = bound_energy(T.k, log2c(n), n, c2, 0.0);
    return (d >= 0.0) || (pl < d);
}

// Book-keeping of a decided attempt (thread 0): counters, log, permutation.
__device__ __forceinline__ void exch_commit(const Tables &T, int g, int64_t e, int q1, int q2, bool acc,
                                            bool band) {
    int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
    cnt[1] += 1;
    if (band) cnt[4] += 1;
    if (acc) {
        cnt[2] += 1;
        T.perm[g] = q2;
        T.perm[g + 1] = q1;
        T.slot_of[q1] = g + 1;
        T.slot_of[q2] = g;
    }
    if (T.exch_log != nullptr && e < T.log_cap) T.exch_log[e * T.total_slots + g] = acc ? 1 : 0;
    T.dig[2 * g + 1] = mix64(T.dig[2 * g + 1] ^ (((uint64_t)e << 1) | (acc ? 1u : 0u)));
}

// The words exch_commit updates, read ahead of the decision by the persistent
// kernel's deciding block (their last writer handed the slot on through the
// handshakes this block has already acquired), so that the commit stores
// without waiting for loads.
struct ExchBook {
    int64_t c1, c2, c4;
    uint64_t dig;
};

__device__ __forceinline__ ExchBook exch_book(const Tables &T, int g) {
    const int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
    return ExchBook{cnt[1], cnt[2], cnt[4], T.dig[2 * g + 1]};
}

__device__ __forceinline__ void exch_commit_from(const Tables &T, const ExchBook &bk, int g, int64_t e, int q1,
                                                 int q2, bool acc, bool band) {
    int64_t *cnt = T.counts + (int64_t)g * PT_NCOUNTS;
    cnt[1] = bk.c1 + 1;
    if (band) cnt[4] = bk.c4 + 1;
    if (acc) {
        cnt[2] = bk.c2 + 1;
        T.perm[g] = q2;
        T.perm[g + 1] = q1;
        T.slot_of[q1] = g + 1;
        T.slot_of[q2] = g;
    }
    if (T.exch_log != nullptr && e < T.log_cap) T.exch_log[e * T.total_slots + g] = acc ? 1 : 0;
    T.dig[2 * g + 1] = mix64(bk.dig ^ (((uint64_t)e << 1) | (acc ? 1u : 0u)));
}

// One exchange step for the chains in `list`: block p of a chain (W
// wavefronts) handles the pair (i, i+1), i = (e mod 2) + 2p.
template <int B, int W>
__global__ __launch_bounds__(64 * W) void k_exchange(const Tables T, const int32_t *__restrict__ list,
                                                     int max_pairs, int force) {
    using G = Geo<B, W>;
    __shared__ double XYZ[3 * G::NP];
    __shared__ double sh[B * W + 1];
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
    double e1 = T.e_run[q1], e2 = T.e_run[q2];
    double bb1 = T.b_run[q1], bb2 = T.b_run[q2];
    bool band = false;
    // Captures by value: a reference to the kernel argument T would force a
    // copy of it into scratch memory.
    const double *src1 = T.coords + T.coord_off[q1], *src2 = T.coords + T.coord_off[q2];
    const Consts K = T.k;
    double *const lds = XYZ;
    double *const shp = sh;
    auto canon = [lds, shp, src1, src2, n, K](int which) {
        __syncthreads();
        copy_replica<B, W, G::NT>(lds, which == 0 ? src1 : src2);
        __syncthreads();
        return energy_block<B, W>(lds, lds + G::NP, lds + 2 * G::NP, n, K, shp);
    };
    const bool acc = exch_decide<B, W>(T, c, i, e, n, g, e1, bb1, e2, bb2, band, canon);
    if (threadIdx.x == 0) {
        if (band) {
            T.e_run[q1] = e1;
            T.b_run[q1] = bb1;
            T.e_run[q2] = e2;
            T.b_run[q2] = bb2;
        }
        exch_commit(T, g, e, q1, q2, acc, band);
    }
}

// ---------------------------------------------------------- persistent run --
// Spin (one thread) until *p >= v; false after a timeout or when another block
// reported one, which also ends the waiting of every other block.  The polls
// are relaxed (an acquiring load would invalidate the caches on every poll);
// the acquire fence after the successful one pairs with the writer's release.
__device__ __forceinline__ bool wait_ge(const int64_t *p, int64_t v, int32_t *err, uint32_t limit) {
    for (uint32_t it = 0; it < limit; ++it) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= v) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// n_sweeps sweeps and exchange steps of conformation q (one block of W
// wavefronts), starting at sweep t0 and exchange step e0.  The block keeps
// the replica in LDS and registers for the whole run and follows it from
// slot to slot.  Exchange attempts synchronise pairs only: after a sweep that
// is followed by an exchange step, the holder of slot g publishes its running
// energy, coordinates and conformation id and sets done[g] = t + 1; the
// holder of the lower slot of an attempted pair waits for its partner's flag,
// decides exactly as k_exchange does, writes the new slot assignment and sets
// dec[g+1] = t + 1, which the partner waits for.  Inside the band the
// partner's FP64-order energy is computed from a copy of its replica in the
// block's LDS, which is then refilled from the block's own published copy.
template <int B, int W, bool MIXED>
__device__ __forceinline__ void run_body(const Tables &T, SweepLds<B, W> &S, int32_t &s_slot, int32_t &s_ok,
                                         const int q, const int64_t n_sweeps, const int64_t t0,
                                         const int64_t e0) {
    using G = Geo<B, W>;
    const int tid = threadIdx.x;
    const int c = T.slot_chain[q];
    const int n = T.chain_n[c];
    const int R = T.chain_slots[c];
    const int s0 = T.chain_slot0[c];
    double *cq = T.coords + T.coord_off[q];
    copy_replica<B, W, G::NT>(S.xyz, cq);
    __syncthreads();
    double rx[B], ry[B], rz[B];
    load_regs<B, W>(S, rx, ry, rz);
    double E = T.e_run[q], Bd = T.b_run[q];
    int g = T.slot_of[q];
    int64_t e = e0;
    for (int64_t s = 0; s < n_sweeps; ++s) {
        const int64_t t64 = t0 + s;
        int64_t n_acc = 0, n_rescore = 0;
        // (The four-wavefront persistent kernel keeps the one-lane prologue: with
        // the split one in its 8-bead body the compiler allocated the 2-bead
        // body's registers worse, N = 500 x 128 0.425 -> 0.439 ms per sweep.)
        sweep_moves<B, W, MIXED, (W < 4)>(T, S, rx, ry, rz, g, n, (uint32_t)t64, t64, E, Bd, n_acc, n_rescore);
        sweep_record<B, W>(T, S, g, q, n, t64, E, Bd, n_acc, n_rescore);
        if (!(T.exchange_every > 0 && (t64 + 1) % T.exchange_every == 0)) continue;
        // Publish this conformation at slot g: the block's writes, then (after
        // the barrier, which completes them) thread 0's releasing flag store.
        copy_replica<B, W, G::NT>(cq, S.xyz);
        if (tid == 0) T.perm[g] = q;
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&T.done[g], t64 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int i = g - s0;
        const int par = (int)(e & 1);
        const bool lower = i >= par && ((i - par) & 1) == 0 && i + 1 < R;
        const bool upper = i >= 1 + par && ((i - 1 - par) & 1) == 0;
        if (lower) {
            // Every wavefront takes part: the FP64-order energies of a decision
            // inside the band use the whole block.
            // wait_ge's acquire (thread 0), then the barrier, orders the
            // block's reads of the partner's data after the partner's flag.
            ExchBook bk{};
            if (tid == 0) {
                bk = exch_book(T, g);
                s_ok = wait_ge(&T.done[g + 1], t64 + 1, T.err, T.spin_limit) ? 1 : 0;
            }
            __syncthreads();
            if (s_ok) {
                const int q2 = T.perm[g + 1];
                double e1 = E, bb1 = Bd;
                double e2 = T.e_run[q2], bb2 = T.b_run[q2];
                bool band = false;
                const double *c2 = T.coords + T.coord_off[q2];
                double *const lds = S.xyz;
                double *const shp = S.eblk;
                const Consts K = T.k;
                auto canon = [lds, shp, c2, cq, n, K](int which) {
                    if (which == 1) {
                        __syncthreads();
                        copy_replica<B, W, G::NT>(lds, c2);
                        __syncthreads();
                    }
                    const double v = energy_block<B, W>(lds, lds + G::NP, lds + 2 * G::NP, n, K, shp);
                    if (which == 1) {
                        copy_replica<B, W, G::NT>(lds, cq);  // after energy_block's last barrier
                        __syncthreads();
                    }
                    return v;
                };
                const bool acc = exch_decide<B, W>(T, c, i, e, n, g, e1, bb1, e2, bb2, band, canon);
                if (tid == 0) {
                    if (band) {
                        T.e_run[q] = e1;
                        T.b_run[q] = bb1;
                        T.e_run[q2] = e2;
                        T.b_run[q2] = bb2;
                        S.bcast[0] = e1;
                        S.bcast[1] = bb1;
                    } else {
                        S.bcast[0] = E;
                        S.bcast[1] = Bd;
                    }
                    exch_commit_from(T, bk, g, e, q, q2, acc, band);
                    __hip_atomic_store(&T.dec[g + 1], t64 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    s_slot = acc ? g + 1 : g;
                }
            } else if (tid == 0) {
                s_slot = g;
            }
        } else if (tid < 64) {
            int32_t ok = 1, slot = g;
            if (upper) {
                if (tid == 0) ok = wait_ge(&T.dec[g], t64 + 1, T.err, T.spin_limit) ? 1 : 0;
                ok = __builtin_amdgcn_readfirstlane(ok);
                if (ok && tid == 0) {  // after wait_ge's acquire
                    S.bcast[0] = T.e_run[q];
                    S.bcast[1] = T.b_run[q];
                    slot = T.slot_of[q];
                }
            } else if (tid == 0) {
                S.bcast[0] = E;
                S.bcast[1] = Bd;
            }
            if (tid == 0) {
                s_slot = slot;
                s_ok = ok;
            }
        }
        __syncthreads();
        if (!s_ok) return;  // a partner never arrived: the error flag is set
        g = s_slot;
        E = S.bcast[0];
        Bd = S.bcast[1];
        e += 1;
        __syncthreads();
        // The LDS copy is current: reloading keeps the register copy dead
        // across the exchange step, which has register needs of its own.
        load_regs<B, W>(S, rx, ry, rz);
    }
    copy_replica<B, W, G::NT>(cq, S.xyz);
}

// Dynamic LDS of the kernels whose blocks take different bead counts per
// lane: each block views it as the SweepLds of its own B.
extern __shared__ double pt_dyn_lds[];

// Persistent run: n_sweeps sweeps and exchange steps of every conformation
// in `list` (one block each, longest chains first), all blocks resident at
// once (the host checks the occupancy before launching; an ordinary launch,
// so it can be captured in a graph).  Chains of any bead count per lane B
// share the launch: each block takes its chain's B from chain_bpl.  The run
// starts at the device's run counters, which only a later kernel advances.
// MINW is the minimum number of wavefronts per SIMD the registers must allow:
// 1 for batches that fit anyway (no spills), more for dense batches.  MAXB is
// the largest bead count per lane built in: 4 leaves out the 8-bead body,
// whose registers make the dense build spill in every body (the 48 uneven
// chains at two wavefronts: 0.609 -> 0.606 ms per sweep).
template <int W, bool MIXED, int MINW, int MAXB = 8>
__global__ __launch_bounds__(64 * W, MINW) void k_run(const Tables T, const int32_t *__restrict__ list,
                                                      int64_t n_sweeps) {
    __shared__ int32_t s_slot, s_ok;
    const int q = list[blockIdx.x];
    const int bpl = T.chain_bpl[T.slot_chain[q]];
    const int64_t t0 = T.te[0], e0 = T.te[1];
    switch (bpl) {
        case 1: run_body<1, W, MIXED>(T, *reinterpret_cast<SweepLds<1, W> *>(pt_dyn_lds), s_slot, s_ok, q, n_sweeps, t0, e0); break;
        case 2: run_body<2, W, MIXED>(T, *reinterpret_cast<SweepLds<2, W> *>(pt_dyn_lds), s_slot, s_ok, q, n_sweeps, t0, e0); break;
        case 4: run_body<4, W, MIXED>(T, *reinterpret_cast<SweepLds<4, W> *>(pt_dyn_lds), s_slot, s_ok, q, n_sweeps, t0, e0); break;
        case 8:
            if constexpr (MAXB >= 8)
                run_body<8, W, MIXED>(T, *reinterpret_cast<SweepLds<8, W> *>(pt_dyn_lds), s_slot, s_ok, q, n_sweeps, t0, e0);
            break;
        default: break;  // not a built class (the host never lists one)
    }
}

// ------------------------------------------------------------- task flow --
// n_sweeps sweeps and exchange steps of the S slots in `list` when they do not
// all fit on the device at once: the resident blocks take tasks k = 0, 1, ...
// from a counter, task k being sweep t0 + k / S of slot list[k mod S].  A
// task first waits until the slot's conformation for that sweep is settled
// (ready[g] >= t: the exchange step after the previous sweep decided, or none
// due), sweeps it from HBM like k_sweep, records it and writes it back.  When
// an exchange step follows, the two tasks of an attempted pair each publish
// and count their arrival on the lower slot (arr, two per attempt); the one
// that arrives second decides exactly as k_exchange does, from the published
// running energies (FP64-order energies from HBM inside the band), and marks
// both slots ready.  A task waits only for tasks handed out before it, so the
// blocks always progress; every wait is bounded as in k_run.
template <int B, int W, bool MIXED>
__global__ __launch_bounds__(64 * W, (B * W >= 16) ? 3 : 1) void k_flow(const Tables T,
                                                                       const int32_t *__restrict__ list,
                                                                       int n_items, int64_t n_sweeps) {
    using G = Geo<B, W>;
    __shared__ SweepLds<B, W> S;
    __shared__ int64_t s_task;
    __shared__ int32_t s_flag;
    const int tid = threadIdx.x;
    const int64_t t0 = T.te[0], e0 = T.te[1];
    const int64_t total = n_sweeps * (int64_t)n_items;
    const int every = T.exchange_every;
    for (;;) {
        if (tid == 0) {
            const bool failed = __hip_atomic_load(T.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            s_task = failed ? total : __hip_atomic_fetch_add(T.flow_task, (int64_t)1, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int64_t k = s_task;
        if (k >= total) return;
        const int64_t s = k / n_items;
        const int g = list[k - s * n_items];
        const int64_t t64 = t0 + s;
        const int c = T.slot_chain[g];
        const int n = T.chain_n[c];
        // The slot's conformation for sweep t64.
        if (s > 0) {
            // wait_ge's acquire (thread 0), then the barrier, orders the
            // block's reads of the conformation after the flag.
            if (tid == 0) s_flag = wait_ge(&T.flow_ready[g], t64, T.err, T.spin_limit) ? 1 : 0;
            __syncthreads();
            if (!s_flag) return;  // a timeout: the error flag is set
        }
        const int q = T.perm[g];
        double *cq = T.coords + T.coord_off[q];
        copy_replica<B, W, G::NT>(S.xyz, cq);
        __syncthreads();
        double rx[B], ry[B], rz[B];
        load_regs<B, W>(S, rx, ry, rz);
        double E = T.e_run[q], Bd = T.b_run[q];
        int64_t n_acc = 0, n_rescore = 0;
        sweep_moves<B, W, MIXED>(T, S, rx, ry, rz, g, n, (uint32_t)t64, t64, E, Bd, n_acc, n_rescore);
        copy_replica<B, W, G::NT>(cq, S.xyz);
        sweep_record<B, W>(T, S, g, q, n, t64, E, Bd, n_acc, n_rescore);
        // The exchange step after this sweep, if one is due: its index e counts
        // the due sweeps before t64 since t0.
        const bool due = every > 0 && (t64 + 1) % every == 0;
        const int64_t e = due ? e0 + (t64 / every - t0 / every) : 0;
        const int R = T.chain_slots[c];
        const int i = g - T.chain_slot0[c];
        const int par = (int)(e & 1);
        const bool lower = due && i >= par && ((i - par) & 1) == 0 && i + 1 < R;
        const bool upper = due && i >= 1 + par && ((i - 1 - par) & 1) == 0;
        // Coordinates, running energy and record are published by the barrier
        // (which completes the block's writes) and thread 0's releasing store
        // or arrival.
        __syncthreads();
        if (!lower && !upper) {
            if (tid == 0) __hip_atomic_store(&T.flow_ready[g], t64 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const int glow = lower ? g : g - 1;
        if (tid == 0) {
            const int64_t old = __hip_atomic_fetch_add(&T.flow_arr[glow], (int64_t)1, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            s_flag = (int32_t)(old & 1);  // 1: the partner has arrived, this task decides
        }
        __syncthreads();
        if (!s_flag) continue;  // else thread 0's arrival acquired the partner's publication
        const int q1 = T.perm[glow], q2 = T.perm[glow + 1];
        double e1 = T.e_run[q1], bb1 = T.b_run[q1];
        double e2 = T.e_run[q2], bb2 = T.b_run[q2];
        bool band = false;
        const double *c1 = T.coords + T.coord_off[q1], *c2 = T.coords + T.coord_off[q2];
        double *const lds = S.xyz;
        double *const shp = S.eblk;
        const Consts K = T.k;
        auto canon = [lds, shp, c1, c2, n, K](int which) {
            __syncthreads();
            copy_replica<B, W, G::NT>(lds, which == 0 ? c1 : c2);
            __syncthreads();
            return energy_block<B, W>(lds, lds + G::NP, lds + 2 * G::NP, n, K, shp);
        };
        const bool acc = exch_decide<B, W>(T, c, glow - T.chain_slot0[c], e, n, glow, e1, bb1, e2, bb2, band, canon);
        if (tid == 0) {
            if (band) {
                T.e_run[q1] = e1;
                T.b_run[q1] = bb1;
                T.e_run[q2] = e2;
                T.b_run[q2] = bb2;
            }
            exch_commit(T, glow, e, q1, q2, acc, band);
            __hip_atomic_store(&T.flow_ready[glow], t64 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&T.flow_ready[glow + 1], t64 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// LDS of a persistent block of bead count per lane bpl (dynamic: the blocks
// of one launch view it as the SweepLds of their own B).
template <int W>
size_t run_lds(int bpl) {
    switch (bpl) {
        case 1: return sizeof(SweepLds<1, W>);
        case 2: return sizeof(SweepLds<2, W>);
        case 4: return sizeof(SweepLds<4, W>);
        default: return sizeof(SweepLds<8, W>);
    }
}

}  // namespace

// The (beads per lane, wavefronts per replica) classes the library builds.
#define PT_DISPATCH(bpl, wpr, CALL)           \
    switch ((bpl) * 16 + (wpr)) {             \
        case 1 * 16 + 1: return CALL(1, 1);   \
        case 2 * 16 + 1: return CALL(2, 1);   \
        case 4 * 16 + 1: return CALL(4, 1);   \
        case 8 * 16 + 1: return CALL(8, 1);   \
        case 1 * 16 + 2: return CALL(1, 2);   \
        case 2 * 16 + 2: return CALL(2, 2);   \
        case 4 * 16 + 2: return CALL(4, 2);   \
        case 8 * 16 + 2: return CALL(8, 2);   \
        case 1 * 16 + 4: return CALL(1, 4);   \
        case 2 * 16 + 4: return CALL(2, 4);   \
        case 4 * 16 + 4: return CALL(4, 4);   \
        case 8 * 16 + 4: return CALL(8, 4);   \
        default: return hipErrorInvalidValue; \
    }

}  // namespace pt
