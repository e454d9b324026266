// pt_pack.hpp -- several replicas per wavefront: the per-sweep kernel for
// short chains (N <= 64 BU, BU = 1 or 2), G = 2 or 4 replicas of one chain
// sharing a wavefront, L = 64 / G lanes each (the occupancy question of the
// paper's Sec. 4.2: a chain of 13 beads fills 13 of 64 lanes).
//
// A replica keeps the HBM layout of its (BU, 1) class, so every other kernel
// (energies, exchange, observables) runs on it unchanged; in the sweep, lane
// l of the replica's lane group holds beads l B .. l B + B - 1, B = BU G, in
// registers (L B = 64 BU, the padded bead range of the class), and the group's
// part of the LDS mirrors the replica in the class layout.  The pair sum of a
// move is the in-lane pairwise tree over the B beads and the butterfly over the
// L lanes of the group (the first log2 L levels of the wavefront butterfly):
// the pairwise tree over the padded bead range, as in every other mapping, so
// decisions, coordinates, energies and bounds equal those of k_sweep<BU, 1>
// bit for bit.  The FP64-order energy, Ree^2 and Rg^2 likewise take the trees
// of energy_wave and shape_wave, their 64 rows or beads per lane group split
// into G consecutive ones per lane.
//
// Each group draws, scores and commits its own moves; the groups of a
// wavefront run their move loops in lockstep (same chain, same N), their
// decisions and commits as lane-group values.  The FP64 re-score of the mixed
// path runs for the wavefront when any group needs it and is kept by the groups
// that do.
#pragma once

#include "pt_kernels.hpp"

namespace pt {

namespace {

// Pairwise tree over the L-lane groups of a wavefront (L = 16 or 32), the same
// in every lane of a group.
template <int L>
__device__ __forceinline__ double group_tree(double v) {
    static_assert(L == 16 || L == 32, "lane groups of 16 or 32");
    v = v + dpp64<dpp_qp1>(v);
    v = v + dpp64<dpp_qp2>(v);
    v = v + dpp64<dpp_hmir>(v);
    v = v + dpp64<dpp_mir>(v);
    if constexpr (L == 32) {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
        v = join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
    }
    return v;
}

template <int L>
__device__ __forceinline__ float group_tree(float v) {
    static_assert(L == 16 || L == 32, "lane groups of 16 or 32");
    v = v + __uint_as_float(dpp_qp1(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_qp2(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_hmir(__float_as_uint(v)));
    v = v + __uint_as_float(dpp_mir(__float_as_uint(v)));
    if constexpr (L == 32) {
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
    return v;
}

template <int BU, int G>
struct PackLds {
    static constexpr int L = 64 / G;   // lanes per replica
    static constexpr int NP = 64 * BU; // padded bead range of the class
    double xyz[G][3 * NP];             // the G replicas, class layout
    MoveRec rec[G][L];                 // the batch's move records, one batch of L moves per replica
    int32_t ks[64];                    // the batch's moved beads, by lane
    double fv[64];                     // bond terms of a conflicting move, by lane
};

// FP64-order energy E(C) of Eq. (4) of the group's replica: energy_wave's
// trees, each lane computing G consecutive rows of every 64-row block.
template <int BU, int G>
__device__ __forceinline__ double pack_energy(const double *X, const double *Y, const double *Z, int n,
                                              const Consts &k, int ll) {
    using GE = Geo<BU, 1>;
    constexpr int L = 64 / G, B = BU * G;
    constexpr int CW = 16, NC = GE::NP / CW, LR = ilog2(NC), LC = ilog2(BU);
    double blk[LC + 1];
#pragma unroll
    for (int l = 0; l <= LC; ++l) blk[l] = 0.0;
    for (int r = 0; r < BU; ++r) {
        double v = 0.0;
        if (r * 64 < n) {
            const double rows = lane_tree<0, G>([&](int rho) {
                const int i = r * 64 + ll * G + rho;
                const int ai = GE::pos(i);
                const double xi = X[ai], yi = Y[ai], zi = Z[ai];
                double row[LR + 1];
#pragma unroll
                for (int l = 0; l <= LR; ++l) row[l] = 0.0;
                for (int c = 0; c < NC; ++c) {
                    double cv = 0.0;
                    if (c * CW + CW > r * 64 && c * CW < n)
                        cv = row_chunk<BU, 1, 0, CW>(X, Y, Z, k, i, n, c * CW, xi, yi, zi);
                    tree_push<LR>(row, c, cv);
                }
                return row[LR];
            });
            v = group_tree<L>(rows);
        }
        tree_push<LC>(blk, r, v);
    }
    const double fb = lane_tree<0, B>([&](int b) {
        const int i = ll * B + b;
        const int i0 = (i < n - 1) ? i : 0;
        const int a0 = GE::pos(i0), a1 = GE::pos(i0 + 1);
        const double v = fene64(k, sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]));
        return (i < n - 1) ? v : 0.0;
    });
    return blk[LC] + group_tree<L>(fb);
}

// Ree^2 and Rg^2 (Eq. 8) of the group's replica: shape_wave's trees.
template <int BU, int G>
__device__ __forceinline__ void pack_shape(const double *X, const double *Y, const double *Z, int n, int ll,
                                           double &ree2, double &rg2) {
    using GE = Geo<BU, 1>;
    constexpr int L = 64 / G, B = BU * G;
    const int a0 = GE::pos(0), a1 = GE::pos(n - 1);
    ree2 = sq3(X[a1] - X[a0], Y[a1] - Y[a0], Z[a1] - Z[a0]);
    auto mean = [&](const double *C) {
        const double s = lane_tree<0, B>([&](int b) {
            const int j = ll * B + b;
            return (j < n) ? C[GE::pos(j)] : 0.0;
        });
        return group_tree<L>(s) / (double)n;
    };
    const double mx = mean(X), my = mean(Y), mz = mean(Z);
    const double s = lane_tree<0, B>([&](int b) {
        const int j = ll * B + b;
        const int a = GE::pos(j);
        const double v = sq3(X[a] - mx, Y[a] - my, Z[a] - mz);
        return (j < n) ? v : 0.0;
    });
    rg2 = group_tree<L>(s) / (double)n;
}

// One sweep and its record for G slots of one chain per wavefront: block b
// takes list[G b .. G b + G - 1] (-1: no replica in that group).
template <int BU, int G, bool MIXED>
__global__ __launch_bounds__(64) void k_sweep_pack(const Tables T, const int32_t *__restrict__ list) {
    using GE = Geo<BU, 1>;
    using P = PackLds<BU, G>;
    constexpr int L = P::L, B = BU * G, NP = P::NP;
    __shared__ P S;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, ll = lane % L, g0 = grp * L;
    const int g = list[blockIdx.x * G + grp];
    if (g < 0) return;
    const int c = T.slot_chain[g];
    const int n = T.chain_n[c];
    const int64_t t64 = T.te[0];
    const uint32_t t = (uint32_t)t64;
    const int q = T.perm[g];
    const Consts &K = T.k;
    double *const X = S.xyz[grp], *const Y = X + NP, *const Z = X + 2 * NP;
    double *cq = T.coords + T.coord_off[q];
    for (int i = ll; i < 3 * NP; i += L) X[i] = cq[i];
    wave_sync();
    double rx[B], ry[B], rz[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int a = GE::pos(ll * B + b);
        rx[b] = X[a];
        ry[b] = Y[a];
        rz[b] = Z[a];
    }
    double E = T.e_run[q], Bd = T.b_run[q];
    int64_t n_acc = 0, n_rescore = 0;
    const double beta = T.beta[g];
    const uint32_t gid = T.slot_gid[g];
    const bool fp64_on_accept = MIXED && T.fp64_on_accept != 0;
    const double kb_band = K.kbound * (1.0 + 0x1p-20) * T.guard_scale;
    const double rel_band = 0x1p-50 * T.guard_scale;
    uint64_t *logrow = (T.accept_log != nullptr && t64 < T.log_cap)
                           ? T.accept_log + t64 * T.words_total + T.word_off[g]
                           : nullptr;
    uint64_t logword = 0;
    uint64_t digest = (ll == 0) ? T.dig[2 * g] : 0;

    for (int m0 = 0; m0 < n; m0 += L) {
        // ---- prologue: lane ll draws move m0 + ll of its replica (the
        // arithmetic of sweep_moves' prologue)
        {
            const uint32_t m = (uint32_t)(m0 + ll);
            const U4 w = philox10(U4{m, t, gid, 0u}, T.seed);
            const U4 v = philox10(U4{m, t, gid, 1u}, T.seed);
            MoveRec r;
            r.k = (int)(((uint64_t)w.x * (uint64_t)(uint32_t)n) >> 32);
            r.dx = (unit_open(w.y) - 0.5) * K.edge;
            r.dy = (unit_open(w.z) - 0.5) * K.edge;
            r.dz = (unit_open(w.w) - 0.5) * K.edge;
            r.th = -det_log(unit_open(v.x));
            const double thb = r.th / beta;
            r.thb = (thb >= 0x1p-1000) ? thb : __builtin_nan("");
            const int k = r.k;
            const int ak = GE::pos(k);
            r.xo = X[ak];
            r.yo = Y[ak];
            r.zo = Z[ak];
            const double xn = r.xo + r.dx, yn = r.yo + r.dy, zn = r.zo + r.dz;
            const bool hl = k > 0, hr = k + 1 < n;
            const int al = GE::pos(hl ? k - 1 : k), ar = GE::pos(hr ? k + 1 : k);
            const double xl = X[al], yl = Y[al], zl = Z[al];
            const double xr = X[ar], yr = Y[ar], zr = Z[ar];
            const double fln = fene64(K, sq3(xl - xn, yl - yn, zl - zn));
            const double flo = fene64(K, sq3(xl - r.xo, yl - r.yo, zl - r.zo));
            const double frn = fene64(K, sq3(xr - xn, yr - yn, zr - zn));
            const double fro = fene64(K, sq3(xr - r.xo, yr - r.yo, zr - r.zo));
            r.dfl = hl ? fln - flo : 0.0;
            r.dfr = hr ? frn - fro : 0.0;
            S.ks[lane] = k;
            wave_sync();
            uint64_t cm = 0;
            for (int j = 0; j < ll; ++j) {
                const int dd = S.ks[g0 + j] - k;
                cm |= (dd >= -1 && dd <= 1) ? (1ull << j) : 0ull;
            }
            r.conflict = cm;
            r.pad = 0;
            S.rec[grp][ll] = r;
        }
        wave_sync();
        const int nb = (n - m0 < L) ? (n - m0) : L;
        uint64_t bits = 0;
        auto one_move = [&](const int i, const MoveRec &r) {
            const int k = r.k;
            const double th = r.th;
            const double thb_lo = r.thb * (1.0 - 0x1p-50), thb_hi = r.thb * (1.0 + 0x1p-50);
            double xo = r.xo, yo = r.yo, zo = r.zo, dfl = r.dfl, dfr = r.dfr;
            if ((r.conflict & bits) != 0) {
                // An accepted move of this batch touched k-1, k or k+1: lanes
                // 0..3 of the group evaluate (k-1,k) new/old, (k,k+1) new/old
                // from the current replica.
                const int pk = GE::pos(k);
                xo = X[pk];
                yo = Y[pk];
                zo = Z[pk];
                const double xq = xo + r.dx, yq = yo + r.dy, zq = zo + r.dz;
                const int nbr = (ll & 2) ? k + 1 : k - 1;
                const bool has = nbr >= 0 && nbr < n;
                const int pa = GE::pos(has ? nbr : k);
                const double xa = X[pa], ya = Y[pa], za = Z[pa];
                const bool nw = (ll & 1) == 0;
                const double fb = fene64(K, sq3(xa - (nw ? xq : xo), ya - (nw ? yq : yo), za - (nw ? zq : zo)));
                S.fv[lane] = has ? fb : 0.0;
                wave_sync();
                dfl = S.fv[g0] - S.fv[g0 + 1];
                dfr = S.fv[g0 + 2] - S.fv[g0 + 3];
                wave_sync();
            }
            const double xn = xo + r.dx, yn = yo + r.dy, zn = zo + r.dz;
            const double df = dfl + dfr;
            const int owner = k / B, slot = k % B;
            const bool mine = (ll == owner);
            bool acc = false, need = !MIXED;
            double de_used = 0.0, bm = 0.0, bsum_acc = 0.0;
            if constexpr (MIXED) {
                const LeafMx s = lane_tree<0, B>([&](int b) {
                    const bool skip = (mine && b == slot) || ll * B + b >= n;
                    return mixed_leaf(K, rx[b], ry[b], rz[b], xn, yn, zn, xo, yo, zo, skip);
                });
                const float smf = group_tree<L>(s.t);
                const float bsf = group_tree<L>(s.b);
                const double bsum = (double)bsf;
                const double dem = K.four_eps * (double)smf + df;
                const double bt = __builtin_fma(rel_band, dabs(dem), kb_band * bsum);
                const double lo = dem - bt, hi = dem + bt;
                const bool sure_acc = hi < thb_lo;
                const bool sure_rej = lo >= thb_hi;
                const bool broken = df == __builtin_inf();
                const bool sure = broken | (finite(dem) & (sure_acc | sure_rej));
                acc = !broken & sure_acc;
                de_used = dem;
                bsum_acc = bsum;
                need = !sure | (fp64_on_accept & acc);
                n_rescore += need ? 1 : 0;
            }
            if (__builtin_amdgcn_ballot_w64(need) != 0) {
                // The FP64-order score, for the wavefront; kept by the groups
                // that need it.
                __asm__ volatile("" ::: "memory");
                const Leaf64 s = lane_tree<0, B>([&](int b) {
                    const double en = lj64(K, sq3(rx[b] - xn, ry[b] - yn, rz[b] - zn));
                    const double eo = lj64(K, sq3(rx[b] - xo, ry[b] - yo, rz[b] - zo));
                    const double tt = (mine && b == slot) ? 0.0 : en - eo;
                    return Leaf64{tt, dabs(tt)};
                });
                const double sc = group_tree<L>(s.t);
                const double ab = group_tree<L>(s.a);
                if (need) {
                    const double de = sc + df;
                    acc = (de <= 0.0) || (beta * de < th);
                    de_used = de;
                    bm = bound64(log2c(n), ab, dfl, dfr, de);
                }
            }
            if (acc) {
                // The FP32 score's bound term, formed for accepted moves only
                // (the arithmetic of sweep_moves).
                if (MIXED && !need)
                    bm = (K.kbound * bsum_acc) * (1.0 + 0x1p-20) +
                         0x1p-52 * (2.0 * (dabs(dfl) + dabs(dfr)) + dabs(de_used));
                if (mine) {
                    const int ak = GE::pos(k);
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
            }
            wave_sync();
        };
        // The next move's record is read while the current move runs, in two
        // alternating register sets (as in sweep_moves at one wavefront).
        MoveRec ra = S.rec[grp][0];
        for (int i = 0; i < nb; i += 2) {
            const MoveRec rb = S.rec[grp][(i + 1 < L) ? i + 1 : L - 1];
            one_move(i, ra);
            if (i + 1 >= nb) break;
            ra = S.rec[grp][(i + 2 < L) ? i + 2 : L - 1];
            one_move(i + 1, rb);
        }
        logword |= bits << (m0 & 63);
        if (ll == 0 && (((m0 + L) & 63) == 0 || m0 + L >= n)) {
            if (logrow != nullptr) logrow[m0 >> 6] = logword;
            digest = mix64(digest ^ logword);
        }
        if (((m0 + L) & 63) == 0) logword = 0;
    }
    if (ll == 0) T.dig[2 * g] = digest;
    for (int i = ll; i < 3 * NP; i += L) cq[i] = X[i];

    // ---- record (sweep_record, per group)
    const bool resync = T.full_energy || !(Bd <= K.resync_rel * (dabs(E) > 1.0 ? dabs(E) : 1.0));
    if (resync) {
        E = pack_energy<BU, G>(X, Y, Z, n, K, ll);
        Bd = bound_energy(K, log2c(n), n, E, 0.0);
    }
    double ree2, rg2;
    pack_shape<BU, G>(X, Y, Z, n, ll, ree2, rg2);
    if (ll == 0) {
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

}  // namespace

}  // namespace pt
