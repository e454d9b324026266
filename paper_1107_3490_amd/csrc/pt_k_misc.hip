// pt_k_misc.hip -- launchers of the energy, exchange, counter and diagnostic kernels.
#include "pt_kernels.hpp"

namespace pt {

namespace {

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

// Advance the run counters past n sweeps run by persistent or task-flow
// launches (which read them at their start): t += n, and e by the exchange
// steps due after sweeps t .. t + n - 1.
__global__ void k_advance_n(const Tables T, int64_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t t = T.te[0];
    const int64_t ev = T.exchange_every;
    T.te[0] = t + n;
    if (ev > 0) T.te[1] += (t + n) / ev - t / ev;
}

// --------------------------------------------------------------- selftest --
__global__ void k_selftest(const Consts k, int op, const double *x, const double *y, double *out,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (op == 9) {
        // The FP32 pair sum of one move as the mixed sweep scores it at 8
        // beads per lane and one wavefront (the per-lane leaf tree and the
        // butterfly), one wavefront per item; whole wavefronts (the launch
        // has 64 n threads).  Item: 512 beads xyz, then N, k, d.
        const int64_t item = i >> 6;
        if (item >= n) return;
        const int lane = threadIdx.x & 63;
        const double *p = x + item * kMoveItem;
        const int nb = (int)p[3 * 512], kk = (int)p[3 * 512 + 1];
        const double xo = p[3 * kk], yo = p[3 * kk + 1], zo = p[3 * kk + 2];
        const double xn = xo + p[3 * 512 + 2], yn = yo + p[3 * 512 + 3], zn = zo + p[3 * 512 + 4];
        const LeafMx s = lane_tree<0, 8>([&](int b) {
            const int j = lane * 8 + b;
            return mixed_leaf(k, p[3 * j], p[3 * j + 1], p[3 * j + 2], xn, yn, zn, xo, yo, zo,
                              j == kk || j >= nb);
        });
        const double sm = (double)wave_tree(s.t), bsum = (double)wave_tree(s.b);
        if (lane == 0) {
            out[2 * item] = k.four_eps * sm;
            out[2 * item + 1] = k.kbound * bsum;
        }
        return;
    }
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
            // One pair whose old separation lies on the cutoff, as the sweep
            // scores it: 4 eps (g(r) - g(rc)) and its bound.
            const Lj32 r = lj32(k, sq3(x[i], y[i], 0.0));
            const Lj32 c = lj32(k, k.rc2);
            out[2 * i] = k.four_eps * (double)(r.g - c.g);
            const float sb = r.s6 + c.s6;
            out[2 * i + 1] = k.kbound * (double)__builtin_fmaf(sb, sb, sb);
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
hipError_t energy_bw(const Tables &T, const int32_t *list, int n, double *oe, double *ob, int by_slot,
                     hipStream_t s) {
    hipLaunchKernelGGL((k_energy<B, W>), dim3(n), dim3(64 * W), 0, s, T, list, oe, ob, by_slot);
    return hipGetLastError();
}

template <int B, int W>
hipError_t energy_pairs_bw(const Tables &T, const int32_t *list, int n, double *oe, double *ob, hipStream_t s) {
    hipLaunchKernelGGL((k_energy_pairs<B, W>), dim3(n), dim3(64 * W), 0, s, T, list, oe, ob);
    return hipGetLastError();
}

template <int B, int W>
hipError_t exchange_bw(const Tables &T, const int32_t *list, int nc, int mp, int force, hipStream_t s) {
    hipLaunchKernelGGL((k_exchange<B, W>), dim3(nc * mp), dim3(64 * W), 0, s, T, list, mp, force);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_energy(int bpl, int wpr, const Tables &T, const int32_t *list, int n, double *out_e,
                         double *out_b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int by_slot = (out_b == nullptr) ? 1 : 0;
#define PT_EN(B, W) energy_bw<B, W>(T, list, n, out_e, out_b, by_slot, s)
    PT_DISPATCH(bpl, wpr, PT_EN)
#undef PT_EN
}

hipError_t launch_energy_pairs(int bpl, int wpr, const Tables &T, const int32_t *list, int n, double *out_e,
                               double *out_b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define PT_EP(B, W) energy_pairs_bw<B, W>(T, list, n, out_e, out_b, s)
    PT_DISPATCH(bpl, wpr, PT_EP)
#undef PT_EP
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

hipError_t launch_advance_n(const Tables &T, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_advance_n, dim3(1), dim3(64), 0, s, T, n);
    return hipGetLastError();
}

hipError_t launch_selftest(const Consts &k, int op, const double *x, const double *y, double *out,
                           int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t threads = (op == 9) ? 64 * n : n;  // op 9: one wavefront per item
    const int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_selftest, dim3((unsigned)blocks), dim3(256), 0, s, k, op, x, y, out, n);
    return hipGetLastError();
}

}  // namespace pt
