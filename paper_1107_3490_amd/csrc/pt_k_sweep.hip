// pt_k_sweep.hip -- launchers of the per-sweep kernels (one wavefront group per replica, and one lane per replica).
#include "pt_kernels.hpp"

namespace pt {

namespace {

template <int B, int W>
hipError_t sweep_bw(bool mixed, const Tables &T, const int32_t *list, int n, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL((k_sweep<B, W, true>), dim3(n), dim3(64 * W), 0, s, T, list);
    else
        hipLaunchKernelGGL((k_sweep<B, W, false>), dim3(n), dim3(64 * W), 0, s, T, list);
    return hipGetLastError();
}

template <int B, int W>
hipError_t sweep_lane_bw(const Tables &T, const int32_t *list, int n, hipStream_t s) {
    hipLaunchKernelGGL((k_sweep_lane<B, W>), dim3((n + 63) / 64), dim3(64), 0, s, T, list, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(int bpl, int wpr, bool mixed, const Tables &T, const int32_t *list, int n,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define PT_SW(B, W) sweep_bw<B, W>(mixed, T, list, n, s)
    PT_DISPATCH(bpl, wpr, PT_SW)
#undef PT_SW
}

hipError_t launch_sweep_lane(int bpl, int wpr, const Tables &T, const int32_t *list, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define PT_SL(B, W) sweep_lane_bw<B, W>(T, list, n, s)
    PT_DISPATCH(bpl, wpr, PT_SL)
#undef PT_SL
}

}  // namespace pt
