// pt_k_flow.hip -- launchers of the task-flow kernel.
#include "pt_kernels.hpp"

namespace pt {

namespace {

// Reset of the task counter of k_flow (a kernel, not a memset: safe to capture).
__global__ void k_flow_reset(const Tables T) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *T.flow_task = 0;
}

template <int B, int W>
hipError_t flow_cap_bw(bool mixed, int64_t *blocks) {
    const void *f = mixed ? (const void *)k_flow<B, W, true> : (const void *)k_flow<B, W, false>;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err == hipSuccess) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64 * W, 0);
    *blocks = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
    return err;
}

template <int B, int W>
hipError_t flow_bw(bool mixed, const Tables &T, const int32_t *list, int n, int64_t n_sweeps, int64_t resident,
                   hipStream_t s) {
    if (n <= 0 || n_sweeps <= 0) return hipSuccess;
    const int64_t tasks = n_sweeps * (int64_t)n;
    const unsigned grid = (unsigned)(tasks < resident ? tasks : resident);
    hipLaunchKernelGGL(k_flow_reset, dim3(1), dim3(64), 0, s, T);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (mixed)
        hipLaunchKernelGGL((k_flow<B, W, true>), dim3(grid), dim3(64 * W), 0, s, T, list, n, n_sweeps);
    else
        hipLaunchKernelGGL((k_flow<B, W, false>), dim3(grid), dim3(64 * W), 0, s, T, list, n, n_sweeps);
    return hipGetLastError();
}

}  // namespace

hipError_t flow_capacity(int bpl, int wpr, bool mixed, int64_t *blocks) {
#define PT_FC(B, W) flow_cap_bw<B, W>(mixed, blocks)
    PT_DISPATCH(bpl, wpr, PT_FC)
#undef PT_FC
}

hipError_t launch_flow(int bpl, int wpr, bool mixed, const Tables &T, const int32_t *list, int n,
                       int64_t n_sweeps, int64_t resident, hipStream_t s) {
#define PT_FL(B, W) flow_bw<B, W>(mixed, T, list, n, n_sweeps, resident, s)
    PT_DISPATCH(bpl, wpr, PT_FL)
#undef PT_FL
}

}  // namespace pt
