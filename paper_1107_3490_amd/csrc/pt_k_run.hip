// pt_k_run.hip -- dispatch of the persistent kernel over its builds (one
// translation unit per wavefront count and precision, pt_k_run<W><m|d>.hip).
#include "pt_internal.hpp"

namespace pt {

hipError_t run_cap_1m(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_1m(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);
hipError_t run_cap_1d(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_1d(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);
hipError_t run_cap_2m(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_2m(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);
hipError_t run_cap_2d(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_2d(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);
hipError_t run_cap_4m(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_4m(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);
hipError_t run_cap_4d(int max_bpl, bool dense, int64_t *blocks);
hipError_t run_launch_4d(bool dense, const Tables &T, const int32_t *list, int n, int max_bpl, int64_t n_sweeps, hipStream_t s);

hipError_t run_capacity(int wpr, bool mixed, int max_bpl, bool dense, int64_t *blocks) {
    switch (wpr * 2 + (mixed ? 1 : 0)) {
        case 3: return run_cap_1m(max_bpl, dense, blocks);
        case 2: return run_cap_1d(max_bpl, dense, blocks);
        case 5: return run_cap_2m(max_bpl, dense, blocks);
        case 4: return run_cap_2d(max_bpl, dense, blocks);
        case 9: return run_cap_4m(max_bpl, dense, blocks);
        case 8: return run_cap_4d(max_bpl, dense, blocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_run(int wpr, bool mixed, bool dense, const Tables &T, const int32_t *list, int n,
                      int max_bpl, int64_t n_sweeps, hipStream_t s) {
    switch (wpr * 2 + (mixed ? 1 : 0)) {
        case 3: return run_launch_1m(dense, T, list, n, max_bpl, n_sweeps, s);
        case 2: return run_launch_1d(dense, T, list, n, max_bpl, n_sweeps, s);
        case 5: return run_launch_2m(dense, T, list, n, max_bpl, n_sweeps, s);
        case 4: return run_launch_2d(dense, T, list, n, max_bpl, n_sweeps, s);
        case 9: return run_launch_4m(dense, T, list, n, max_bpl, n_sweeps, s);
        case 8: return run_launch_4d(dense, T, list, n, max_bpl, n_sweeps, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pt
