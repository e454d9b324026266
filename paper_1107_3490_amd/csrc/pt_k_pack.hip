// pt_k_pack.hip -- launcher of the per-sweep kernel that packs two or four
// replicas of a short chain into one wavefront.
#include "pt_pack.hpp"

namespace pt {

namespace {

template <int BU, int G>
hipError_t sweep_pack_bg(bool mixed, const Tables &T, const int32_t *list, int n_blocks, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL((k_sweep_pack<BU, G, true>), dim3(n_blocks), dim3(64), 0, s, T, list);
    else
        hipLaunchKernelGGL((k_sweep_pack<BU, G, false>), dim3(n_blocks), dim3(64), 0, s, T, list);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_pack(int bpl, int pack, bool mixed, const Tables &T, const int32_t *list, int n_blocks,
                             hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    switch (bpl * 16 + pack) {
        case 1 * 16 + 2: return sweep_pack_bg<1, 2>(mixed, T, list, n_blocks, s);
        case 1 * 16 + 4: return sweep_pack_bg<1, 4>(mixed, T, list, n_blocks, s);
        case 2 * 16 + 2: return sweep_pack_bg<2, 2>(mixed, T, list, n_blocks, s);
        case 2 * 16 + 4: return sweep_pack_bg<2, 4>(mixed, T, list, n_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pt
