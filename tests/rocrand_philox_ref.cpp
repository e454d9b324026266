// Test helper: exposes rocRAND's Philox4x32-10 block function (header-only,
// host-callable) so the oracle's Philox can be checked against a library.
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>
namespace {
struct probe : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}
extern "C" void ref_philox(const uint32_t* ctr, uint64_t seed, uint32_t* out) {
  probe p;
  uint4 c = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint2 k = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint4 r = p.rounds(c, k);
  out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}
