// Hop dispatch: the kernel file is compiled once per supported hop L, and
// each compilation provides the hop_* launchers for its L.
#include <type_traits>

#include "tvolap_internal.h"

namespace tvx {

namespace {

template <typename F>
hipError_t by_hop(int L, F&& f) {
  switch (L) {
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride, float* hist, void* fdl,
                      const uint64_t* counter, hipStream_t s) {
  return by_hop(P.L, [&](auto Lc) {
    return hop_fwd<decltype(Lc)::value>(P, dtype, in, in_stride, hist, fdl, counter, s);
  });
}

hipError_t launch_inv(const DevPlan& P, int dtype, const float2* ypart, const void* bank, const void* fdl,
                      const int32_t* sel, float* ola, float* out, int64_t out_stride, int32_t copy_sel,
                      int32_t* sel_store, int32_t* done, uint64_t* counter, hipStream_t s) {
  return by_hop(P.L, [&](auto Lc) {
    return hop_inv<decltype(Lc)::value>(P, dtype, ypart, bank, fdl, sel, ola, out, out_stride, copy_sel,
                                        sel_store, done, counter, s);
  });
}

hipError_t launch_block(const BlockArgs& A, int dtype, const MacShape& shape, int grid, hipStream_t s) {
  return by_hop(A.P.L, [&](auto Lc) { return hop_block<decltype(Lc)::value>(A, dtype, shape, grid, s); });
}

hipError_t launch_batch(const BatchArgs& B, int dtype, const MacShape& shape, int grid, const float* in,
                        int64_t in_stride, float* hist, float* ola, float* out, int64_t out_stride, hipStream_t s,
                        hipEvent_t* ev) {
  return by_hop(B.P.L, [&](auto Lc) {
    return hop_batch<decltype(Lc)::value>(B, dtype, shape, grid, in, in_stride, hist, ola, out, out_stride, s,
                                          ev);
  });
}

hipError_t launch_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M, void* dst,
                         hipStream_t s) {
  return by_hop(P.L, [&](auto Lc) { return hop_irprep<decltype(Lc)::value>(P, dtype, taps, n_taps, M, dst, s); });
}

}  // namespace tvx
