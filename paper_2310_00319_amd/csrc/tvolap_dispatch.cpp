// Hop and storage-type dispatch: the kernel file is compiled once per
// supported hop L and storage type, and each compilation provides the hop_*
// launchers for its pair.
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

template <typename F>
hipError_t by_dtype(int dt, F&& f) {
  switch (dt) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename F>
hipError_t by_hop_dtype(int L, int dt, F&& f) {
  return by_hop(L, [&](auto Lc) { return by_dtype(dt, [&](auto Dc) { return f(Lc, Dc); }); });
}

}  // namespace

hipError_t launch_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride, float* hist, void* fdl,
                      const uint64_t* counter, hipStream_t s) {
  return by_hop_dtype(P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_fwd<decltype(Lc)::value, decltype(Dc)::value>(P, dtype, in, in_stride, hist, fdl, counter, s);
  });
}

hipError_t launch_inv(const DevPlan& P, int dtype, const float2* ypart, const void* bank, const void* fdl,
                      const int32_t* sel, float* ola, float* out, int64_t out_stride, int32_t copy_sel,
                      int32_t* sel_store, int32_t* done, uint64_t* counter, hipStream_t s) {
  return by_hop_dtype(P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_inv<decltype(Lc)::value, decltype(Dc)::value>(P, dtype, ypart, bank, fdl, sel, ola, out, out_stride,
                                                             copy_sel, sel_store, done, counter, s);
  });
}

hipError_t launch_block(const BlockArgs& A, int dtype, const MacShape& shape, int grid, hipStream_t s) {
  return by_hop_dtype(A.P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_block<decltype(Lc)::value, decltype(Dc)::value>(A, dtype, shape, grid, s);
  });
}

hipError_t launch_batch(const BatchArgs& B, int dtype, const MacShape& shape, int grid, const float* in,
                        int64_t in_stride, float* hist, float* ola, float* out, int64_t out_stride, hipStream_t s,
                        hipEvent_t* ev) {
  return by_hop_dtype(B.P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_batch<decltype(Lc)::value, decltype(Dc)::value>(B, dtype, shape, grid, in, in_stride, hist, ola, out,
                                                               out_stride, s, ev);
  });
}

hipError_t launch_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M, void* dst,
                         hipStream_t s) {
  return by_hop_dtype(P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_irprep<decltype(Lc)::value, decltype(Dc)::value>(P, dtype, taps, n_taps, M, dst, s);
  });
}

hipError_t launch_irprep_all(const DevPlan& P, int dtype, const int32_t* part_base, int32_t total_parts,
                             const int32_t* ch_taps, const float* taps, int64_t taps_stride, int32_t slot, void* bank,
                             hipStream_t s) {
  return by_hop_dtype(P.L, dtype, [&](auto Lc, auto Dc) {
    return hop_irprep_all<decltype(Lc)::value, decltype(Dc)::value>(P, dtype, part_base, total_parts, ch_taps, taps,
                                                                    taps_stride, slot, bank, s);
  });
}

hipError_t launch_mac(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items, int n_items,
                      const void* bank, const void* fdl, const int32_t* sel, float2* ypart,
                      const uint64_t* counter, hipStream_t s) {
  return by_dtype(dtype, [&](auto Dc) {
    return mac_dt<decltype(Dc)::value>(P, dtype, shape, items, n_items, bank, fdl, sel, ypart, counter, s);
  });
}

}  // namespace tvx
