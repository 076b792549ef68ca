// gfx950 kernels of the TVOLAP hot path (Jaeger et al., arXiv 2310.00319, Sec. 2).
//
// Fused path (one launch per block):
//   k_block   Two kinds of work item. Spectrum items (one per input) build the
//             new input spectrum: Hann-weighted 2L block (eq. 1-2), zero pad to
//             4L (eq. 5), real 4L-point DFT (eq. 4), stored in the delay line.
//             MAC items cover (input, up to 4 channels of that input, bin tile,
//             chunk of partitions m >= 1): the spectral MAC of eq. 8 streamed
//             from HBM in 16-byte lanes, FP32 accumulation, partitions split
//             across the waves and reduced in LDS, partial spectrum tiles
//             written out. The last item to arrive for a channel (device-scope
//             counter; no item ever waits for another) adds the m = 0 term,
//             sums the channel's partial tiles, runs the inverse DFT (eq. 9) and
//             the overlap-add at hop L (eq. 10-13).
// Plain path (three launches per block, the unfused baseline):
//   k_fwd, k_mac, k_inv with the same arithmetic.
//   k_irprep  IR partition spectra (eq. 3, 6-7) into a bank slot.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>
#include <numeric>

#include "fft_lds.hpp"
#include "tvolap_internal.h"

#if !defined(TVX_HOP) || !defined(TVX_DT)
#error "compile once per hop and storage type with -DTVX_HOP=64|128|256|512 -DTVX_DT=0|1|2"
#endif
static_assert(TVX_HOP == 64 || TVX_HOP == 128 || TVX_HOP == 256 || TVX_HOP == 512, "unsupported hop");
static_assert(TVX_DT == 0 || TVX_DT == 1 || TVX_DT == 2, "unsupported storage type");

namespace tvx {
namespace {

using fft::cadd;
using fft::cmul;

// ---------------------------------------------------------------- storage types

// dtype 0: float2 per complex value. dtype 1: two bf16 in a 32-bit word
// (real in the low half). dtype 2: two IEEE binary16 in a 32-bit word.
template <int DT> struct Store { using T = uint32_t; };
template <> struct Store<0> { using T = float2; };

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t f32_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}

template <int DT> __device__ __forceinline__ typename Store<DT>::T pack(float2 v);
template <> __device__ __forceinline__ float2 pack<0>(float2 v) { return v; }
template <> __device__ __forceinline__ uint32_t pack<1>(float2 v) {
  return f32_to_bf16_rne(v.x) | (f32_to_bf16_rne(v.y) << 16);
}
template <> __device__ __forceinline__ uint32_t pack<2>(float2 v) {
  return f32_to_f16_rne(v.x) | (f32_to_f16_rne(v.y) << 16);
}

template <int DT> __device__ __forceinline__ float2 unpack(typename Store<DT>::T w);
template <> __device__ __forceinline__ float2 unpack<0>(float2 w) { return w; }
template <> __device__ __forceinline__ float2 unpack<1>(uint32_t w) {
  return make_float2(bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16));
}
template <> __device__ __forceinline__ float2 unpack<2>(uint32_t w) {
  return make_float2(f16_to_f32(w), f16_to_f32(w >> 16));
}

// Load V consecutive stored complex values (16 bytes per lane where possible).
template <int DT, int V>
__device__ __forceinline__ void load_vec(const typename Store<DT>::T* __restrict__ p, float2 (&o)[V]) {
  if constexpr (DT == 0 && V == 1) {
    o[0] = p[0];
  } else if constexpr (DT == 0) {
#pragma unroll
    for (int j = 0; j < V; j += 2) {
      const float4 t = *reinterpret_cast<const float4*>(p + j);
      o[j] = make_float2(t.x, t.y);
      o[j + 1] = make_float2(t.z, t.w);
    }
  } else {
    uint32_t w[V];
    if constexpr (V == 1) {
      w[0] = p[0];
    } else if constexpr (V == 2) {
      const uint2 t = *reinterpret_cast<const uint2*>(p);
      w[0] = t.x; w[1] = t.y;
    } else {
#pragma unroll
      for (int j = 0; j < V; j += 4) {
        const uint4 t = *reinterpret_cast<const uint4*>(p + j);
        w[j] = t.x; w[j + 1] = t.y; w[j + 2] = t.z; w[j + 3] = t.w;
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) o[j] = unpack<DT>(w[j]);
  }
}

// load_vec with the non-temporal hint: partition spectra are streamed once per
// block, so they are kept from displacing the delay line (read again two
// blocks later) in the caches.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
template <int DT, int V>
__device__ __forceinline__ void load_vec_nt(const typename Store<DT>::T* __restrict__ p, float2 (&o)[V]) {
  if constexpr (DT == 0 && V % 2 == 0) {
#pragma unroll
    for (int j = 0; j < V; j += 2) {
      const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p + j));
      o[j] = make_float2(t.x, t.y);
      o[j + 1] = make_float2(t.z, t.w);
    }
  } else if constexpr (DT != 0 && V == 2) {
    const nt_u2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p));
    o[0] = unpack<DT>(t.x);
    o[1] = unpack<DT>(t.y);
  } else if constexpr (DT != 0 && V % 4 == 0) {
#pragma unroll
    for (int j = 0; j < V; j += 4) {
      const nt_u4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p + j));
      o[j] = unpack<DT>(t.x);
      o[j + 1] = unpack<DT>(t.y);
      o[j + 2] = unpack<DT>(t.z);
      o[j + 3] = unpack<DT>(t.w);
    }
  } else {
    load_vec<DT, V>(p, o);
  }
}

// 16-bit storage: V stored words as they are (16 bytes per lane where
// possible), plain or with the non-temporal hint.
template <int V, bool NT>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ p, uint32_t (&w)[V]) {
  if constexpr (V == 1) {
    w[0] = p[0];
  } else if constexpr (V == 2) {
    const nt_u2 t = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p))
                       : *reinterpret_cast<const nt_u2*>(p);
    w[0] = t.x; w[1] = t.y;
  } else {
#pragma unroll
    for (int j = 0; j < V; j += 4) {
      const nt_u4 t = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p + j))
                         : *reinterpret_cast<const nt_u4*>(p + j);
      w[j] = t.x; w[j + 1] = t.y; w[j + 2] = t.z; w[j + 3] = t.w;
    }
  }
}

// a.lo b.lo + a.hi b.hi + c in FP32 for two 16-bit values per word (bf16 for
// DT 1, binary16 for DT 2); products of 16-bit values are exact in FP32.
template <int DT>
__device__ __forceinline__ float dot2w(uint32_t a, uint32_t b, float c) {
  if constexpr (DT == 1) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2, a), __builtin_bit_cast(b2, b), c, false);
  } else {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, a), __builtin_bit_cast(h2, b), c, false);
  }
}

// Device-coherent publication of partial spectra between workgroups of one
// launch. Relaxed agent-scope atomic stores and loads of the 8-byte values are
// performed at the device coherence point (they are not kept in, or served
// from, the non-coherent per-XCD L2), so a writer that waits for its stores to
// complete before incrementing a counter, and a reader that loads after seeing
// that increment, need no cache-wide write-back or invalidate.
__device__ __forceinline__ void store_coherent(float2* p, float2 v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 load_coherent(const float2* p) {
  return __builtin_bit_cast(
      float2, __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ uint32_t load_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool COHERENT, typename T>
__device__ __forceinline__ void store_maybe(T* p, T v) {
  if constexpr (COHERENT) store_coherent(p, v); else *p = v;
}
template <bool COHERENT, typename T>
__device__ __forceinline__ T load_maybe(const T* p) {
  if constexpr (COHERENT) return load_coherent(p); else return *p;
}
// Wait until every memory operation of this wave has completed.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------- shared steps

// Twiddles exp(-2 pi i t / 4L) (t < 4L) and the window (2L) into LDS.
template <int L, int T>
__device__ __forceinline__ void load_tables(const DevPlan& P, float2* twl, float* winl, int tid) {
#pragma unroll
  for (int i = tid; i < 4 * L; i += T) twl[i] = P.tw[i];
#pragma unroll
  for (int i = tid; i < 2 * L; i += T) winl[i] = P.win[i];
}

// Block counter -> delay-line position: parity p of the call, slot q within
// the parity's ring of M_i spectra.
__device__ __forceinline__ int ring_slot(uint64_t cnt, int Mi) { return (int)((cnt >> 1) % (uint64_t)Mi); }

// Where the completion of a channel reads (stored-element offsets): X(l), its
// input's spectrum of this block, in the delay line; H_{c, slot}(0) in the
// bank; its first partial row and the partial rows per tile.
struct FinDesc {
  int64_t x, h;
  int32_t rows, nch;
};
template <int L>
__device__ __forceinline__ FinDesc lookup_desc(const DevPlan& P, const int32_t* __restrict__ sel, int c, int p,
                                               uint64_t cnt) {
  constexpr int N = 2 * L;
  const int i = P.ch_input[c];
  const int Mi = P.in_M[i];
  int s = sel[c];
  s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s);
  FinDesc d;
  d.x = P.in_fdl_off[i] + ((int64_t)p * Mi + ring_slot(cnt, Mi)) * N;
  d.h = P.ch_bank_off[c] + (int64_t)s * P.ch_M[c] * N;
  d.rows = P.ch_row_base[c];
  d.nch = P.ch_nchunks[c];
  return d;
}

// New input spectrum of input i (eq. 1, 2, 4, 5): the 2L-sample block (the
// previous L samples, history parity p^1, then the L new ones) weighted by the
// window, zero padded to 4L and transformed; the packed spectrum, rounded to
// the storage type, goes to delay-line slot (p, q). The new samples become the
// history of parity p. COHERENT: publish for readers in the same launch.
template <int L, int T, int DT, bool COHERENT>
__device__ __forceinline__ void input_spectrum(const DevPlan& P, const float* __restrict__ in, int64_t in_stride,
                                               float* __restrict__ hist, typename Store<DT>::T* __restrict__ fdl,
                                               int i, int p, uint64_t cnt, const float2* twl, const float* winl,
                                               float2* bufA, float2* bufB, int tid) {
  constexpr int N = 2 * L;
  const float* hold = hist + ((size_t)(p ^ 1) * P.I + i) * L;
  float* hnew = hist + ((size_t)p * P.I + i) * L;
  const float* xin = in + (int64_t)i * in_stride;
#pragma unroll
  for (int n = tid; n < L; n += T) {
    const int t0 = 2 * n, t1 = 2 * n + 1;
    const float s0 = (t0 < L) ? hold[t0] : xin[t0 - L];
    const float s1 = (t1 < L) ? hold[t1] : xin[t1 - L];
    bufA[n] = make_float2(winl[t0] * s0, winl[t1] * s1);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int n = tid; n < L; n += T) hnew[n] = xin[n];
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  const int Mi = P.in_M[i];
  typename Store<DT>::T* dst = fdl + P.in_fdl_off[i] + ((int64_t)p * Mi + ring_slot(cnt, Mi)) * N;
#pragma unroll
  for (int k = tid; k < N; k += T) store_maybe<COHERENT>(dst + k, pack<DT>(fft::real_fwd_post<N>(Z, k, twl)));
}

// Spectral MAC of one work item (eq. 8) over partitions m >= 1 of its range:
// acc[g] += H_{c_g, slot}(m) X(l - 2m) for this lane's V bins. The waves of the
// workgroup take every NW-th partition; two partitions are in flight per wave.
// The packed bin 0 holds two real bins and multiplies component-wise.
// fd (LDS, may be null): thread 0 also records there the completion
// descriptors of the item's channels, from the offsets the MAC computes anyway.
template <int V, int G, int NW, int DT, int U>
__device__ __forceinline__ void mac_item(const DevPlan& P, const WorkItem& it,
                                         const typename Store<DT>::T* __restrict__ bank,
                                         const typename Store<DT>::T* __restrict__ fdl,
                                         const int32_t* __restrict__ sel, int p, uint64_t cnt, int lane, int w,
                                         float2 (&acc)[G][V], FinDesc* fd = nullptr) {
  using ST = typename Store<DT>::T;
  constexpr int TW = 64 * V;
  const int N = 2 * P.L;
  const int Mi = P.in_M[it.input];
  const int q = ring_slot(cnt, Mi);
  const int kbase = it.tile * TW + lane * V;
  // Row bases are uniform across the wave; lanes add a 32-bit offset.
  const ST* xbase = fdl + P.in_fdl_off[it.input] + (int64_t)p * Mi * N;
  const ST* hbase[G];
  int Mc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g < it.n_ch) {
      const int ch = it.ch[g];
      int s = sel[ch];
      s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s);
      Mc[g] = P.ch_M[ch];
      hbase[g] = bank + P.ch_bank_off[ch] + (int64_t)s * Mc[g] * N;
    } else {
      Mc[g] = 0;
      hbase[g] = bank;
    }
  }
  if (fd != nullptr && lane == 0 && w == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g < it.n_ch) {
        FinDesc d;
        d.x = (xbase - fdl) + (int64_t)q * N;
        d.h = hbase[g] - bank;
        d.rows = it.row[g] - it.tile * it.nch - it.chunk;
        d.nch = it.nch;
        fd[g] = d;
      }
    }
  }
  const bool dc_lane = (kbase == 0);
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[g][v] = make_float2(0.f, 0.f);

  // f32: complex values, four FMAs per product. 16-bit: the stored words,
  // two packed dot products per product (Re += (h.re, -h.im).(x.re, x.im),
  // Im += (h.re, h.im).(x.im, x.re)), nothing unpacked.
  using LW = std::conditional_t<DT == 0, float2, uint32_t>;
  auto load_x = [&](const ST* p, LW (&o)[V]) {
    if constexpr (DT == 0) load_vec<0, V>(p, o); else load_words<V, false>(p, o);
  };
  auto load_h = [&](const ST* p, LW (&o)[V]) {
    if constexpr (DT == 0) load_vec_nt<0, V>(p, o); else load_words<V, true>(p, o);
  };
  auto accumulate = [&](int g, const LW (&H)[V], const LW (&X)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if constexpr (DT == 0) {
        float2 prod = cmul(H[v], X[v]);
        if (v == 0 && dc_lane) prod = make_float2(H[0].x * X[0].x, H[0].y * X[0].y);
        acc[g][v] = cadd(acc[g][v], prod);
      } else {
        const uint32_t h = H[v], x = X[v];
        uint32_t hr = h ^ 0x80000000u, hi = h, xi = __builtin_amdgcn_alignbit(x, x, 16);
        if (v == 0 && dc_lane) {
          // packed (Re X(0), Re X(2L)): component-wise products
          hr = h & 0xffffu;
          hi = h & 0xffff0000u;
          xi = x;
        }
        acc[g][v].x = dot2w<DT>(hr, x, acc[g][v].x);
        acc[g][v].y = dot2w<DT>(hi, xi, acc[g][v].y);
      }
    }
  };
  int m = (it.m0 > 1 ? it.m0 : 1) + w;
  for (; m + (U - 1) * NW < it.m1; m += U * NW) {
    LW X[U][V];
    LW H[U][G][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int xr = q - (m + u * NW);
      if (xr < 0) xr += Mi;
      load_x(xbase + (uint32_t)(xr * N + kbase), X[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (m + u * NW < Mc[g]) load_h(hbase[g] + (uint32_t)((m + u * NW) * N + kbase), H[u][g]);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (m + u * NW < Mc[g]) accumulate(g, H[u][g], X[u]);
  }
  for (; m < it.m1; m += NW) {
    int xr = q - m;
    if (xr < 0) xr += Mi;
    LW X[V];
    load_x(xbase + (uint32_t)(xr * N + kbase), X);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (m < Mc[g]) {
        LW H[V];
        load_h(hbase[g] + (uint32_t)(m * N + kbase), H);
        accumulate(g, H, X);
      }
    }
  }
}

// Reduce the waves' accumulators through LDS and write the item's partial
// spectrum tiles (row[g] of the partial buffer).
template <int V, int G, int NW, bool COHERENT>
__device__ __forceinline__ void write_partials(const WorkItem& it, float2 (&acc)[G][V], float2 (*red)[G][64 * V],
                                               float2* __restrict__ ypart, int lane, int w, int tid) {
  constexpr int TW = 64 * V;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < V; ++v) red[w][g][lane * V + v] = acc[g][v];
  __syncthreads();
  // g runs over compile-time indices so that the item stays in registers
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g < it.n_ch) {
      float2* dst = ypart + (int64_t)it.row[g] * TW;
      for (int b = tid; b < TW; b += 64 * NW) {
        float2 s = red[0][g][b];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) s = cadd(s, red[ww][g][b]);
        store_maybe<COHERENT>(dst + b, s);
      }
    }
  }
}

// Inverse real DFT of the packed spectrum Y (eq. 9) and overlap-add (eq. 10-13):
// out(n) = state(n) + y(n) for n < L, state'(n) = state(n + L) + y(n + L) for
// n < 2L, state'(2L + n) = y(3L + n) for n < L. Y, bufA, bufB in LDS.
template <int L, int T>
__device__ __forceinline__ void ola_prefetch(const float* __restrict__ st, float (&old)[(4 * L + T - 1) / T],
                                             int tid) {
#pragma unroll
  for (int j = 0; j < (4 * L + T - 1) / T; ++j) {
    const int n = tid + j * T;
    old[j] = (n < 3 * L) ? st[n] : 0.f;
  }
}

template <int L, int T>
__device__ __forceinline__ void inverse_ola(float2* Y, float2* bufA, float2* bufB, const float2* twl,
                                            const float (&old)[(4 * L + T - 1) / T], float* __restrict__ st,
                                            float* __restrict__ o, int tid) {
  constexpr int N = 2 * L;
  constexpr int NPT = (4 * L + T - 1) / T;
#pragma unroll
  for (int k = tid; k < N; k += T) bufA[k] = fft::real_inv_pre_conj<N>(Y, k, twl);
  __syncthreads();
  const float2* R = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  constexpr float scale = 1.0f / (float)(4 * L);
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int n = tid + j * T;
    if (n < 4 * L) {
      const float2 z = R[n >> 1];
      const float yv = ((n & 1) ? -z.y : z.x) * scale;
      if (n < L) {
        o[n] = old[j] + yv;
      } else if (n < 3 * L) {
        st[n - L] = old[j] + yv;
      } else {
        st[n - L] = yv;
      }
    }
  }
}

// Spectrum of channel c for this block into Y (LDS): the sum of its partial
// tiles (partitions m >= 1) plus H_{c, slot}(0) X(l) (eq. 8, m = 0 term, X(l)
// read back from the delay line). COHERENT: the partial tiles and X(l) were
// published by other workgroups of the same launch. No barrier at the end.
template <int L, int T, int DT, bool COHERENT, bool ACC = false>
__device__ __forceinline__ void channel_spectrum(const DevPlan& P, const float2* __restrict__ ypart,
                                                 const typename Store<DT>::T* __restrict__ bank,
                                                 const typename Store<DT>::T* __restrict__ fdl,
                                                 const int32_t* __restrict__ sel, int c, int p, uint64_t cnt,
                                                 float2* Y, int tid) {
  using ST = typename Store<DT>::T;
  constexpr int N = 2 * L;
  const int TW = P.tile_width;
  const int base = P.ch_row_base[c];
  const int nch = P.ch_nchunks[c];
  const int i = P.ch_input[c];
  const int Mi = P.in_M[i];
  const ST* xrow = fdl + P.in_fdl_off[i] + ((int64_t)p * Mi + ring_slot(cnt, Mi)) * N;
  int s = sel[c];
  s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s);
  const ST* h0 = bank + P.ch_bank_off[c] + (int64_t)s * P.ch_M[c] * N;
#pragma unroll
  for (int k = tid; k < N; k += T) {
    const float2 X = unpack<DT>(load_maybe<COHERENT>(xrow + k));
    const float2 H = unpack<DT>(h0[k]);
    float2 s0 = (k == 0) ? make_float2(H.x * X.x, H.y * X.y) : cmul(H, X);
    float2 s1 = make_float2(0.f, 0.f), s2 = s1, s3 = s1;
    const int t = k / TW;
    const int b = k - t * TW;
    const float2* src = ypart + ((int64_t)base + (int64_t)t * nch) * TW + b;
    int j = 0;
    for (; j + 4 <= nch; j += 4) {
      const float2 a0 = load_maybe<COHERENT>(src + (int64_t)(j + 0) * TW);
      const float2 a1 = load_maybe<COHERENT>(src + (int64_t)(j + 1) * TW);
      const float2 a2 = load_maybe<COHERENT>(src + (int64_t)(j + 2) * TW);
      const float2 a3 = load_maybe<COHERENT>(src + (int64_t)(j + 3) * TW);
      s0 = cadd(s0, a0); s1 = cadd(s1, a1); s2 = cadd(s2, a2); s3 = cadd(s3, a3);
    }
    for (; j < nch; ++j) s0 = cadd(s0, load_maybe<COHERENT>(src + (int64_t)j * TW));
    const float2 v = cadd(cadd(s0, s1), cadd(s2, s3));
    Y[k] = ACC ? cadd(Y[k], v) : v;   // ACC: add to the bus sum (each thread owns its k)
  }
}

// Spectra of NC (1 or 2) channels into Y[0 .. NC) (LDS), as channel_spectrum
// computes each (the same sums in the same order), from their completion
// descriptors. The delay-line, bank and first partial-row loads of all the
// channels are issued before any of them is used, so the completion waits
// for memory once. COHERENT as in channel_spectrum. No barrier at the end.
template <int L, int T, int DT, bool COHERENT, int NC>
__device__ __forceinline__ void desc_spectra(const float2* __restrict__ ypart, int TW,
                                             const typename Store<DT>::T* __restrict__ bank,
                                             const typename Store<DT>::T* __restrict__ fdl, const FinDesc* d,
                                             float2* const (&Y)[NC], int tid) {
  using ST = typename Store<DT>::T;
  constexpr int N = 2 * L;
  const ST* xrow[NC];
  const ST* h0[NC];
  const float2* rows[NC];
  int nch[NC];
#pragma unroll
  for (int g = 0; g < NC; ++g) {
    xrow[g] = fdl + d[g].x;
    h0[g] = bank + d[g].h;
    rows[g] = ypart + (int64_t)d[g].rows * TW;
    nch[g] = d[g].nch;
  }
#pragma unroll
  for (int k = tid; k < N; k += T) {
    const int t = k / TW;
    const int b = k - t * TW;
    float2 X[NC], H[NC], a0[NC];
    const float2* src[NC];
#pragma unroll
    for (int g = 0; g < NC; ++g) {
      X[g] = unpack<DT>(load_maybe<COHERENT>(xrow[g] + k));
      H[g] = unpack<DT>(h0[g][k]);
      src[g] = rows[g] + (int64_t)t * nch[g] * TW + b;
      a0[g] = nch[g] > 0 ? load_maybe<COHERENT>(src[g]) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int g = 0; g < NC; ++g) {
      float2 s0 = (k == 0) ? make_float2(H[g].x * X[g].x, H[g].y * X[g].y) : cmul(H[g], X[g]);
      float2 s1 = make_float2(0.f, 0.f), s2 = s1, s3 = s1;
      const int n = nch[g];
      int j = 0;
      if (n >= 4) {
        s0 = cadd(s0, a0[g]);
        s1 = cadd(s1, load_maybe<COHERENT>(src[g] + (int64_t)1 * TW));
        s2 = cadd(s2, load_maybe<COHERENT>(src[g] + (int64_t)2 * TW));
        s3 = cadd(s3, load_maybe<COHERENT>(src[g] + (int64_t)3 * TW));
        for (j = 4; j + 4 <= n; j += 4) {
          const float2 b0 = load_maybe<COHERENT>(src[g] + (int64_t)(j + 0) * TW);
          const float2 b1 = load_maybe<COHERENT>(src[g] + (int64_t)(j + 1) * TW);
          const float2 b2 = load_maybe<COHERENT>(src[g] + (int64_t)(j + 2) * TW);
          const float2 b3 = load_maybe<COHERENT>(src[g] + (int64_t)(j + 3) * TW);
          s0 = cadd(s0, b0); s1 = cadd(s1, b1); s2 = cadd(s2, b2); s3 = cadd(s3, b3);
        }
      }
      for (; j < n; ++j) s0 = cadd(s0, j == 0 ? a0[g] : load_maybe<COHERENT>(src[g] + (int64_t)j * TW));
      Y[g][k] = cadd(cadd(s0, s1), cadd(s2, s3));
    }
  }
}

// Complete channel c (completion descriptor d): spectrum, inverse transform
// and overlap-add.
template <int L, int T, int DT, bool COHERENT>
__device__ __forceinline__ void channel_final(const float2* __restrict__ ypart, int TW,
                                              const typename Store<DT>::T* __restrict__ bank,
                                              const typename Store<DT>::T* __restrict__ fdl, const FinDesc* d, int c,
                                              float2* Y, float2* bufA, float2* bufB, const float2* twl,
                                              float* __restrict__ ola, float* __restrict__ out, int64_t out_stride,
                                              int tid) {
  float* st = ola + (int64_t)c * 3 * L;
  float old[(4 * L + T - 1) / T];
  ola_prefetch<L, T>(st, old, tid);    // in flight together with the spectrum's loads
  float2* const Ys[1] = {Y};
  desc_spectra<L, T, DT, COHERENT, 1>(ypart, TW, bank, fdl, d, Ys, tid);
  __syncthreads();
  inverse_ola<L, T>(Y, bufA, bufB, twl, old, st, out + (int64_t)c * out_stride, tid);
}

// Complete channels c0 and c1 together: both spectra, one 4L-point complex
// inverse transform of Y0 + i Y1 (both outputs are real, so the real part is
// channel c0's block and the imaginary part channel c1's), overlap-add of both.
// Ya, Yb: 2L each; F0, F1: 4L each (LDS). twl holds exp(-2 pi i t / 4L).
// d: the completion descriptors of c0 and c1.
template <int L, int T, int DT, bool COHERENT>
__device__ __forceinline__ void pair_final(const float2* __restrict__ ypart, int TW,
                                           const typename Store<DT>::T* __restrict__ bank,
                                           const typename Store<DT>::T* __restrict__ fdl, const FinDesc* d, int c0,
                                           int c1, float2* Ya, float2* Yb, float2* F0, float2* F1, const float2* twl,
                                           float* __restrict__ ola, float* __restrict__ out, int64_t out_stride,
                                           int tid) {
  constexpr int N = 2 * L;
  constexpr int NPT = (4 * L + T - 1) / T;
  float* st0 = ola + (int64_t)c0 * 3 * L;
  float* st1 = ola + (int64_t)c1 * 3 * L;
  float old0[NPT], old1[NPT];
  ola_prefetch<L, T>(st0, old0, tid);
  ola_prefetch<L, T>(st1, old1, tid);
  float2* const Ys[2] = {Ya, Yb};
  desc_spectra<L, T, DT, COHERENT, 2>(ypart, TW, bank, fdl, d, Ys, tid);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int k = tid + j * T;
    if (k < 4 * L) {
      float2 y0, y1;
      if (k == 0) {
        y0 = make_float2(Ya[0].x, 0.f);
        y1 = make_float2(Yb[0].x, 0.f);
      } else if (k == N) {
        y0 = make_float2(Ya[0].y, 0.f);
        y1 = make_float2(Yb[0].y, 0.f);
      } else if (k < N) {
        y0 = Ya[k];
        y1 = Yb[k];
      } else {
        y0 = fft::cconj(Ya[4 * L - k]);
        y1 = fft::cconj(Yb[4 * L - k]);
      }
      F0[k] = make_float2(y0.x - y1.y, -(y0.y + y1.x));
    }
  }
  __syncthreads();
  const float2* R = fft::fft_nat<4 * L, T>(F0, F1, twl, tid);
  constexpr float scale = 1.0f / (float)(4 * L);
  float* o0 = out + (int64_t)c0 * out_stride;
  float* o1 = out + (int64_t)c1 * out_stride;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int n = tid + j * T;
    if (n < 4 * L) {
      const float2 z = R[n];
      const float v0 = z.x * scale, v1 = -z.y * scale;
      if (n < L) {
        o0[n] = old0[j] + v0;
        o1[n] = old1[j] + v1;
      } else if (n < 3 * L) {
        st0[n - L] = old0[j] + v0;
        st1[n - L] = old1[j] + v1;
      } else {
        st0[n - L] = v0;
        st1[n - L] = v1;
      }
    }
  }
}

// ---------------------------------------------------------------- fused per-block kernel

// Work items: kind 1 = new spectrum of one input (placed first), kind 0 = MAC
// over a partition chunk of up to G channels sharing an input. Every channel
// waits for needed[c] arrivals (its MAC items plus its input's spectrum item);
// the item that arrives last completes the channel. No item ever waits. An
// item counts its arrivals for all its channels at once, counts itself done
// (the last item advances the call counter, which only the next launch reads)
// and then completes its channels, two at a time with one complex transform.
template <int L, int V, int G, int NW, int DT>
__global__ __launch_bounds__(64 * NW) void k_block(BlockArgs A) {
  using ST = typename Store<DT>::T;
  constexpr int N = 2 * L;
  constexpr int T = 64 * NW;
  constexpr int TW = 64 * V;
  // the MAC reduction buffer doubles as the pair completion's 4L-point buffers
  constexpr int RED = NW * G * TW;
  constexpr int POOL = RED > 4 * N ? RED : 4 * N;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  __shared__ float2 ybuf[N];
  __shared__ float2 pool[POOL];
  __shared__ int cand[4];
  __shared__ FinDesc fin[4];   // completion descriptors of cand
  __shared__ int won[4];
  __shared__ int nwon;
  auto red = reinterpret_cast<float2 (*)[G][TW]>(pool);
  const DevPlan& P = A.P;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const uint64_t cnt = *A.counter;
  const int p = (int)(cnt & 1u);
  const ST* bank = static_cast<const ST*>(A.bank);
  ST* fdl = static_cast<ST*>(A.fdl);
  const bool inl = A.inverse_inline != 0;
  // The FFT tables are loaded up front (made visible by the first barrier), so
  // neither spectrum items nor channel completions wait for them later.
  load_tables<L, T>(P, twl, winl, tid);

  // Count one arrival for the channel group cand[0 .. n) (channels and their
  // completion descriptors fin[0 .. n) set by the caller; they go through LDS
  // so that the work item stays in registers) and, if last, the item itself. A group (the channels of an input that share
  // work items) has one counter, kept under its first channel: every item
  // publishes all the group's data before it counts, so the arrival that
  // completes the counter completes every channel of the group, and the
  // group is always finished the same way (two channels per complex
  // transform), whichever workgroups arrive last.
  auto arrive = [&](int n, bool last_of_item) {
    if (tid == 0) {
      const int c0 = cand[0];
      // The group's quota and both counters are in flight together (one
      // round trip). Increments rather than additions: the compiler issues
      // them as written, without the wave-level aggregation it builds around
      // an addition, whose wait would put the second counter behind the first.
      const int need = A.needed[c0];
      const int a = (int)atomicInc(reinterpret_cast<unsigned int*>(&A.arrive[c0]), 0xffffffffu);
      const int d = last_of_item ? (int)atomicInc(reinterpret_cast<unsigned int*>(A.done), 0xffffffffu) : -1;
      int k = 0;
      if (a == need - 1) {
        for (int j = 0; j < n; ++j) won[j] = cand[j];
        k = n;
      }
      // (won[j] keeps fin[j]: the winner completes cand in order)
      nwon = k;
      if (d == A.n_items - 1) {
        // every item has started, so every workgroup has read the call count
        *A.done = 0;
        *A.counter = cnt + 1u;
      }
    }
    __syncthreads();
    const int k = nwon;
    for (int j = 0; j < k; j += 2) {
      if (j + 1 < k)
        pair_final<L, T, DT, true>(A.ypart, TW, bank, fdl, fin + j, won[j], won[j + 1], bufA, bufB, pool,
                                   pool + 2 * N, twl, A.ola, A.out, A.out_stride, tid);
      else
        channel_final<L, T, DT, true>(A.ypart, TW, bank, fdl, fin + j, won[j], ybuf, bufA, bufB, twl, A.ola,
                                      A.out, A.out_stride, tid);
      __syncthreads();
    }
    if (tid < k) {
      const int c = won[tid];
      if (tid == 0) A.arrive[c] = 0;
      if (A.copy_sel) A.sel_store[c] = A.sel[c];
    }
    __syncthreads();
  };

  for (int idx = blockIdx.x; idx < A.n_items; idx += gridDim.x) {
    const WorkItem it = A.items[idx];
    if (it.kind == 1) {
      if (inl) {
        input_spectrum<L, T, DT, true>(P, A.in, A.in_stride, A.hist, fdl, it.input, p, cnt, twl, winl, bufA, bufB,
                                       tid);
        wait_memory();
        __syncthreads();
        // the input's channels in groups of G, as the work items group them
        const int j1 = P.in_ch_ptr[it.input + 1];
        for (int j = P.in_ch_ptr[it.input]; j < j1; j += G) {
          const int n = min(G, j1 - j);
          if (tid < n) {
            const int c = P.in_ch[j + tid];
            cand[tid] = c;
            fin[tid] = lookup_desc<L>(P, A.sel, c, p, cnt);
          }
          __syncthreads();
          arrive(n, j + G >= j1);
        }
      } else {
        input_spectrum<L, T, DT, false>(P, A.in, A.in_stride, A.hist, fdl, it.input, p, cnt, twl, winl, bufA, bufB,
                                        tid);
        __syncthreads();
        continue;
      }
    } else {
      float2 acc[G][V];
      // two partitions in flight per wave keep the streaming loop well within
      // the register budget
      mac_item<V, G, NW, DT, 2>(P, it, bank, fdl, A.sel, p, cnt, lane, w, acc, inl ? fin : nullptr);
      if (inl) {
        write_partials<V, G, NW, true>(it, acc, red, A.ypart, lane, w, tid);
        wait_memory();
        __syncthreads();
        if (tid == 0) {
#pragma unroll
          for (int g = 0; g < G; ++g) cand[g] = it.ch[g];
        }
        arrive(it.n_ch, true);
      } else {
        write_partials<V, G, NW, false>(it, acc, red, A.ypart, lane, w, tid);
        __syncthreads();
        continue;
      }
    }
  }
}

// ---------------------------------------------------------------- batched blocks

// Batches of n consecutive blocks (calls cnt .. cnt+n-1) in three launches:
// all input spectra, one MAC launch that writes partial spectrum rows per
// (block, channel), and one launch that transforms back and overlap-adds the
// outputs' windows. The delay line holds M_i + (n_max-1)/2 spectra per
// parity, so a batch's new spectra never replace ones that its own blocks
// still read.

// Blocks per workgroup in the batched transform kernels (their twiddle and
// window tables are loaded once per workgroup).
constexpr int kBatchBlocksPerWg = 4;

// Spectra of input i for blocks j of the batch (block j's 2L samples are the
// previous call's L samples, from the history for j = 0, then its own L).
template <int L, int DT>
__global__ __launch_bounds__(256) void k_batch_spectra(DevPlan P, const float* __restrict__ in, int64_t in_stride,
                                                       const float* __restrict__ hist,
                                                       typename Store<DT>::T* __restrict__ fdl,
                                                       const uint64_t* __restrict__ counter, int n_blocks,
                                                       int32_t* __restrict__ defer_count, int bpw) {
  constexpr int N = 2 * L;
  constexpr int T = 256;
  // the matrix-core MAC of this call appends to an empty deferred list
  if (defer_count && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *defer_count = 0;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int i = blockIdx.y, tid = threadIdx.x;
  const uint64_t cnt0 = *counter;
  const int Mi = P.in_M[i];
  load_tables<L, T>(P, twl, winl, tid);
  __syncthreads();
  // bpw consecutive blocks per workgroup (tables loaded once)
  for (int u = 0; u < bpw; ++u) {
    const int j = blockIdx.x * bpw + u;
    if (j >= n_blocks) break;
    const uint64_t cnt = cnt0 + (uint64_t)j;
    const int p = (int)(cnt & 1u);
    const float* xin = in + (int64_t)i * in_stride + (int64_t)j * L;
    const float* hold = (j == 0) ? hist + ((size_t)(p ^ 1) * P.I + i) * L : xin - L;
    for (int n = tid; n < L; n += T) {
      const int t0 = 2 * n, t1 = 2 * n + 1;
      const float s0 = (t0 < L) ? hold[t0] : xin[t0 - L];
      const float s1 = (t1 < L) ? hold[t1] : xin[t1 - L];
      bufA[n] = make_float2(winl[t0] * s0, winl[t1] * s1);
      bufA[n + L] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    const float2* Z = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
    typename Store<DT>::T* dst = fdl + P.in_fdl_off[i] + ((int64_t)p * Mi + ring_slot(cnt, Mi)) * N;
    for (int k = tid; k < N; k += T) dst[k] = pack<DT>(fft::real_fwd_post<N>(Z, k, twl));
    __syncthreads();
  }
}

// Spectral MAC of a batch (eq. 8), blocked in time. Blocks of one parity
// read the same delay-line ring: block l + 2 at partition m + 1 reads the
// spectrum that block l reads at partition m, and blocks that use the same IR
// slot read the same partition spectra. An item covers (up to G channels of
// one input, a bin tile, partitions [m0, m1)) for up to TB blocks of one
// parity; each wave owns 64 V bins of the tile and walks the partitions in
// order, keeping the TB delay-line rows of the current partition in a
// circular register buffer (one new row per partition) and loading each
// partition spectrum once per distinct slot. Every (block, channel) gets one
// partial spectrum row per partition chunk.

// Slot pattern of an item's blocks, per channel: one slot for all blocks,
// two slots alternating with the block index, two slots in any order (each
// block picks its slot's spectrum with a select), any assignment of up to two
// slots per pass (blocks of further slots take further passes), or every
// block its own slot's spectrum in one pass (the delay-line window is read
// once however many slots the blocks use; for one-channel items small enough
// to hold a partition row per block in registers).
enum TmacPattern { kOneSlot = 1, kAlternating = 2, kSelect = 3, kTwoSlots = 4, kPerBlock = 5 };

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Number of distinct values among n uniform slots.
template <int n>
__device__ __forceinline__ int distinct_slots(const int (&sl)[n]) {
  int d = 0;
#pragma unroll
  for (int b = 0; b < n; ++b) {
    bool seen = false;
#pragma unroll
    for (int a = 0; a < b; ++a) seen = seen || (sl[a] == sl[b]);
    d += seen ? 0 : 1;
  }
  return d;
}

// f(integral_constant<int, i>) for i = 0 .. n-1, unrolled at compile time.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int n, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, n>{});
}

template <int L, int V, int G, int TB, int DT>
__global__ __launch_bounds__(256) void k_tmac(BatchArgs B) {
  using ST = typename Store<DT>::T;
  constexpr int N = 2 * L;
  const int TW = B.tile_width;   // 64 V bins per wave, blockDim.x / 64 waves
  constexpr int PD = (TB == 16 && DT != 0) ? 8 : 4;   // partitions loaded ahead
  const DevPlan& P = B.P;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const uint64_t cnt0 = *B.counter;
  const int n = B.n_blocks;
  const int groups = ((n + 1) / 2 + TB - 1) / TB;     // time groups per parity class
  // Workgroup w runs on XCD w mod 8. The time groups of one (item, parity
  // class) read the same partition spectra, so they get indices 8 apart: the
  // same XCD (and L2), dispatched one after the other.
  const int pairs = 2 * B.n_mac;                      // (item, class)
  const int lanes8 = (pairs + 7) / 8;
  const int total = 8 * lanes8 * groups;
  const ST* bank = static_cast<const ST*>(B.bank);
  const ST* fdl = static_cast<const ST*>(B.fdl);
  // from_list: the units the matrix-core MAC deferred (index space as below)
  const int n_units = B.from_list ? *B.defer_count : total;
  for (int u = blockIdx.x; u < n_units; u += gridDim.x) {
    const int idx = B.from_list ? B.defer_list[u] : u;
    const int x = idx & 7, y = idx >> 3;
    const int gi = y % groups;
    const int pr = x + 8 * (y / groups);               // (item, class) pair
    if (pr >= pairs) continue;
    const int cls = pr & 1;
    const WorkItem it = B.items[pr >> 1];
    const int j0 = cls + 2 * TB * gi;                  // first block of the group
    if (j0 >= n) continue;
    const int nb = min(TB, (n - j0 + 1) / 2);            // blocks j0, j0 + 2, ...
    const int i = uniform(it.input);
    const int n_ch = uniform(it.n_ch);
    const int m0 = uniform(it.m0), m1 = uniform(it.m1);
    const int Mi = uniform(P.in_M[i]);
    const uint64_t c0 = cnt0 + (uint64_t)j0;
    const int p = (int)(c0 & 1u);
    const int q0 = ring_slot(c0, Mi);
    const uint32_t kb = (uint32_t)(it.tile * TW + w * 64 * V + lane * V);
    const ST* xbase = fdl + P.in_fdl_off[i] + (int64_t)p * Mi * N;
    int Mc[G], McL[G], ch[G];
    const ST* hch[G];
    int slot[G][TB];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ch[g] = uniform(g < n_ch ? it.ch[g] : it.ch[0]);
      McL[g] = uniform(P.ch_M[ch[g]]);
      Mc[g] = g < n_ch ? McL[g] : 0;
      hch[g] = bank + P.ch_bank_off[ch[g]];
    }
    // slots of every block (loads issued together; block indices past the
    // group repeat its last block)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) slot[g][b] = B.sel[(int64_t)(j0 + 2 * min(b, nb - 1)) * B.sel_stride + ch[g]];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int sv = uniform(slot[g][b]);
        slot[g][b] = sv < 0 ? 0 : (sv >= P.K ? P.K - 1 : sv);
      }
    bool one = true, alt = true, two_slots = true;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      int other = slot[g][0];
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        one = one && (slot[g][b] == slot[g][0]);
        alt = alt && (slot[g][b] == slot[g][b & 1]);
        if (slot[g][b] != slot[g][0]) other = slot[g][b];
      }
#pragma unroll
      for (int b = 0; b < TB; ++b) two_slots = two_slots && (slot[g][b] == slot[g][0] || slot[g][b] == other);
    }
    float2 acc[G][TB][V];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[g][b][v] = make_float2(0.f, 0.f);

    int mlast[G];
#pragma unroll
    for (int g = 0; g < G; ++g) mlast[g] = min(m1, McL[g]) - 1;

    // The partition loop for one slot pattern. X: circular buffer of the TB
    // delay-line rows of the current partition (block b at partition m0 + t
    // is in X[(b - t) mod TB]); Hq / Xq: ring of PD partitions' spectra and
    // next rows, loaded ahead of use.
    const bool dcw = (it.tile == 0 && w == 0);   // this wave holds the packed DC / Nyquist bin
    const bool dc_lane = dcw && lane == 0;
    // hr[g][d]: partition rows of slot set d of channel g (d < 2; for
    // kPerBlock d = block, d < TB)
    auto run = [&](auto patc, auto dcwc, const auto& hr, const uint32_t (&sel1)[G], const uint32_t (&take)[G]) {
      constexpr int PAT = decltype(patc)::value;
      constexpr bool DCW = decltype(dcwc)::value;
      constexpr int ND = (PAT == kOneSlot) ? 1 : (PAT == kPerBlock ? TB : 2);
      // partitions loaded ahead (a row per block in flight for kPerBlock)
      constexpr int PDP = (PAT == kPerBlock) ? 2 : PD;
      // f32 storage: values as float2, four FMAs per complex product. 16-bit
      // storage: raw words (Re in the low half, Im in the high half) and two
      // packed dot products with FP32 accumulation per complex product:
      // Re += (h.re, -h.im).(x.re, x.im), Im += (h.re, h.im).(x.im, x.re); every
      // delay-line word in the window is kept beside its half-swapped copy.
      using HW = std::conditional_t<DT == 0, float2, uint32_t>;   // loaded value
      using XW = std::conditional_t<DT == 0, float2, uint2>;      // window entry
      auto load_raw = [&](const ST* p, HW (&o)[V]) {
        if constexpr (DT == 0) {
          load_vec<0, V>(p, o);
        } else if constexpr (V == 1) {
          o[0] = *reinterpret_cast<const uint32_t*>(p);
        } else {
          const uint2 t = *reinterpret_cast<const uint2*>(p);
          o[0] = t.x;
          o[1] = t.y;
        }
      };
      // window entry of a loaded delay-line value (v: bin within the lane)
      auto entry = [&](const HW& w, int v) -> XW {
        if constexpr (DT == 0) {
          return w;
        } else {
          // on the DC lane the products are component-wise: no swap
          const bool keep = DCW && v == 0 && dc_lane;
          return make_uint2(w, keep ? w : __builtin_amdgcn_alignbit(w, w, 16));
        }
      };
      XW X[TB][V];
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        int r = q0 + min(b, nb - 1) - m0;
        r = r < 0 ? r + Mi : (r >= Mi ? r - Mi : r);
        HW w[V];
        load_raw(xbase + (uint32_t)r * N + kb, w);
#pragma unroll
        for (int v = 0; v < V; ++v) X[b][v] = entry(w[v], v);
      }
      HW Hq[PDP][G][ND][V];
      HW Xq[PDP][V];
      auto load_h = [&](HW (&Hs)[G][ND][V], int mm) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int mr = min(mm, mlast[g]);
#pragma unroll
          for (int d = 0; d < ND; ++d) load_raw(hr[g][d] + (uint32_t)mr * N + kb, Hs[g][d]);
        }
      };
      auto load_x = [&](HW (&Xs)[V], int mm) {   // delay-line row of partition mm for block 0
        int r = q0 - min(mm, m1 - 1);
        r = r < 0 ? r + Mi : r;
        load_raw(xbase + (uint32_t)r * N + kb, Xs);
      };
      // acc += h x for one (channel, block, bin); hp: the prepared h terms
      auto mac = [&](float2& a, const auto& hp, const XW& x) {
        if constexpr (DT == 0) {
          a.x = fmaf(hp[0], x.x, a.x);
          a.x = fmaf(hp[1], x.y, a.x);
          a.y = fmaf(hp[2], x.y, a.y);
          a.y = fmaf(hp[3], x.x, a.y);
        } else if constexpr (DT == 1) {
          a.x = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, hp[0]), __builtin_bit_cast(bf16x2_t, x.x),
                                                a.x, false);
          a.y = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, hp[1]), __builtin_bit_cast(bf16x2_t, x.y),
                                                a.y, false);
        } else {
          a.x = __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, hp[0]), __builtin_bit_cast(f16x2_t, x.x), a.x, false);
          a.y = __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, hp[1]), __builtin_bit_cast(f16x2_t, x.y), a.y, false);
        }
      };
      // partition mm = m0 + t (t = step index): accumulate, using X rows at
      // circular offset t
      auto step = [&](const HW (&Hs)[G][ND][V], int mm, auto tc) {
        constexpr int T0 = decltype(tc)::value;   // t mod TB
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (mm < Mc[g]) {
#pragma unroll
            for (int d = 0; d < (PAT == kTwoSlots ? 1 : ND); ++d) {
#pragma unroll
              for (int v = 0; v < V; ++v) {
                // the h terms of the product; on the DC lane (packed Re X(0),
                // Re X(2L)) the product is component-wise
                const HW h = Hs[g][d][v];
                std::conditional_t<DT == 0, float[4], uint32_t[2]> hp;
                if constexpr (DT == 0) {
                  hp[0] = h.x; hp[1] = -h.y; hp[2] = h.x; hp[3] = h.y;
                  if (DCW && v == 0) {
                    hp[1] = dc_lane ? 0.f : -h.y;
                    hp[2] = dc_lane ? h.y : h.x;
                    hp[3] = dc_lane ? 0.f : h.y;
                  }
                } else {
                  hp[0] = h ^ 0x80000000u;
                  hp[1] = h;
                  if (DCW && v == 0) {
                    hp[0] = dc_lane ? (h & 0xffffu) : hp[0];
                    hp[1] = dc_lane ? (h & 0xffff0000u) : hp[1];
                  }
                }
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                  bool use;
                  if constexpr (PAT == kOneSlot) use = true;
                  else if constexpr (PAT == kAlternating) use = ((b & 1) == d);
                  else if constexpr (PAT == kPerBlock) use = (b == d);
                  else use = true;
                  if (use) {
                    const XW& x = X[(b - T0 + TB) % TB][v];
                    if constexpr (PAT == kTwoSlots) {
                      // slot 1 or slot 0 for this block: uniform select
                      const bool s1 = ((sel1[g] >> b) & 1u) != 0u;
                      decltype(hp) hq;
                      const HW h1 = Hs[g][1][v];
                      if constexpr (DT == 0) {
                        const float a0 = s1 ? h1.x : h.x, a1 = s1 ? h1.y : h.y;
                        hq[0] = a0; hq[1] = -a1; hq[2] = a0; hq[3] = a1;
                        if (DCW && v == 0) {
                          hq[1] = dc_lane ? 0.f : -a1;
                          hq[2] = dc_lane ? a1 : a0;
                          hq[3] = dc_lane ? 0.f : a1;
                        }
                      } else {
                        const uint32_t w = s1 ? h1 : h;
                        hq[0] = w ^ 0x80000000u;
                        hq[1] = w;
                        if (DCW && v == 0) {
                          hq[0] = dc_lane ? (w & 0xffffu) : hq[0];
                          hq[1] = dc_lane ? (w & 0xffff0000u) : hq[1];
                        }
                      }
                      mac(acc[g][b][v], hq, x);
                    } else if constexpr (PAT == kSelect) {
                      // uniform per (g, b): slot d of this pass, or nothing
                      const bool on = ((take[g] >> b) & 1u) && ((((sel1[g] >> b) & 1u) != 0u) == (d == 1));
                      if (on) mac(acc[g][b][v], hp, x);
                    } else {
                      mac(acc[g][b][v], hp, x);
                    }
                  }
                }
              }
            }
          }
        }
      };
#pragma unroll
      for (int st = 0; st < PDP; ++st) {
        load_h(Hq[st], m0 + st);
        load_x(Xq[st], m0 + st + 1);
      }
      // one partition: accumulate, then load the spectra PD partitions ahead
      // and move the prefetched row of partition mm + 1 (block 0) to where
      // block TB - 1's row of partition mm was
      auto advance = [&](int mm, auto tc) {
        constexpr int t = decltype(tc)::value;
        step(Hq[t % PDP], mm, tc);
        load_h(Hq[t % PDP], mm + PDP);
#pragma unroll
        for (int v = 0; v < V; ++v) X[(TB - 1 - t) % TB][v] = entry(Xq[t % PDP][v], v);
        load_x(Xq[t % PDP], mm + 1 + PDP);
      };
      int mb = m0;
      for (; mb + TB <= m1; mb += TB) static_for<TB>([&](auto tc) { advance(mb + decltype(tc)::value, tc); });
      static_for<TB>([&](auto tc) {
        if (mb + decltype(tc)::value < m1) advance(mb + decltype(tc)::value, tc);
      });
    };

    if (one || alt) {
      const ST* hr[G][2];
      uint32_t none[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        none[g] = 0u;
        hr[g][0] = hch[g] + (int64_t)slot[g][0] * McL[g] * N;
        hr[g][1] = hch[g] + (int64_t)slot[g][1] * McL[g] * N;
      }
      if (one) {
        if (dcw) run(std::integral_constant<int, kOneSlot>{}, std::true_type{}, hr, none, none);
        else run(std::integral_constant<int, kOneSlot>{}, std::false_type{}, hr, none, none);
      } else {
        if (dcw) run(std::integral_constant<int, kAlternating>{}, std::true_type{}, hr, none, none);
        else run(std::integral_constant<int, kAlternating>{}, std::false_type{}, hr, none, none);
      }
    } else if (two_slots) {
      const ST* hr[G][2];
      uint32_t sel1[G], none[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        none[g] = 0u;
        const int s0 = slot[g][0];
        int s1v = s0;
        uint32_t m1b = 0u;
#pragma unroll
        for (int b = 0; b < TB; ++b)
          if (slot[g][b] != s0) { s1v = slot[g][b]; m1b |= 1u << b; }
        sel1[g] = m1b;
        hr[g][0] = hch[g] + (int64_t)s0 * McL[g] * N;
        hr[g][1] = hch[g] + (int64_t)s1v * McL[g] * N;
      }
      if (dcw) run(std::integral_constant<int, kTwoSlots>{}, std::true_type{}, hr, sel1, none);
      else run(std::integral_constant<int, kTwoSlots>{}, std::false_type{}, hr, sel1, none);
    } else if (G == 1 && TB * V <= 16 && 2 * distinct_slots(slot[0]) > TB) {
      // more distinct slots than half the blocks: every block its own row,
      // one pass (a pass per two slots would read the delay-line window
      // more than TB / 4 times; with fewer slots the passes issue fewer
      // loads). One-channel items only: the row registers would cost the
      // two-channel forms occupancy on every pattern.
      const ST* hr[G][TB];
      uint32_t none[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        none[g] = 0u;
#pragma unroll
        for (int b = 0; b < TB; ++b) hr[g][b] = hch[g] + (int64_t)slot[g][b] * McL[g] * N;
      }
      if constexpr (G == 1 && TB * V <= 16) {
        if (dcw) run(std::integral_constant<int, kPerBlock>{}, std::true_type{}, hr, none, none);
        else run(std::integral_constant<int, kPerBlock>{}, std::false_type{}, hr, none, none);
      }
    } else {
      // passes of up to two slots per channel
      uint32_t todo[G];
#pragma unroll
      for (int g = 0; g < G; ++g) todo[g] = (g < n_ch) ? ((1u << nb) - 1u) : 0u;
      while (true) {
        bool any = false;
#pragma unroll
        for (int g = 0; g < G; ++g) any = any || (todo[g] != 0u);
        if (!any) break;
        const ST* hr[G][2];
        uint32_t sel1[G], take[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          uint32_t mk[2] = {0u, 0u};
          int sl[2] = {0, 0};
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            if (todo[g] != 0u) {
              const int first = __builtin_ctz(todo[g]);
              int sv = 0;
#pragma unroll
              for (int b = 0; b < TB; ++b)
                if (b == first) sv = slot[g][b];
#pragma unroll
              for (int b = 0; b < TB; ++b)
                if (((todo[g] >> b) & 1u) && slot[g][b] == sv) mk[d] |= 1u << b;
              todo[g] &= ~mk[d];
              sl[d] = sv;
            } else {
              sl[d] = sl[0];
            }
          }
          sel1[g] = mk[1];
          take[g] = mk[0] | mk[1];
          hr[g][0] = hch[g] + (int64_t)sl[0] * McL[g] * N;
          hr[g][1] = hch[g] + (int64_t)sl[1] * McL[g] * N;
        }
        if (dcw) run(std::integral_constant<int, kSelect>{}, std::true_type{}, hr, sel1, take);
        else run(std::integral_constant<int, kSelect>{}, std::false_type{}, hr, sel1, take);
      }
    }
    // partial rows: block j0 + 2b, channel g
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g < n_ch) {
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          if (b < nb) {
            float2* dst = B.ypart + ((int64_t)(j0 + 2 * b) * B.n_rows + it.row[g]) * TW + w * 64 * V + lane * V;
            if constexpr (V == 1) {
              dst[0] = acc[g][b][0];
            } else {
#pragma unroll
              for (int v = 0; v < V; v += 2)
                *reinterpret_cast<float4*>(dst + v) =
                    make_float4(acc[g][b][v].x, acc[g][b][v].y, acc[g][b][v + 1].x, acc[g][b][v + 1].y);
            }
          }
        }
      }
    }
  }
}

// Matrix-core form of the time-blocked MAC (eq. 8) for f32 spectra. For one
// bin, a time group of 16 blocks of one parity class and the (up to) two
// channels of one input, the products form outer products of delay-line and
// partition spectra. One 4x4x1 MFMA with 16 blocks takes 16 bins: in each
// block, rows are (Re, Im) of X for two blocks t and t + 8 and columns (Re,
// Im) of H for the two channels; its 4x4 accumulator collects the four real
// products Re X Re H, Im X Re H, Re X Im H, Im X Im H of every (block,
// channel), combined into Re Y and Im Y once after the last partition. Pair q
// (blocks q and q + 8) at partition m + 1 needs the delay-line values that
// pair q - 1 used at m, so each lane keeps a circular window of 8 values per
// bin that moves down one pair per partition; only pair 0 is loaded afresh.
// Even and odd pairs may take different slots (a stream that switches every
// block alternates two slots in a parity class); other slot patterns run
// passes in which the blocks of other slots are masked out of the A operand.
// A wave covers 16 bins; its operands are fetched PG partitions ahead with
// 16-byte loads and passed through LDS (see the staging comment).
template <int L, int NP, int R, int PG, int NWV, int DT>
__global__ __launch_bounds__(64 * NWV) void k_tmfma(BatchArgs B) {
  static_assert(DT == 0, "matrix-core MAC: f32 spectra");
  static_assert(NP == 8 || NP == 16, "pairs per time group");
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int U = 1;                      // 16 bins per wave
  constexpr int TB = 2 * NP;                // blocks of one parity per time group
  constexpr int N = 2 * L;
  constexpr uint32_t RB = 8u * N;           // bytes per delay-line / partition row
  constexpr int LS = 4;                     // staging slots per wave
  constexpr int PER = std::lcm(std::lcm(R, LS), std::lcm(PG, 3));   // unroll period (static register indices)
  static_assert(R >= NP + 2 && PG >= 4, "window and load ring");
  // Staging: per step a wave needs two delay-line row pieces and four
  // partition-spectrum row pieces of 128 B (its 16 bins); 48 lanes fetch them
  // with one 16-byte load each (lanes 48..63 repeat delay-line pieces), the
  // wave writes them to its slot and every lane reads its own three operands
  // back. The bank and the delay line share one allocation, so every lane
  // addresses its piece with a 32-bit offset from the bank.
  __shared__ f4 stage[NWV][LS][64];
  const int TW = B.tile_width;              // 16 U bins per wave
  const DevPlan& P = B.P;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int b16 = lane >> 2;                // bin of the lane's MFMA block
  const int hh = (lane >> 1) & 1;           // A: block half (t = q + NP hh); B and C: channel
  const int comp = lane & 1;                // Re (0) or Im (1)
  const uint64_t cnt0 = *B.counter;
  const int n = B.n_blocks;
  const int groups = ((n + 1) / 2 + TB - 1) / TB;
  // same XCD-aware index space as k_tmac
  const int pairs = 2 * B.n_mac;
  const int lanes8 = (pairs + 7) / 8;
  const int total = 8 * lanes8 * groups;
  const char* bank = static_cast<const char*>(B.bank);
  const char* fdl = static_cast<const char*>(B.fdl);
  for (int idx = blockIdx.x; idx < total; idx += gridDim.x) {
    const int x = idx & 7, y = idx >> 3;
    const int gi = y % groups;
    const int pr = x + 8 * (y / groups);
    if (pr >= pairs) continue;
    const int cls = pr & 1;
    const WorkItem it = B.items[pr >> 1];
    const int j0 = cls + 2 * TB * gi;
    if (j0 >= n) continue;
    const int nb = min(TB, (n - j0 + 1) / 2);
    const int i = uniform(it.input);
    const int n_ch = uniform(it.n_ch);
    const int m0 = uniform(it.m0), m1 = uniform(it.m1);
    const int Mi = uniform(P.in_M[i]);
    const uint64_t c0 = cnt0 + (uint64_t)j0;
    const int p = (int)(c0 & 1u);
    const int qh = hh ? ring_slot(c0 + 2u * NP, Mi) : ring_slot(c0, Mi);   // ring slot of block NP hh
    const uint32_t f0 = 2u * (uint32_t)(it.tile * TW + w * 16 * U + b16) + (uint32_t)comp;   // float in a row
    const uint32_t lane_bytes = 4u * f0;
    // delay line of input i, parity p: Mi rows from a uniform base
    const char* xb = fdl + 8 * (P.in_fdl_off[i] + (int64_t)p * Mi * N);
    const uint32_t ring_bytes = (uint32_t)Mi * RB;
    int ch[2], McL[2], Mc[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      ch[g] = uniform(g < n_ch ? it.ch[g] : it.ch[0]);
      McL[g] = uniform(P.ch_M[ch[g]]);
      Mc[g] = g < n_ch ? McL[g] : 0;
    }
    int slot[2][TB];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) slot[g][b] = B.sel[(int64_t)(j0 + 2 * min(b, nb - 1)) * B.sel_stride + ch[g]];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int sv = uniform(slot[g][b]);
        slot[g][b] = sv < 0 ? 0 : (sv >= P.K ? P.K - 1 : sv);
      }
    // partition spectra: a uniform base at channel ch[0] and 32-bit byte
    // offsets (the channels of an item are in increasing bank order; the
    // host keeps the span below 2^32 and pads the bank with zero rows, which
    // the loads ahead of the last partition may reach)
    const char* hb = bank + 8 * P.ch_bank_off[ch[0]];
    const uint32_t ch_bytes = hh ? (uint32_t)(8 * (P.ch_bank_off[ch[1]] - P.ch_bank_off[ch[0]])) : 0u;
    const uint32_t slot_bytes = (uint32_t)(hh ? McL[1] : McL[0]) * RB;

    f4 acc[NP][U];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) acc[q][u] = f4{0.f, 0.f, 0.f, 0.f};

    auto ldf = [](const char* base, uint32_t off) { return *reinterpret_cast<const float*>(base + off); };
    // loader role of lanes 0..47: part 0, 1: delay-line row of block NP part;
    // part 2 + 2 d + g: partition spectrum of channel g, slot set d (even, odd)
    const int part = lane < 48 ? (lane >> 3) : ((lane >> 3) - 6), within = lane & 7;
    const uint32_t tile_bytes = (uint32_t)(it.tile * TW + w * 16) * 8u;
    const int gq = ring_slot(c0 + (part == 1 ? 2u * NP : 0u), Mi);   // loader's ring slot of block NP part
    const int lg = part & 1;                                     // loader's channel (H parts)
    const uint32_t lch_bytes = lg ? (uint32_t)(8 * (P.ch_bank_off[ch[1]] - P.ch_bank_off[ch[0]])) : 0u;
    const uint32_t lslot_bytes = (uint32_t)(lg ? McL[1] : McL[0]) * RB;
    f4* st = stage[w][0];
    const uint32_t xbo = (uint32_t)(xb - bank);    // delay line of (input, parity) from the bank base
    const float* stf = reinterpret_cast<const float*>(stage[w][0]);
    const int rx = 32 * hh + 2 * b16 + comp;   // reader's float in a slot: X; He at +64, Ho at +128

    // The partitions [m0, m1): even pairs take the spectra of slots se, odd
    // pairs those of so.
    auto run = [&](const int (&se)[2], const int (&so)[2]) {
      // Delay-line values by d = q - s (pair q at step s = mm - m0) in a
      // circular buffer of R registers: d = NP - 1 - s .. -s are in use at
      // step s, d = -s - 1 was read during step s - 1 and d = -s - 2 is read
      // from its staging slot during step s (two steps ahead of its use).
      float W[R];
      float Bq[3][2];
      f4 G[PG];                                // row-step k (d = -k, partition m0 + k) in G[k mod PG]
      const uint32_t he = ch_bytes + (uint32_t)(hh ? se[1] : se[0]) * slot_bytes + lane_bytes;
      const uint32_t ho = ch_bytes + (uint32_t)(hh ? so[1] : so[0]) * slot_bytes + lane_bytes;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        int r = (qh + q - m0) % Mi;
        r = r < 0 ? r + Mi : r;
        W[q] = ldf(xb, (uint32_t)r * RB + lane_bytes);
      }
      Bq[0][0] = ldf(hb, he + (uint32_t)m0 * RB);
      Bq[0][1] = ldf(hb, ho + (uint32_t)m0 * RB);
      // loader address of row-step k
      const int lslot = part < 2 ? 0 : ((part >> 1) == 1 ? (lg ? se[1] : se[0]) : (lg ? so[1] : so[0]));
      const uint32_t lh = lch_bytes + (uint32_t)lslot * lslot_bytes + tile_bytes + 16u * (uint32_t)within;
      // loader's running byte offset from the bank base for row-steps 1, 2,
      // ...: delay-line rows go down the ring (wrapping at lo), partition
      // rows up the bank
      const bool xl = part < 2;
      const uint32_t lo = xl ? xbo + tile_bytes + 16u * (uint32_t)within : 0u;   // ring row 0
      const uint32_t wrap = xl ? ring_bytes : 0u;
      const uint32_t dl = xl ? (uint32_t)(-(int32_t)RB) : RB;
      uint32_t goff;
      {
        int r = (gq - m0 - 1) % Mi;
        r = r < 0 ? r + Mi : r;
        goff = xl ? lo + (uint32_t)r * RB : (uint32_t)(hb - bank) + lh + (uint32_t)(m0 + 1) * RB;
      }
      auto gload = [&](f4& o) {                // the next row-step
        o = *reinterpret_cast<const f4*>(bank + goff);
        goff += dl;
        goff += goff < lo ? wrap : 0u;
      };
#pragma unroll
      for (int k = 1; k <= PG; ++k) gload(G[k % PG]);
      st[1 * 64 + lane] = G[1];
      st[2 * 64 + lane] = G[2];
      gload(G[1]);                             // row-step 1 + PG
      gload(G[2]);                             // row-step 2 + PG
      {
        const float* sl = stf + 1 * 256;       // row-step 1
        W[R - 1] = sl[rx];
        Bq[1][0] = sl[64 + rx];
        Bq[1][1] = sl[128 + rx];
      }
      auto advance = [&](auto sc) {
        constexpr int S = decltype(sc)::value;   // step index mod PER
        // a. operands of row-step s + 2 from its staging slot
        {
          const float* sl = stf + ((S + 2) % LS) * 256;
          W[(((-S - 2) % R) + R) % R] = sl[rx];
          Bq[(S + 2) % 3][0] = sl[64 + rx];
          Bq[(S + 2) % 3][1] = sl[128 + rx];
        }
        // b. the products of step s
#pragma unroll
        for (int q = 0; q < NP; ++q)
          acc[q][0] = __builtin_amdgcn_mfma_f32_4x4x1f32(W[(((q - S) % R) + R) % R], Bq[S % 3][q & 1], acc[q][0], 0,
                                                         0, 0);
        // c. stage row-step s + 3; d. fetch row-step s + 3 + PG
        st[((S + 3) % LS) * 64 + lane] = G[(S + 3) % PG];
        gload(G[(S + 3) % PG]);
      };
      int mb = m0;
      for (; mb + PER <= m1; mb += PER) static_for<PER>([&](auto sc) { advance(sc); });
      static_for<PER>([&](auto sc) {
        if (mb + decltype(sc)::value < m1) advance(sc);
      });
    };

    // Regular units: every even block of the group takes the slots of block
    // 0, every odd block those of block 1 (a stream switching every block, or
    // never), and both channels reach m1. Others go to the deferred list,
    // which the vector-ALU MAC processes after this kernel.
    int se[2], so[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      se[g] = slot[g][0];
      so[g] = slot[g][nb > 1 ? 1 : 0];
    }
    bool regular = m1 <= Mc[0] && (n_ch < 2 || m1 <= Mc[1]);
#pragma unroll
    for (int b = 0; b < TB; ++b)
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (b < nb) regular = regular && slot[g][b] == ((b & 1) ? so[g] : se[g]);
    if (!regular) {
      // the vector-ALU MAC takes time groups of 16 blocks: defer those of this
      // group in its index space
      if (threadIdx.x == 0) {
        const int g16 = ((n + 1) / 2 + 15) / 16;
        for (int h2 = 0; h2 < TB / 16; ++h2) {
          const int gi16 = gi * (TB / 16) + h2;
          if (cls + 32 * gi16 < n) B.defer_list[atomicAdd(B.defer_count, 1)] = 8 * ((pr >> 3) * g16 + gi16) + (pr & 7);
        }
      }
      continue;
    }
    run(se, so);

    // Re Y = ReX ReH - ImX ImH (Re lane), Im Y = ReX ImH + ImX ReH (Im lane);
    // the packed DC / Nyquist bin takes ReX ReH and ImX ImH
    const bool dcl = it.tile == 0 && w == 0 && b16 == 0;
    const int rowl = hh ? it.row[1] : it.row[0];
    const bool wr = hh < n_ch;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const f4 c = acc[q][u];
        const float p1 = __shfl_xor(c[1], 1);
        const float p3 = __shfl_xor(c[3], 1);
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int t = q + NP * h2;
          const float cr = h2 ? c[2] : c[0];
          const float ci = h2 ? c[3] : c[1];
          const float pi = h2 ? p3 : p1;
          float v = comp ? cr + pi : cr - pi;
          if (dcl && u == 0) v = comp ? ci : cr;
          if (t < nb && wr) {
            float* dst = reinterpret_cast<float*>(B.ypart + ((int64_t)(j0 + 2 * t) * B.n_rows + rowl) * TW) +
                         2 * (w * 16 * U + 16 * u) + (f0 & 31u);
            *dst = v;
          }
        }
      }
  }
}

// Matrix-core form of the time-blocked MAC for 16-bit (bf16 / f16) spectra.
// One 4x4x4 MFMA with 16 blocks takes 16 bins; in each, K runs over two
// partitions m, m + 1 and (Re, Im): A rows are (X(t, m), X(t, m + 1)) of four
// blocks t = q + NPQ i (raw delay-line words), B columns are the two channels'
// (H(m), H(m + 1)) arranged so that the sums are Re Y and Im Y directly:
// (Re H, -Im H) for the Re column, (Im H, Re H) for the Im column (products of
// 16-bit values are exact in FP32; the sums are FP32). The packed DC / Nyquist
// bin takes (Re H, 0) and (0, Im H). Quad q at partition pair m + 2 needs the
// delay-line pairs quad q - 2 used at m, so each lane keeps a circular buffer of
// word pairs and reads two new pairs per step. Staging as in k_tmfma: per step
// 64 lanes fetch 16 bytes each (four delay-line rows x two values, and two
// partitions x two slot sets x two channels of partition spectra, 64 B each),
// write them to the wave's LDS slot and read their operands back. Regular time
// groups only; others are deferred to k_tmac as in k_tmfma.
template <int L, int NPQ, int R, int PG, int NWV, int DT>
__global__ __launch_bounds__(64 * NWV) void k_tmfma16(BatchArgs B) {
  static_assert(DT == 1 || DT == 2, "16-bit spectra");
  static_assert(NPQ == 4 || NPQ == 8, "quads per time group");
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  typedef short s4 __attribute__((ext_vector_type(4)));
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  constexpr int TB = 4 * NPQ;               // blocks of one parity per time group
  constexpr int N = 2 * L;
  constexpr uint32_t RB = 4u * N;           // bytes per row (16-bit complex words)
  constexpr int LS = 4;                     // staging slots per wave
  constexpr int PER = std::lcm(std::lcm(R, LS), std::lcm(PG, 3));
  static_assert(R >= NPQ + 4 && PG >= 4, "window and load ring");
  __shared__ u4 stage[NWV][LS][64];
  const int TW = B.tile_width;              // 16 bins per wave
  const DevPlan& P = B.P;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int b16 = lane >> 2;                // bin of the lane's MFMA block
  const int rowi = lane & 3;                // A: row (block q + NPQ rowi)
  const int gl = (lane >> 1) & 1;           // B and C: channel
  const int comp = lane & 1;                // B and C: Re (0) or Im (1)
  const uint64_t cnt0 = *B.counter;
  const int n = B.n_blocks;
  const int groups = ((n + 1) / 2 + TB - 1) / TB;
  const int pairs = 2 * B.n_mac;
  const int lanes8 = (pairs + 7) / 8;
  const int total = 8 * lanes8 * groups;
  const char* bank = static_cast<const char*>(B.bank);
  const char* fdl = static_cast<const char*>(B.fdl);
  for (int idx = blockIdx.x; idx < total; idx += gridDim.x) {
    const int x = idx & 7, y = idx >> 3;
    const int gi = y % groups;
    const int pr = x + 8 * (y / groups);
    if (pr >= pairs) continue;
    const int cls = pr & 1;
    const WorkItem it = B.items[pr >> 1];
    const int j0 = cls + 2 * TB * gi;
    if (j0 >= n) continue;
    const int nb = min(TB, (n - j0 + 1) / 2);
    const int i = uniform(it.input);
    const int n_ch = uniform(it.n_ch);
    const int m0 = uniform(it.m0), m1 = uniform(it.m1);
    const int Mi = uniform(P.in_M[i]);
    const uint64_t c0 = cnt0 + (uint64_t)j0;
    const int p = (int)(c0 & 1u);
    const int bin = it.tile * TW + w * 16 + b16;
    const char* xb = fdl + 4 * (P.in_fdl_off[i] + (int64_t)p * Mi * N);
    const uint32_t ring_bytes = (uint32_t)Mi * RB;
    int ch[2], McL[2], Mc[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      ch[g] = uniform(g < n_ch ? it.ch[g] : it.ch[0]);
      McL[g] = uniform(P.ch_M[ch[g]]);
      Mc[g] = g < n_ch ? McL[g] : 0;
    }
    int slot[2][TB];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) slot[g][b] = B.sel[(int64_t)(j0 + 2 * min(b, nb - 1)) * B.sel_stride + ch[g]];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int sv = uniform(slot[g][b]);
        slot[g][b] = sv < 0 ? 0 : (sv >= P.K ? P.K - 1 : sv);
      }
    int se[2], so[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      se[g] = slot[g][0];
      so[g] = slot[g][nb > 1 ? 1 : 0];
    }
    bool regular = m1 <= Mc[0] && (n_ch < 2 || m1 <= Mc[1]);
#pragma unroll
    for (int b = 0; b < TB; ++b)
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (b < nb) regular = regular && slot[g][b] == ((b & 1) ? so[g] : se[g]);
    if (!regular) {
      if (threadIdx.x == 0) {
        const int g16 = ((n + 1) / 2 + 15) / 16;
        for (int h2 = 0; h2 < TB / 16; ++h2) {
          const int gi16 = gi * (TB / 16) + h2;
          if (cls + 32 * gi16 < n) B.defer_list[atomicAdd(B.defer_count, 1)] = 8 * ((pr >> 3) * g16 + gi16) + (pr & 7);
        }
      }
      continue;
    }
    const char* hb = bank + 4 * P.ch_bank_off[ch[0]];
    const uint32_t ch1_bytes = (uint32_t)(4 * (P.ch_bank_off[ch[1]] - P.ch_bank_off[ch[0]]));
    const uint32_t xbo = (uint32_t)(xb - bank);

    // B operand arrangement of the lane: (Re H, -Im H) for the Re column,
    // (Im H, Re H) for the Im column; the DC lane keeps one half
    const bool dcl = bin == 0;
    const uint32_t bsh = (comp && !dcl) ? 16u : 0u;
    const uint32_t bxm = (comp || dcl) ? 0u : 0x80000000u;
    const uint32_t bam = dcl ? (comp ? 0xffff0000u : 0x0000ffffu) : 0xffffffffu;
    auto barr = [&](uint32_t v) { return (__builtin_amdgcn_alignbit(v, v, bsh) ^ bxm) & bam; };

    // loader role: pieces 0..7: delay-line row of block NPQ (piece >> 1), value
    // d = -2k - (piece & 1); pieces 8..15: partition m0 + 2k + dl, slot set sd,
    // channel lg (64 B each, four lanes of 16 B)
    const int piece = lane >> 2, within = lane & 3;
    const bool xl = piece < 8;
    const int li = piece >> 1, lv = piece & 1;
    const int hp = piece - 8, ldl = (hp >> 2) & 1, lsd = (hp >> 1) & 1, lg = hp & 1;
    const uint32_t pos_bytes = (uint32_t)(it.tile * TW + w * 16) * 4u + 16u * (uint32_t)within;
    const int gq = ring_slot(c0 + 2u * (uint32_t)(NPQ * li), Mi);
    const uint32_t* stw = reinterpret_cast<const uint32_t*>(stage[w][0]);
    u4* st = stage[w][0];

    f4 acc[NPQ];
#pragma unroll
    for (int q = 0; q < NPQ; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    {
      // window of pairs (X_i[c], X_i[c - 1]) by c = q - 2s, X_i[e] = X(block
      // NPQ rowi + e, partition m0): c = NPQ - 1 - 2s .. -2s in use at step s,
      // -2s - 1 and -2s - 2 read during step s - 1, -2s - 3 and -2s - 4 during
      // step s (two steps ahead of their use)
      uint2 W[R];
      uint32_t Bq[3][2][2];                 // [step mod 3][set][partition of the pair]
      u4 G[PG];
      const int qr = ring_slot(c0 + 2u * (uint32_t)(NPQ * rowi), Mi);
      auto xword = [&](int e) {
        int r = (qr + e - m0) % Mi;
        r = r < 0 ? r + Mi : r;
        return *reinterpret_cast<const uint32_t*>(xb + (uint32_t)r * RB + 4u * (uint32_t)bin);
      };
#pragma unroll
      for (int c = 0; c < NPQ; ++c) W[c] = make_uint2(xword(c), xword(c - 1));
      {
        const uint32_t hbase = (gl ? ch1_bytes : 0u) + 4u * (uint32_t)bin + (uint32_t)m0 * RB;
        const uint32_t sbe = (uint32_t)(gl ? McL[1] * se[1] : McL[0] * se[0]) * RB;
        const uint32_t sbo = (uint32_t)(gl ? McL[1] * so[1] : McL[0] * so[0]) * RB;
        const bool on1 = m0 + 1 < m1;
        Bq[0][0][0] = barr(*reinterpret_cast<const uint32_t*>(hb + hbase + sbe));
        Bq[0][0][1] = on1 ? barr(*reinterpret_cast<const uint32_t*>(hb + hbase + sbe + RB)) : 0u;
        Bq[0][1][0] = barr(*reinterpret_cast<const uint32_t*>(hb + hbase + sbo));
        Bq[0][1][1] = on1 ? barr(*reinterpret_cast<const uint32_t*>(hb + hbase + sbo + RB)) : 0u;
      }
      // loader offsets from the bank base, row-step 1 (k = 1)
      const bool xlr = xl;
      const uint32_t lo = xlr ? xbo + pos_bytes : 0u;
      const uint32_t wrap = xlr ? ring_bytes : 0u;
      uint32_t goff;
      {
        int r = (gq - m0 - 2 - lv) % Mi;
        r = r < 0 ? r + Mi : r;
        const int lslot = lsd ? (lg ? so[1] : so[0]) : (lg ? se[1] : se[0]);
        const uint32_t lh = (lg ? ch1_bytes : 0u) + (uint32_t)(lg ? McL[1] : McL[0]) * (uint32_t)lslot * RB + pos_bytes;
        goff = xlr ? lo + (uint32_t)r * RB : (uint32_t)(hb - bank) + lh + (uint32_t)(m0 + 2 + ldl) * RB;
      }
      auto gload = [&](u4& o) {
        o = *reinterpret_cast<const u4*>(bank + goff);
        // two rows per step: down the ring (wrapping) or up the bank
        uint32_t dn = goff - 2 * RB;
        dn = dn < lo ? dn + wrap : dn;
        dn = dn < lo ? dn + wrap : dn;             // rings of one row
        goff = xlr ? dn : goff + 2 * RB;
      };
#pragma unroll
      for (int k = 1; k <= PG; ++k) gload(G[k % PG]);
      st[1 * 64 + lane] = G[1];
      st[2 * 64 + lane] = G[2];
      gload(G[1]);
      gload(G[2]);
      // piece word index of the lane's operands in a slot
      const int ax0 = 16 * (2 * rowi) + b16;          // X_i[-2k] (value 0), X_i[-2k - 1] at +16
      const int bh = 16 * (8 + gl) + b16;             // H: + 32 * set + 64 * partition
      {
        // operands of step 1 (row-step 1, partitions m0 + 2, m0 + 3)
        const uint32_t* sp = stw + 1 * 256;
        const uint32_t x0 = sp[ax0], x1 = sp[ax0 + 16];
        W[(R - 1) % R] = make_uint2(W[0].y, x0);
        W[(R - 2) % R] = make_uint2(x0, x1);
        const bool on2 = m0 + 2 < m1, on3 = m0 + 3 < m1;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          Bq[1][d][0] = on2 ? barr(sp[bh + 32 * d]) : 0u;
          Bq[1][d][1] = on3 ? barr(sp[bh + 32 * d + 64]) : 0u;
        }
      }
      auto advance = [&](int mm, auto sc, auto tailc) {
        constexpr int S = decltype(sc)::value;       // step index mod PER
        (void)tailc;
        // a. operands of step s + 2 (row-step s + 2): pairs c = -2s - 3 and
        //    -2s - 4, spectra of partitions m + 4, m + 5
        {
          const uint32_t* sp = stw + ((S + 2) % LS) * 256;   // row-step s + 2
          const uint32_t* sq = stw + ((S + 1) % LS) * 256;   // row-step s + 1
          const uint32_t x0 = sp[ax0], x1 = sp[ax0 + 16];      // X_i[-2s - 4], X_i[-2s - 5]
          const uint32_t xp = sq[ax0 + 16];                    // X_i[-2s - 3]
          W[(((-2 * S - 3) % R) + R) % R] = make_uint2(xp, x0);
          W[(((-2 * S - 4) % R) + R) % R] = make_uint2(x0, x1);
          // step s + 2 runs only if m + 4 < m1; its second partition may be m1
          const bool on5 = mm + 5 < m1;
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const uint32_t h4 = sp[bh + 32 * d], h5 = sp[bh + 32 * d + 64];
            Bq[(S + 2) % 3][d][0] = barr(h4);
            Bq[(S + 2) % 3][d][1] = on5 ? barr(h5) : 0u;
          }
        }
        // b. the products of step s
#pragma unroll
        for (int q = 0; q < NPQ; ++q) {
          const uint2 a = W[(((q - 2 * S) % R) + R) % R];
          const uint2 b2 = make_uint2(Bq[S % 3][q & 1][0], Bq[S % 3][q & 1][1]);
          if constexpr (DT == 1)
            acc[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b2),
                                                            acc[q], 0, 0, 0);
          else
            acc[q] = __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b2),
                                                        acc[q], 0, 0, 0);
        }
        // c. stage row-step s + 3; d. fetch row-step s + 3 + PG
        st[((S + 3) % LS) * 64 + lane] = G[(S + 3) % PG];
        gload(G[(S + 3) % PG]);
      };
      int mb = m0;
      for (; mb + 2 * PER <= m1; mb += 2 * PER)
        static_for<PER>([&](auto sc) { advance(mb + 2 * decltype(sc)::value, sc, std::false_type{}); });
      static_for<PER>([&](auto sc) {
        if (mb + 2 * decltype(sc)::value < m1) advance(mb + 2 * decltype(sc)::value, sc, std::true_type{});
      });
    }
    // C: lane column (channel gl, component comp), register r = block q + NPQ r
    const int rowl = gl ? it.row[1] : it.row[0];
    if (gl < n_ch) {
#pragma unroll
      for (int q = 0; q < NPQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = q + NPQ * r;
          if (t < nb) {
            float* dst = reinterpret_cast<float*>(B.ypart + ((int64_t)(j0 + 2 * t) * B.n_rows + rowl) * TW) +
                         2 * (w * 16 + b16) + comp;
            *dst = acc[q][r];
          }
        }
    }
  }
}

// Mixdown of a batch: for block j, bus e and 64 bins, the sum over the bus's
// channels and their partition chunks of the partial rows (the channels'
// spectra Y, eq. 8, are added before one inverse transform per bus), written
// over the first channel's chunk-0 row, which k_batch_out then reads alone.
// Four slices of the channel list are summed apart (four channels' loads in
// flight per thread) and added in a fixed order.
template <int L>
__global__ __launch_bounds__(256) void k_bus_sum(BatchArgs B) {
  const DevPlan& P = B.P;
  const int tid = threadIdx.x, kx = tid & 63, sl = tid >> 6;
  const int k = blockIdx.x * 64 + kx;
  const int e = blockIdx.y, j = blockIdx.z;
  const int TW = B.tile_width;
  const int t = k / TW, kk = k - t * TW;
  const int c0 = P.out_ptr[e], c1 = P.out_ptr[e + 1];
  float2* yp = B.ypart + (int64_t)j * B.n_rows * TW;
  float2 a[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = make_float2(0.f, 0.f);
  // this slice's channels c0 + sl + 4 i, four at a time
  for (int q = c0 + sl; q < c1; q += 16) {
    const float2* src[4];
    int nch[4];
    int mx = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int qq = q + 4 * x;
      nch[x] = 0;
      src[x] = yp;
      if (qq < c1) {
        const int c = P.out_ch[qq];
        nch[x] = B.nchunks[c];
        src[x] = yp + ((int64_t)B.row_base[c] + (int64_t)t * nch[x]) * TW + kk;
      }
      mx = max(mx, nch[x]);
    }
    for (int r = 0; r < mx; ++r) {
      float2 v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) v[x] = (r < nch[x]) ? src[x][(int64_t)r * TW] : make_float2(0.f, 0.f);
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = cadd(a[x], v[x]);
    }
  }
  __shared__ float2 red[4][64];
  red[sl][kx] = cadd(cadd(a[0], a[1]), cadd(a[2], a[3]));
  __syncthreads();
  if (sl == 0) {
    const float2 v = cadd(cadd(red[0][kx], red[1][kx]), cadd(red[2][kx], red[3][kx]));
    const int cf = P.out_ch[c0];
    yp[((int64_t)B.row_base[cf] + (int64_t)t * B.nchunks[cf]) * TW + kk] = v;
  }
}

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// v * i^m (m = 0..3): a quarter-turn rotation of a complex value.
__device__ __forceinline__ float2 rot_i(float2 v, int m) {
  const float a = (m & 1) ? v.y : v.x;
  const float b = (m & 1) ? v.x : v.y;
  return make_float2(((m + 1) & 2) ? -a : a, (m & 2) ? -b : b);
}

// Windows per workgroup of the batched output (at most).
constexpr int kOutWindows = 8;

// Fused inverse transform and overlap-add of a batch (eq. 9-13), grid
// (max(n_out, I), G): workgroup (e, g) owns output bus e and the windows
// [gW, min(n, gW + W)) of the batch, window w being the samples wL .. wL + L
// of the call's output. A circular shift by dL samples of a 4L-sample block is
// the factor i^{kd} on bin k of its spectrum, so the sum that the overlap-add
// forms for window w, quarter d of block w - d over d = 0..3, is the first
// quarter of one inverse transform of Z_w(k) = sum_d i^{kd} Y_{w-d}(k). The
// workgroup loads its blocks at once (three before its first window, W <=
// kOutWindows windows), forms the windows' Z four at a time and transforms
// them side by side, one wave per window. Windows 0..2 add the state carried
// from the previous call. Workgroups (e, 0) also form the new carried state
// (windows n .. n+2, from blocks n-3 .. n-1 and the old state where n + q < 3)
// after they have read the old one, so no workgroup waits for another;
// workgroups (x, 0) store the input history and the selection, and the last
// of them advances the call count by n.
template <int L>
__global__ __launch_bounds__(256) void k_batch_out(BatchArgs B, int W, const float* __restrict__ in,
                                                   int64_t in_stride, float* __restrict__ hist,
                                                   float* __restrict__ ola, float* __restrict__ out,
                                                   int64_t out_stride) {
  constexpr int T = 256;
  constexpr int NWV = T / 64;              // windows transformed side by side
  constexpr int N = 2 * L;                 // packed bins; the inverse is an N-point complex FFT
  constexpr int BP = (L + T - 1) / T;      // bin pairs per thread
  constexpr int NB = kOutWindows + 6;      // block slots of one pass (window w uses slot w - b0 + 3)
  __shared__ float2 twl[2 * N];
  __shared__ float2 Zs[NWV][N];            // window sums, then the transforms' second buffer
  __shared__ float2 Fs[NWV][N];            // the transforms' first buffer
  const DevPlan& P = B.P;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int e = blockIdx.x, g = blockIdx.y;
  const int n = B.n_blocks;
  const uint64_t cnt0 = (g == 0) ? *B.counter : 0;
  if (e < P.n_out) {
    for (int i = tid; i < 2 * N; i += T) twl[i] = P.tw[i];
    float* st = ola + (int64_t)e * 3 * L;
    // carried state of the previous call: window w < 3 is transformed by
    // wave w in the first round of group 0, which keeps its L samples in
    // registers (loaded before the barrier below, so before any wave stores
    // new state)
    float sto[L / 64];
#pragma unroll
    for (int i = 0; i < L / 64; ++i) sto[i] = (g == 0 && wv < 3) ? st[wv * L + lane + 64 * i] : 0.f;
    const int TW = B.tile_width;
    // the bus's spectrum rows: its first channel's rows (with a mixdown, that
    // channel's chunk-0 rows hold the bus sum), nsum rows per tile
    const int c = P.out_ch[P.out_ptr[e]];
    const int nrow = B.nchunks[c];
    const int nsum = B.bus_rows ? 1 : nrow;
    const float4* src[BP];
#pragma unroll
    for (int r = 0; r < BP; ++r) {
      const int k = 2 * (tid + T * r);
      const int t = k / TW;
      src[r] = reinterpret_cast<const float4*>(B.ypart + ((int64_t)B.row_base[c] + (int64_t)t * nrow) * TW +
                                               (k - t * TW));
    }
    const int64_t bstride = (int64_t)B.n_rows * TW / 2;   // float4 per block
    const int rstride = TW / 2;                           // float4 per row
    auto load_y = [&](int b, float4 (&y)[BP]) {
#pragma unroll
      for (int r = 0; r < BP; ++r) {
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        if (2 * (tid + T * r) < N) {
          const float4* s = src[r] + (int64_t)b * bstride;
          a = s[0];
          for (int q = 1; q < nsum; ++q) a = add4(a, s[(int64_t)q * rstride]);
        }
        y[r] = a;
      }
    };
    constexpr float scale = 1.0f / (float)(4 * L);
    wait_memory();     // the old state is in registers before any wave can store the new one
    __syncthreads();   // twiddles

    // One or two passes: the windows [w0, w1) from the blocks [b0, b1), all
    // of whose spectra are loaded first (at most W + 3 of them: every load of
    // the pass is in flight at once), block b into slot b - w0 + 3, so that
    // window w = w0 + v - 3 sums the slots v - 3 .. v (slots of blocks outside
    // [b0, b1) hold zeros: before the batch, the carried state stands for
    // them). The first window group also forms the windows n .. n+2 of the
    // new carried state: in its own pass over the last three blocks when it
    // does not reach them.
    const int j0 = g * W, j1 = min(n, j0 + W);
    const int npass = (g == 0 && j1 < n) ? 2 : 1;
    for (int ps = 0; ps < npass; ++ps) {
      int w0, w1, b0, b1;
      if (g != 0) {
        w0 = j0; w1 = j1; b0 = j0 - 3; b1 = j1;
      } else if (ps == 0) {
        w0 = 0; w1 = (j1 == n) ? n + 3 : j1; b0 = 0; b1 = j1;
      } else {
        w0 = n; w1 = n + 3; b0 = n - 3; b1 = n;
      }
      float4 y[NB][BP];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = w0 - 3 + u;
        if (b >= b0 && b < b1) {
          load_y(b, y[u]);
        } else {
#pragma unroll
          for (int r = 0; r < BP; ++r) y[u][r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      // windows w = w0 + v - 3, v from 3, NWV at a time
#pragma unroll
      for (int v0 = 3; v0 < NB; v0 += NWV) {
        if (w0 + v0 - 3 < w1) {
          // Z_w = sum over d of i^{kd} Y_{w-d}, oldest block first, into Zs
#pragma unroll
          for (int h = 0; h < NWV; ++h) {
            const int v = v0 + h;
            if (v < NB) {
#pragma unroll
              for (int r = 0; r < BP; ++r) {
                const int k = 2 * (tid + T * r);
                float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int d = 3; d >= 0; --d) {
                  if (v - d >= 0) {   // slots outside [b0, b1) hold zeros
                    const float4 yy = y[v >= d ? v - d : 0][r];
                    // k = 0: slot 0 holds the real bins 0 and 2L, whose
                    // factors are 1 (L is even)
                    const float2 lo = rot_i(make_float2(yy.x, yy.y), (k * d) & 3);
                    const float2 hi = rot_i(make_float2(yy.z, yy.w), ((k + 1) * d) & 3);
                    z = add4(z, make_float4(lo.x, lo.y, hi.x, hi.y));
                  }
                }
                if (k < N) reinterpret_cast<float4*>(Zs[h])[k >> 1] = z;
              }
            }
          }
          __syncthreads();
          // wave wv transforms window w0 + v0 - 3 + wv (every wave runs the
          // transform; one outside [w0, w1) discards its result)
          float2* Z = Zs[wv];
          float2* F = Fs[wv];
          for (int k = lane; k < N; k += 64) F[k] = fft::real_inv_pre_conj<N>(Z, k, twl);
          __syncthreads();
          const float2* R = fft::fft_fwd<N, 64>(F, Z, twl, lane);
          const int w = w0 + v0 - 3 + wv;
          if (w >= w0 && w < w1) {
#pragma unroll
            for (int i = 0; i < L / 64; ++i) {
              const int t = lane + 64 * i;
              const float2 zz = R[t >> 1];
              float val = ((t & 1) ? -zz.y : zz.x) * scale;
              if (w < 3) val += sto[i];   // w < 3: wave w, group 0, first round
              if (w < n) out[(int64_t)e * out_stride + (int64_t)w * L + t] = val;
              else st[(w - n) * L + t] = val;   // new carried state
            }
          }
          __syncthreads();   // Zs and Fs are reused by the next windows
        }
      }
    }
    // slots of the bus's channels at the batch's last block
    if (g == 0 && B.copy_sel)
      for (int q = P.out_ptr[e] + tid; q < P.out_ptr[e + 1]; q += T)
        B.sel_store[P.out_ch[q]] = B.sel[(int64_t)(n - 1) * B.sel_stride + P.out_ch[q]];
  }
  if (e < P.I && g == 0) {
    const uint64_t lastc = cnt0 + (uint64_t)(n - 1);
    float* hnew = hist + ((size_t)(lastc & 1u) * P.I + e) * L;
    const float* xin = in + (int64_t)e * in_stride + (int64_t)(n - 1) * L;
    for (int k = tid; k < L; k += T) hnew[k] = xin[k];
  }
  __syncthreads();
  if (tid == 0 && g == 0) {
    if (atomicAdd(B.done, 1) == (int)gridDim.x - 1) {
      *B.done = 0;
      *B.counter = cnt0 + (uint64_t)n;
    }
  }
}

// ---------------------------------------------------------------- plain path

// One workgroup (one wave) per input: new input spectrum into the delay line.
template <int L, int DT>
__global__ __launch_bounds__(64) void k_fwd(DevPlan P, const float* __restrict__ in, int64_t in_stride,
                                            float* __restrict__ hist, typename Store<DT>::T* __restrict__ fdl,
                                            const uint64_t* __restrict__ counter) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int tid = threadIdx.x;
  const uint64_t cnt = *counter;
  load_tables<L, 64>(P, twl, winl, tid);
  __syncthreads();
  input_spectrum<L, 64, DT, false>(P, in, in_stride, hist, fdl, blockIdx.x, (int)(cnt & 1u), cnt, twl, winl, bufA,
                                   bufB, tid);
}

// One workgroup per MAC work item: partial spectrum tiles.
template <int V, int G, int NW, int DT>
__global__ __launch_bounds__(64 * NW) void k_mac(DevPlan P, const WorkItem* __restrict__ items,
                                                 const typename Store<DT>::T* __restrict__ bank,
                                                 const typename Store<DT>::T* __restrict__ fdl,
                                                 const int32_t* __restrict__ sel, float2* __restrict__ ypart,
                                                 const uint64_t* __restrict__ counter) {
  __shared__ float2 red[NW][G][64 * V];
  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const uint64_t cnt = *counter;
  float2 acc[G][V];
  mac_item<V, G, NW, DT, (G * V <= 4) ? 4 : 2>(P, it, bank, fdl, sel, (int)(cnt & 1u), cnt, tid & 63, tid >> 6, acc);
  write_partials<V, G, NW, false>(it, acc, red, ypart, tid & 63, tid >> 6, tid);
}

// Mixdown of one block: for 64 bins of bus e, the sum over the bus's channels
// of each channel's spectrum Y (its partial rows plus the m = 0 term,
// eq. 8) into P.ybus. Four slices of the channel list are summed apart and
// added in a fixed order.
template <int L, int DT>
__global__ __launch_bounds__(256) void k_bus_sum1(DevPlan P, const float2* __restrict__ ypart,
                                                  const typename Store<DT>::T* __restrict__ bank,
                                                  const typename Store<DT>::T* __restrict__ fdl,
                                                  const int32_t* __restrict__ sel,
                                                  const uint64_t* __restrict__ counter) {
  using ST = typename Store<DT>::T;
  constexpr int N = 2 * L;
  const int tid = threadIdx.x, kx = tid & 63, sl = tid >> 6;
  const int k = blockIdx.x * 64 + kx, e = blockIdx.y;
  const uint64_t cnt = *counter;
  const int p = (int)(cnt & 1u);
  const int TW = P.tile_width;
  const int t = k / TW, b = k - t * TW;
  float2 acc = make_float2(0.f, 0.f);
  for (int q = P.out_ptr[e] + sl; q < P.out_ptr[e + 1]; q += 4) {
    const int c = P.out_ch[q];
    const int i = P.ch_input[c];
    const int Mi = P.in_M[i];
    const ST* xrow = fdl + P.in_fdl_off[i] + ((int64_t)p * Mi + ring_slot(cnt, Mi)) * N;
    int s = sel[c];
    s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s);
    const float2 X = unpack<DT>(xrow[k]);
    const float2 H = unpack<DT>(bank[P.ch_bank_off[c] + (int64_t)s * P.ch_M[c] * N + k]);
    float2 v = (k == 0) ? make_float2(H.x * X.x, H.y * X.y) : cmul(H, X);
    const int nch = P.ch_nchunks[c];
    const float2* src = ypart + ((int64_t)P.ch_row_base[c] + (int64_t)t * nch) * TW + b;
    for (int j = 0; j < nch; ++j) v = cadd(v, src[(int64_t)j * TW]);
    acc = cadd(acc, v);
  }
  __shared__ float2 red[4][64];
  red[sl][kx] = acc;
  __syncthreads();
  if (sl == 0) P.ybus[(int64_t)e * N + k] = cadd(cadd(red[0][kx], red[1][kx]), cadd(red[2][kx], red[3][kx]));
}

// One workgroup per output bus: the sum of its channels' spectra, the inverse
// transform and the overlap-add; the last workgroup to finish advances the
// call count.
template <int L, int DT>
__global__ __launch_bounds__(64) void k_inv(DevPlan P, const float2* __restrict__ ypart,
                                            const typename Store<DT>::T* __restrict__ bank,
                                            const typename Store<DT>::T* __restrict__ fdl,
                                            const int32_t* __restrict__ sel, float* __restrict__ ola,
                                            float* __restrict__ out, int64_t out_stride, int32_t copy_sel,
                                            int32_t* __restrict__ sel_store, int32_t* __restrict__ done,
                                            uint64_t* __restrict__ counter) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 Y[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const uint64_t cnt = *counter;
  const int p = (int)(cnt & 1u);
  load_tables<L, 64>(P, twl, winl, tid);
  float* st = ola + (int64_t)e * 3 * L;
  float old[(4 * L + 63) / 64];
  ola_prefetch<L, 64>(st, old, tid);
  const int c0 = P.out_ptr[e], c1 = P.out_ptr[e + 1];
  if (P.ybus) {
    // mixdown: the bus spectrum, summed over the bus's channels by k_bus_sum1
    for (int k = tid; k < N; k += 64) Y[k] = P.ybus[(int64_t)e * N + k];
  } else {
    channel_spectrum<L, 64, DT, false>(P, ypart, bank, fdl, sel, P.out_ch[c0], p, cnt, Y, tid);
  }
  __syncthreads();
  inverse_ola<L, 64>(Y, bufA, bufB, twl, old, st, out + (int64_t)e * out_stride, tid);
  // slots of the bus's channels, one channel per thread
  if (copy_sel)
    for (int q = c0 + tid; q < c1; q += 64) sel_store[P.out_ch[q]] = sel[P.out_ch[q]];
  if (tid == 0) {
    if (atomicAdd(done, 1) == (int)gridDim.x - 1) {
      *done = 0;
      *counter = cnt + 1u;
    }
  }
}

// One workgroup per partition: spectra of the 2L-tap partitions of one IR.
template <int L, int DT>
__global__ __launch_bounds__(64) void k_irprep(DevPlan P, const float* __restrict__ taps, int32_t n_taps,
                                               typename Store<DT>::T* __restrict__ dst) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  load_tables<L, 64>(P, twl, winl, tid);
  for (int n = tid; n < L; n += 64) {
    const int t0 = 2 * L * m + 2 * n;
    const float h0 = (t0 < n_taps) ? taps[t0] : 0.f;
    const float h1 = (t0 + 1 < n_taps) ? taps[t0 + 1] : 0.f;
    bufA[n] = make_float2(h0, h1);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, 64>(bufA, bufB, twl, tid);
  for (int k = tid; k < N; k += 64) dst[(int64_t)m * N + k] = pack<DT>(fft::real_fwd_post<N>(Z, k, twl));
}

// Partition spectra of one slot of every channel (eq. 3, 5, 7) in one launch:
// global partition g (of sum_c M_c, prefix part_base[c]) is channel c's
// partition m; one partition per wave, 4 waves per workgroup (tables loaded
// once). Channel c reads taps[c * taps_stride + t] for t < n_taps(c) =
// min(taps_stride, taps_of_channel[c]); the rest of its partitions are zero.
template <int L, int DT>
__global__ __launch_bounds__(256) void k_irprep_all(DevPlan P, const int32_t* __restrict__ part_base,
                                                    const int32_t* __restrict__ ch_taps, const float* __restrict__ taps,
                                                    int64_t taps_stride, int32_t slot,
                                                    typename Store<DT>::T* __restrict__ bank) {
  constexpr int N = 2 * L;
  constexpr int W = 4;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[W][N];
  __shared__ float2 bufB[W][N];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  load_tables<L, 64 * W>(P, twl, winl, tid);
  const int total = part_base[P.C];
  const int gr = blockIdx.x * W + w;
  const bool live = gr < total;
  const int g = live ? gr : total - 1;
  // channel of partition g: the last c with part_base[c] <= g
  int lo = 0, hi = P.C - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (part_base[mid] <= g) lo = mid; else hi = mid - 1;
  }
  const int c = lo;
  const int m = g - part_base[c];
  const int Mc = P.ch_M[c];
  const int64_t nt = min((int64_t)ch_taps[c], taps_stride);
  const float* tc = taps + (int64_t)c * taps_stride;
  for (int n = lane; n < L; n += 64) {
    const int64_t t0 = (int64_t)2 * L * m + 2 * n;
    const float h0 = (t0 < nt) ? tc[t0] : 0.f;
    const float h1 = (t0 + 1 < nt) ? tc[t0 + 1] : 0.f;
    bufA[w][n] = make_float2(h0, h1);
    bufA[w][n + L] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, 64>(bufA[w], bufB[w], twl, lane);
  if (live) {
    typename Store<DT>::T* dst = bank + P.ch_bank_off[c] + ((int64_t)slot * Mc + m) * N;
    for (int k = lane; k < N; k += 64) dst[k] = pack<DT>(fft::real_fwd_post<N>(Z, k, twl));
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4* __restrict__ p, size_t n16, uint8_t* __restrict__ tail,
                                                   size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

// ---------------------------------------------------------------- dispatch

// Storage types compiled in this file: TVX_DT only.
template <typename F>
hipError_t by_dtype(int dt, F&& f) {
  if (dt != TVX_DT) return hipErrorInvalidValue;
  return f(std::integral_constant<int, TVX_DT>{});
}

template <typename F>
hipError_t by_shape(const MacShape& sh, F&& f) {
  auto nw = [&](auto V, auto G) -> hipError_t {
    switch (sh.NW) {
      case 4: return f(V, G, std::integral_constant<int, 4>{});
      case 8: return f(V, G, std::integral_constant<int, 8>{});
      default: return hipErrorInvalidValue;
    }
  };
  auto g = [&](auto V) -> hipError_t {
    switch (sh.G) {
      case 1: return nw(V, std::integral_constant<int, 1>{});
      case 2: return nw(V, std::integral_constant<int, 2>{});
      case 4: return nw(V, std::integral_constant<int, 4>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (sh.V) {
    case 2: return g(std::integral_constant<int, 2>{});
    case 4: return g(std::integral_constant<int, 4>{});
    default: return hipErrorInvalidValue;
  }
}

// Batched MAC shapes: V in {1, 2} bins per lane, G in {1, 2} channels per
// item (the waves per tile, 1, 2 or 4, are a launch parameter).
template <typename F>
hipError_t by_bshape(const MacShape& sh, F&& f) {
  auto g = [&](auto V) -> hipError_t {
    switch (sh.G) {
      case 1: return f(V, std::integral_constant<int, 1>{});
      case 2: return f(V, std::integral_constant<int, 2>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (sh.V) {
    case 1: return g(std::integral_constant<int, 1>{});
    case 2: return g(std::integral_constant<int, 2>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Launchers that depend on the hop L. This file is compiled once per hop and
// storage type (TVX_HOP, TVX_DT) and instantiates them for that pair only; the
// hop-independent launchers are compiled with the smallest hop.

template <int L, int DTT>
hipError_t hop_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride, float* hist, void* fdl,
                   const uint64_t* counter, hipStream_t s) {
  return by_dtype(dtype, [&](auto Dc) {
    constexpr int DT = decltype(Dc)::value;
    hipLaunchKernelGGL((k_fwd<L, DT>), dim3(P.I), dim3(64), 0, s, P, in, in_stride, hist,
                       static_cast<typename Store<DT>::T*>(fdl), counter);
    return hipGetLastError();
  });
}

template <int L, int DTT>
hipError_t hop_inv(const DevPlan& P, int dtype, const float2* ypart, const void* bank, const void* fdl,
                   const int32_t* sel, float* ola, float* out, int64_t out_stride, int32_t copy_sel,
                   int32_t* sel_store, int32_t* done, uint64_t* counter, hipStream_t s) {
  return by_dtype(dtype, [&](auto Dc) {
    constexpr int DT = decltype(Dc)::value;
    using ST = typename Store<DT>::T;
    if (P.ybus) {
      hipLaunchKernelGGL((k_bus_sum1<L, DT>), dim3(2 * L / 64, P.n_out), dim3(256), 0, s, P, ypart,
                         static_cast<const ST*>(bank), static_cast<const ST*>(fdl), sel, counter);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_inv<L, DT>), dim3(P.n_out), dim3(64), 0, s, P, ypart, static_cast<const ST*>(bank),
                       static_cast<const ST*>(fdl), sel, ola, out, out_stride, copy_sel, sel_store, done, counter);
    return hipGetLastError();
  });
}

template <int L, int DTT>
hipError_t hop_block(const BlockArgs& A, int dtype, const MacShape& shape, int grid, hipStream_t s) {
  if (A.n_items <= 0 || grid <= 0) return hipErrorInvalidValue;
  return by_dtype(dtype, [&](auto Dc) {
    return by_shape(shape, [&](auto Vc, auto Gc, auto NWc) {
      constexpr int DT = decltype(Dc)::value, V = decltype(Vc)::value, G = decltype(Gc)::value,
                    NW = decltype(NWc)::value;
      if constexpr (64 * V > 2 * L) {
        return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((k_block<L, V, G, NW, DT>), dim3(grid), dim3(64 * NW), 0, s, A);
        return hipGetLastError();
      }
    });
  });
}

template <int L, int DTT>
hipError_t hop_batch(const BatchArgs& B, int dtype, const MacShape& shape, int grid, const float* in,
                     int64_t in_stride, float* hist, float* ola, float* out, int64_t out_stride, hipStream_t s,
                     hipEvent_t* ev) {
  if (B.n_blocks <= 0) return hipSuccess;
  return by_dtype(dtype, [&](auto Dc) {
    constexpr int DT = decltype(Dc)::value;
    using ST = typename Store<DT>::T;
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    const int bgroups = (B.n_blocks + kBatchBlocksPerWg - 1) / kBatchBlocksPerWg;
    // fewer than 16 workgroups per CU at kBatchBlocksPerWg blocks each: two
    // blocks per workgroup, for more workgroups in flight
    const int sbpw = (B.P.I * bgroups < 16 * 256) ? 2 : kBatchBlocksPerWg;
    hipLaunchKernelGGL((k_batch_spectra<L, DT>), dim3((B.n_blocks + sbpw - 1) / sbpw, B.P.I), dim3(256), 0, s, B.P,
                       in, in_stride, hist, static_cast<ST*>(B.fdl), B.counter, B.n_blocks, B.defer_count, sbpw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (B.n_mac > 0) {
      if (shape.E == 1) {
        // matrix-core MAC: up to two channels per item, time groups of 16 or 32
        if constexpr (DT != 0) {
          if (shape.G > 2 || (B.time_block != 16 && B.time_block != 32) || shape.V != 1 ||
              (shape.NW != 4 && shape.NW != 8))
            return hipErrorInvalidValue;
          if (B.tile_width != 16 * shape.NW || B.tile_width > 2 * L || !B.defer_list || !B.defer_count)
            return hipErrorInvalidValue;
          const dim3 tb(64 * shape.NW);
          if (B.time_block == 32) {
            if (shape.NW == 8) hipLaunchKernelGGL((k_tmfma16<L, 8, 12, 12, 8, DT>), dim3(grid), tb, 0, s, B);
            else hipLaunchKernelGGL((k_tmfma16<L, 8, 12, 12, 4, DT>), dim3(grid), tb, 0, s, B);
          } else {
            if (shape.NW == 8) hipLaunchKernelGGL((k_tmfma16<L, 4, 8, 12, 8, DT>), dim3(grid), tb, 0, s, B);
            else hipLaunchKernelGGL((k_tmfma16<L, 4, 8, 12, 4, DT>), dim3(grid), tb, 0, s, B);
          }
          e = hipGetLastError();
          if (e != hipSuccess) return e;
          BatchArgs Bd = B;
          Bd.from_list = 1;
          const dim3 tv(B.tile_width);
          const dim3 gd(grid < 1024 ? grid : 1024);
          if (shape.G == 1)
            hipLaunchKernelGGL((k_tmac<L, 1, 1, 16, DT>), gd, tv, 0, s, Bd);
          else
            hipLaunchKernelGGL((k_tmac<L, 1, 2, 16, DT>), gd, tv, 0, s, Bd);
          e = hipGetLastError();
        } else {
          if (shape.G > 2 || (B.time_block != 16 && B.time_block != 32) || shape.V != 1 ||
              (shape.NW != 4 && shape.NW != 8))
            return hipErrorInvalidValue;
          if (B.tile_width != 16 * shape.NW || B.tile_width > 2 * L || !B.defer_list || !B.defer_count)
            return hipErrorInvalidValue;
          const dim3 tb(64 * shape.NW);
          if (B.time_block == 32) {
            if (shape.NW == 8) hipLaunchKernelGGL((k_tmfma<L, 16, 24, 12, 8, DT>), dim3(grid), tb, 0, s, B);
            else hipLaunchKernelGGL((k_tmfma<L, 16, 24, 12, 4, DT>), dim3(grid), tb, 0, s, B);
          } else {
            if (shape.NW == 8) hipLaunchKernelGGL((k_tmfma<L, 8, 12, 12, 8, DT>), dim3(grid), tb, 0, s, B);
            else hipLaunchKernelGGL((k_tmfma<L, 8, 12, 12, 4, DT>), dim3(grid), tb, 0, s, B);
          }
          e = hipGetLastError();
          if (e != hipSuccess) return e;
          // the deferred units on the vector ALU: one wave per 64 bins of the
          // tile, a grid of at most 1024 workgroups striding over the list
          BatchArgs Bd = B;
          Bd.from_list = 1;
          const dim3 tv(B.tile_width);
          const dim3 gd(grid < 1024 ? grid : 1024);
          if (shape.G == 1)
            hipLaunchKernelGGL((k_tmac<L, 1, 1, 16, DT>), gd, tv, 0, s, Bd);
          else
            hipLaunchKernelGGL((k_tmac<L, 1, 2, 16, DT>), gd, tv, 0, s, Bd);
          e = hipGetLastError();
        }
      } else {
      e = by_bshape(shape, [&](auto Vc, auto Gc) {
        constexpr int V = decltype(Vc)::value, G = decltype(Gc)::value;
        if (shape.NW != 1 && shape.NW != 2 && shape.NW != 4) return hipErrorInvalidValue;
        if (64 * V * shape.NW != B.tile_width || B.tile_width > 2 * L) return hipErrorInvalidValue;
        if (B.time_block == 8) {
          hipLaunchKernelGGL((k_tmac<L, V, G, 8, DT>), dim3(grid), dim3(64 * shape.NW), 0, s, B);
        } else if constexpr (V == 1) {
          if (B.time_block != 16) return hipErrorInvalidValue;
          hipLaunchKernelGGL((k_tmac<L, V, G, 16, DT>), dim3(grid), dim3(64 * shape.NW), 0, s, B);
        } else {
          return hipErrorInvalidValue;
        }
        return hipGetLastError();
      });
      }
      if (e != hipSuccess) return e;
    }
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    if (B.bus_rows) {
      hipLaunchKernelGGL((k_bus_sum<L>), dim3(2 * L / 64, B.P.n_out, B.n_blocks), dim3(256), 0, s, B);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    // windows per workgroup: enough workgroups for four per compute unit, at
    // least four windows each (a group also reads the three blocks before its
    // first), at most kOutWindows
    const int no = B.P.n_out;
    const int want = (B.n_blocks * no + 1023) / 1024;
    const int W = std::min(kOutWindows, std::max(4, want));
    const int groups = (B.n_blocks + W - 1) / W;
    const int gx = no > B.P.I ? no : B.P.I;
    hipLaunchKernelGGL((k_batch_out<L>), dim3(gx, groups), dim3(256), 0, s, B, W, in, in_stride, hist, B.ola_state,
                       out, out_stride);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev) e = hipEventRecord(ev[3], s);
    return e;
  });
}

template <int L, int DTT>
hipError_t hop_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M, void* dst,
                      hipStream_t s) {
  return by_dtype(dtype, [&](auto Dc) {
    constexpr int DT = decltype(Dc)::value;
    hipLaunchKernelGGL((k_irprep<L, DT>), dim3(M), dim3(64), 0, s, P, taps, n_taps,
                       static_cast<typename Store<DT>::T*>(dst));
    return hipGetLastError();
  });
}

template hipError_t hop_fwd<TVX_HOP, TVX_DT>(const DevPlan&, int, const float*, int64_t, float*, void*, const uint64_t*,
                                     hipStream_t);
template hipError_t hop_inv<TVX_HOP, TVX_DT>(const DevPlan&, int, const float2*, const void*, const void*, const int32_t*,
                                     float*, float*, int64_t, int32_t, int32_t*, int32_t*, uint64_t*, hipStream_t);
template hipError_t hop_block<TVX_HOP, TVX_DT>(const BlockArgs&, int, const MacShape&, int, hipStream_t);
template hipError_t hop_batch<TVX_HOP, TVX_DT>(const BatchArgs&, int, const MacShape&, int, const float*, int64_t, float*,
                                       float*, float*, int64_t, hipStream_t, hipEvent_t*);
template hipError_t hop_irprep<TVX_HOP, TVX_DT>(const DevPlan&, int, const float*, int32_t, int32_t, void*, hipStream_t);

template <int L, int DTT>
hipError_t hop_irprep_all(const DevPlan& P, int dtype, const int32_t* part_base, int32_t total_parts,
                          const int32_t* ch_taps, const float* taps, int64_t taps_stride, int32_t slot, void* bank,
                          hipStream_t s) {
  if (total_parts <= 0) return hipSuccess;
  return by_dtype(dtype, [&](auto Dc) {
    constexpr int DT = decltype(Dc)::value;
    hipLaunchKernelGGL((k_irprep_all<L, DT>), dim3((total_parts + 3) / 4), dim3(256), 0, s, P, part_base, ch_taps,
                       taps, taps_stride, slot, static_cast<typename Store<DT>::T*>(bank));
    return hipGetLastError();
  });
}
template hipError_t hop_irprep_all<TVX_HOP, TVX_DT>(const DevPlan&, int, const int32_t*, int32_t, const int32_t*,
                                                    const float*, int64_t, int32_t, void*, hipStream_t);

#if TVX_HOP == 64
template <int DTT>
hipError_t mac_dt(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items, int n_items,
                  const void* bank, const void* fdl, const int32_t* sel, float2* ypart, const uint64_t* counter,
                  hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  return by_dtype(dtype, [&](auto Dc) {
    return by_shape(shape, [&](auto Vc, auto Gc, auto NWc) {
      constexpr int DT = decltype(Dc)::value, V = decltype(Vc)::value, G = decltype(Gc)::value,
                    NW = decltype(NWc)::value;
      using ST = typename Store<DT>::T;
      hipLaunchKernelGGL((k_mac<V, G, NW, DT>), dim3(n_items), dim3(64 * NW), 0, s, P, items,
                         static_cast<const ST*>(bank), static_cast<const ST*>(fdl), sel, ypart, counter);
      return hipGetLastError();
    });
  });
}

template hipError_t mac_dt<TVX_DT>(const DevPlan&, int, const MacShape&, const WorkItem*, int, const void*,
                                   const void*, const int32_t*, float2*, const uint64_t*, hipStream_t);
#endif

#if TVX_HOP == 64 && TVX_DT == 0
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes - n16 * 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4*>(p), n16,
                     static_cast<uint8_t*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}
#endif

}  // namespace tvx
