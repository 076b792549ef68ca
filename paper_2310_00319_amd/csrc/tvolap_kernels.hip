// gfx950 kernels of the TVOLAP hot path (Jaeger et al., arXiv 2310.00319, Sec. 2).
//
//   k_fwd     Hann-weighted 2L block (eq. 1-2), zero pad to 4L (eq. 5), real
//             4L-point DFT (eq. 4) via a 2L-point complex FFT in LDS; the new
//             spectrum goes into its delay-line slot.
//   k_mac     spectral MAC of eq. 8: Y = sum_m H_{g(l)}(m) X(l - 2m), streamed
//             from HBM in 16-byte lanes, FP32 accumulation, partitions split
//             across the waves of a workgroup and reduced through LDS.
//   k_inv     sums the partial spectra of a channel, inverse DFT (eq. 9) via a
//             2L-point complex FFT, overlap-add at hop L (eq. 10-13).
//   k_irprep  IR partition spectra (eq. 3, 6-7) into a bank slot.
//
// The complex FFT is a Stockham autosort FFT with radix-8/4 stages and one LDS
// ping-pong per stage. A real 4L-point transform is done as a 2L-point complex
// transform of z(n) = x(2n) + i x(2n+1) plus a post-processing pass; the
// inverse runs the same steps backwards. Twiddles come from a table computed in
// double precision on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tvolap_internal.h"

namespace tvx {
namespace {

// ---------------------------------------------------------------- complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }   // a * (+i)
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

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

__device__ __forceinline__ float2 unpack_bf16(uint32_t w) {
  return make_float2(bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16));
}
__device__ __forceinline__ float2 unpack_f16(uint32_t w) {
  return make_float2(f16_to_f32(w), f16_to_f32(w >> 16));
}

// Load V consecutive stored complex values (16 bytes per lane where possible).
template <int DT, int V>
__device__ __forceinline__ void load_vec(const typename Store<DT>::T* __restrict__ p, float2 (&o)[V]) {
  if constexpr (DT == 0) {
    if constexpr (V == 1) {
      o[0] = *p;
    } else {
#pragma unroll
      for (int j = 0; j < V; j += 2) {
        float4 t = *reinterpret_cast<const float4*>(p + j);
        o[j] = make_float2(t.x, t.y);
        o[j + 1] = make_float2(t.z, t.w);
      }
    }
  } else {
    uint32_t w[V];
    if constexpr (V == 1) {
      w[0] = *p;
    } else if constexpr (V == 2) {
      uint2 t = *reinterpret_cast<const uint2*>(p);
      w[0] = t.x; w[1] = t.y;
    } else {
#pragma unroll
      for (int j = 0; j < V; j += 4) {
        uint4 t = *reinterpret_cast<const uint4*>(p + j);
        w[j] = t.x; w[j + 1] = t.y; w[j + 2] = t.z; w[j + 3] = t.w;
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) o[j] = (DT == 1) ? unpack_bf16(w[j]) : unpack_f16(w[j]);
  }
}

// ---------------------------------------------------------------- small DFTs (forward sign)

template <int R> __device__ __forceinline__ void dft(float2 (&v)[R]);

template <> __device__ __forceinline__ void dft<2>(float2 (&v)[2]) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void dft<4>(float2 (&v)[4]) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <> __device__ __forceinline__ void dft<8>(float2 (&v)[8]) {
  constexpr float c = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft<4>(e);
  dft<4>(o);
  // o[k] *= exp(-2 pi i k / 8)
  o[1] = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
  o[2] = cmul_mi(o[2]);
  o[3] = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// ---------------------------------------------------------------- Stockham stages

// One radix-R stage of an N-point forward FFT run by T threads. NS is the
// product of the radices of the earlier stages. `tw` holds exp(-2 pi i t / 2N).
template <int N, int R, int NS, int T>
__device__ __forceinline__ void stage(const float2* __restrict__ src, float2* __restrict__ dst,
                                      const float2* __restrict__ tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TWS = 2 * (N / (NS * R));
#pragma unroll
  for (int j0 = 0; j0 < NB; j0 += T) {
    const int j = j0 + tid;
    if ((NB % T == 0) || j < NB) {
      const int k = j & (NS - 1);
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[j + r * NB];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * TWS]);
      }
      dft<R>(v);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[base + r * NS] = v[r];
    }
  }
}

// N-point forward complex FFT of `a` (LDS); `b` is scratch of the same size.
// Returns the buffer that holds the result. Callers synchronise before.
template <int N, int T>
__device__ __forceinline__ float2* fft_fwd(float2* a, float2* b, const float2* tw, int tid) {
  if constexpr (N == 128) {
    stage<128, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<128, 4, 8, T>(b, a, tw, tid); __syncthreads();
    stage<128, 4, 32, T>(a, b, tw, tid); __syncthreads();
    return b;
  } else if constexpr (N == 256) {
    stage<256, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<256, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage<256, 4, 64, T>(a, b, tw, tid); __syncthreads();
    return b;
  } else if constexpr (N == 512) {
    stage<512, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<512, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage<512, 8, 64, T>(a, b, tw, tid); __syncthreads();
    return b;
  } else {
    static_assert(N == 1024, "unsupported FFT size");
    stage<1024, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<1024, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage<1024, 4, 64, T>(a, b, tw, tid); __syncthreads();
    stage<1024, 4, 256, T>(b, a, tw, tid); __syncthreads();
    return a;
  }
}

// Packed bin k of the real 4L-point DFT from Z = FFT_2L(x(2n) + i x(2n+1)).
// N = 2L. Slot 0 packs the two real bins (X(0), X(2L)).
template <int N>
__device__ __forceinline__ float2 real_fwd_post(const float2* Z, int k, const float2* tw) {
  if (k == 0) {
    const float2 z = Z[0];
    return make_float2(z.x + z.y, z.x - z.y);
  }
  const float2 A = Z[k];
  const float2 B = cconj(Z[N - k]);
  const float2 E = cscale(cadd(A, B), 0.5f);
  const float2 D = cscale(csub(A, B), 0.5f);
  return cadd(E, cmul_mi(cmul(tw[k], D)));
}

// conj of Z'(k), the 2L-point spectrum whose inverse transform interleaves the
// even and odd samples of the real inverse DFT of the packed spectrum Y.
template <int N>
__device__ __forceinline__ float2 real_inv_pre_conj(const float2* Y, int k, const float2* tw) {
  if (k == 0) {
    const float2 y = Y[0];
    return make_float2(y.x + y.y, -(y.x - y.y));
  }
  const float2 A = Y[k];
  const float2 B = cconj(Y[N - k]);
  const float2 S = cadd(A, B);
  const float2 D = csub(A, B);
  const float2 Zp = cadd(S, cmul_pi(cmul(cconj(tw[k]), D)));
  return cconj(Zp);
}

// ---------------------------------------------------------------- kernels

// One workgroup (one wave) per input: window, transform, store in the delay line.
template <int L, int DT>
__global__ __launch_bounds__(64) void k_fwd(DevPlan P, const float* __restrict__ in, int64_t in_stride,
                                            float* __restrict__ hist, typename Store<DT>::T* __restrict__ fdl,
                                            const uint64_t* __restrict__ counter) {
  constexpr int N = 2 * L;
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const uint64_t c = *counter;
  const int p = (int)(c & 1u);
  const int Mi = P.in_M[i];
  const int q = (int)((c >> 1) % (uint64_t)Mi);
  const float* hold = hist + ((size_t)(p ^ 1) * P.I + i) * L;
  float* hnew = hist + ((size_t)p * P.I + i) * L;
  const float* xin = in + (int64_t)i * in_stride;

  for (int n = tid; n < L; n += 64) {
    const int t0 = 2 * n, t1 = 2 * n + 1;
    const float s0 = (t0 < L) ? hold[t0] : xin[t0 - L];
    const float s1 = (t1 < L) ? hold[t1] : xin[t1 - L];
    bufA[n] = make_float2(P.win[t0] * s0, P.win[t1] * s1);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
  for (int n = tid; n < L; n += 64) hnew[n] = xin[n];
  __syncthreads();
  const float2* Z = fft_fwd<N, 64>(bufA, bufB, P.tw, tid);
  typename Store<DT>::T* dst = fdl + P.in_fdl_off[i] + ((int64_t)p * Mi + q) * N;
  for (int k = tid; k < N; k += 64) dst[k] = pack<DT>(real_fwd_post<N>(Z, k, P.tw));
}

// Spectral MAC over one work item per workgroup.
template <int V, int G, int NW, int DT>
__global__ __launch_bounds__(64 * NW) void k_mac(DevPlan P, const WorkItem* __restrict__ items,
                                                 const typename Store<DT>::T* __restrict__ bank,
                                                 const typename Store<DT>::T* __restrict__ fdl,
                                                 const int32_t* __restrict__ sel, float2* __restrict__ ypart,
                                                 const uint64_t* __restrict__ counter) {
  using ST = typename Store<DT>::T;
  constexpr int TW = 64 * V;
  __shared__ float2 red[NW][G][TW];
  const WorkItem it = items[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int N = 2 * P.L;
  const uint64_t c = *counter;
  const int p = (int)(c & 1u);
  const int Mi = P.in_M[it.input];
  const int q = (int)((c >> 1) % (uint64_t)Mi);
  const int kbase = it.tile * TW + lane * V;
  const ST* xrow = fdl + P.in_fdl_off[it.input] + (int64_t)p * Mi * N + kbase;
  const ST* hrow[G];
  int Mc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g < it.n_ch) {
      const int ch = it.ch[g];
      int s = sel[ch];
      s = s < 0 ? 0 : (s >= P.K ? P.K - 1 : s);
      Mc[g] = P.ch_M[ch];
      hrow[g] = bank + P.ch_bank_off[ch] + (int64_t)s * Mc[g] * N + kbase;
    } else {
      Mc[g] = 0;
      hrow[g] = bank;
    }
  }
  const bool dc_lane = (kbase == 0);
  float2 acc[G][V];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[g][v] = make_float2(0.f, 0.f);

  for (int m = it.m0 + w; m < it.m1; m += NW) {
    int xr = q - m;
    if (xr < 0) xr += Mi;
    float2 X[V];
    load_vec<DT, V>(xrow + (int64_t)xr * N, X);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (m < Mc[g]) {
        float2 H[V];
        load_vec<DT, V>(hrow[g] + (int64_t)m * N, H);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          float2 prod = cmul(H[v], X[v]);
          if (v == 0 && dc_lane) prod = make_float2(H[0].x * X[0].x, H[0].y * X[0].y);
          acc[g][v] = cadd(acc[g][v], prod);
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int v = 0; v < V; ++v) red[w][g][lane * V + v] = acc[g][v];
  __syncthreads();
  for (int idx = threadIdx.x; idx < G * TW; idx += 64 * NW) {
    const int g = idx / TW;
    const int b = idx - g * TW;
    if (g < it.n_ch) {
      float2 s = red[0][g][b];
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) s = cadd(s, red[ww][g][b]);
      ypart[(int64_t)(it.row + g) * TW + b] = s;
    }
  }
}

// One workgroup per channel: gather the spectrum, inverse transform, overlap-add.
template <int L>
__global__ __launch_bounds__(64) void k_inv(DevPlan P, int TW, const float2* __restrict__ ypart,
                                            const int32_t* __restrict__ rows_ptr, const int32_t* __restrict__ rows,
                                            float* __restrict__ ola, float* __restrict__ out, int64_t out_stride,
                                            const int32_t* __restrict__ sel_in, int32_t* __restrict__ sel_store,
                                            uint64_t* __restrict__ counter) {
  constexpr int N = 2 * L;
  __shared__ float2 Y[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int T = N / TW;
  for (int k = tid; k < N; k += 64) {
    const int t = k / TW;
    const int b = k - t * TW;
    float2 s = make_float2(0.f, 0.f);
    const int r0 = rows_ptr[c * T + t], r1 = rows_ptr[c * T + t + 1];
    for (int r = r0; r < r1; ++r) s = cadd(s, ypart[(int64_t)rows[r] * TW + b]);
    Y[k] = s;
  }
  __syncthreads();
  for (int k = tid; k < N; k += 64) bufA[k] = real_inv_pre_conj<N>(Y, k, P.tw);
  __syncthreads();
  const float2* R = fft_fwd<N, 64>(bufA, bufB, P.tw, tid);
  // y(2n) = Re z(n) / 4L, y(2n+1) = Im z(n) / 4L with z = conj(R)
  constexpr float scale = 1.0f / (float)(4 * L);
  float* old = reinterpret_cast<float*>(Y);   // 4L floats of room, 3L used
  float* st = ola + (int64_t)c * 3 * L;
  for (int n = tid; n < 3 * L; n += 64) old[n] = st[n];
  __syncthreads();
  float* o = out + (int64_t)c * out_stride;
  for (int n = tid; n < 4 * L; n += 64) {
    const float2 z = R[n >> 1];
    const float yv = ((n & 1) ? -z.y : z.x) * scale;
    if (n < L) {
      o[n] = old[n] + yv;
    } else if (n < 3 * L) {
      st[n - L] = old[n] + yv;
    } else {
      st[n - L] = yv;
    }
  }
  if (tid == 0 && sel_in != nullptr) sel_store[c] = sel_in[c];
  if (c == 0 && tid == 0) *counter = *counter + 1u;
}

// One workgroup per partition: spectra of the 2L-tap partitions of one IR.
template <int L, int DT>
__global__ __launch_bounds__(64) void k_irprep(DevPlan P, const float* __restrict__ taps, int32_t n_taps,
                                               typename Store<DT>::T* __restrict__ dst) {
  constexpr int N = 2 * L;
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int m = blockIdx.x;
  const int tid = threadIdx.x;
  for (int n = tid; n < L; n += 64) {
    const int t0 = 2 * L * m + 2 * n;
    const float h0 = (t0 < n_taps) ? taps[t0] : 0.f;
    const float h1 = (t0 + 1 < n_taps) ? taps[t0 + 1] : 0.f;
    bufA[n] = make_float2(h0, h1);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Z = fft_fwd<N, 64>(bufA, bufB, P.tw, tid);
  for (int k = tid; k < N; k += 64) dst[(int64_t)m * N + k] = pack<DT>(real_fwd_post<N>(Z, k, P.tw));
}

__global__ __launch_bounds__(256) void k_fill_zero(uint4* __restrict__ p, size_t n16, uint8_t* __restrict__ tail,
                                                   size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

// ---------------------------------------------------------------- dispatch helpers

template <int L, int DT>
hipError_t fwd_l(const DevPlan& P, const float* in, int64_t in_stride, float* hist, void* fdl,
                 const uint64_t* counter, hipStream_t s) {
  hipLaunchKernelGGL((k_fwd<L, DT>), dim3(P.I), dim3(64), 0, s, P, in, in_stride, hist,
                     static_cast<typename Store<DT>::T*>(fdl), counter);
  return hipGetLastError();
}

template <int DT>
hipError_t fwd_dt(const DevPlan& P, const float* in, int64_t in_stride, float* hist, void* fdl,
                  const uint64_t* counter, hipStream_t s) {
  switch (P.L) {
    case 64: return fwd_l<64, DT>(P, in, in_stride, hist, fdl, counter, s);
    case 128: return fwd_l<128, DT>(P, in, in_stride, hist, fdl, counter, s);
    case 256: return fwd_l<256, DT>(P, in, in_stride, hist, fdl, counter, s);
    case 512: return fwd_l<512, DT>(P, in, in_stride, hist, fdl, counter, s);
    default: return hipErrorInvalidValue;
  }
}

template <int V, int G, int NW, int DT>
hipError_t mac_inst(const DevPlan& P, const WorkItem* items, int n_items, const void* bank, const void* fdl,
                    const int32_t* sel, float2* ypart, const uint64_t* counter, hipStream_t s) {
  using ST = typename Store<DT>::T;
  hipLaunchKernelGGL((k_mac<V, G, NW, DT>), dim3(n_items), dim3(64 * NW), 0, s, P, items,
                     static_cast<const ST*>(bank), static_cast<const ST*>(fdl), sel, ypart, counter);
  return hipGetLastError();
}

template <int V, int G, int DT>
hipError_t mac_nw(const DevPlan& P, const MacShape& sh, const WorkItem* items, int n_items, const void* bank,
                  const void* fdl, const int32_t* sel, float2* ypart, const uint64_t* counter, hipStream_t s) {
  switch (sh.NW) {
    case 4: return mac_inst<V, G, 4, DT>(P, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 8: return mac_inst<V, G, 8, DT>(P, items, n_items, bank, fdl, sel, ypart, counter, s);
    default: return hipErrorInvalidValue;
  }
}

template <int V, int DT>
hipError_t mac_g(const DevPlan& P, const MacShape& sh, const WorkItem* items, int n_items, const void* bank,
                 const void* fdl, const int32_t* sel, float2* ypart, const uint64_t* counter, hipStream_t s) {
  switch (sh.G) {
    case 1: return mac_nw<V, 1, DT>(P, sh, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 2: return mac_nw<V, 2, DT>(P, sh, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 4: return mac_nw<V, 4, DT>(P, sh, items, n_items, bank, fdl, sel, ypart, counter, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
hipError_t mac_v(const DevPlan& P, const MacShape& sh, const WorkItem* items, int n_items, const void* bank,
                 const void* fdl, const int32_t* sel, float2* ypart, const uint64_t* counter, hipStream_t s) {
  switch (sh.V) {
    case 2: return mac_g<2, DT>(P, sh, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 4: return mac_g<4, DT>(P, sh, items, n_items, bank, fdl, sel, ypart, counter, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L>
hipError_t inv_l(const DevPlan& P, int TW, const float2* ypart, const int32_t* rows_ptr, const int32_t* rows,
                 float* ola, float* out, int64_t out_stride, const int32_t* sel_in, int32_t* sel_store,
                 uint64_t* counter, hipStream_t s) {
  hipLaunchKernelGGL((k_inv<L>), dim3(P.C), dim3(64), 0, s, P, TW, ypart, rows_ptr, rows, ola, out, out_stride,
                     sel_in, sel_store, counter);
  return hipGetLastError();
}

template <int L, int DT>
hipError_t irprep_l(const DevPlan& P, const float* taps, int32_t n_taps, int32_t M, void* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_irprep<L, DT>), dim3(M), dim3(64), 0, s, P, taps, n_taps,
                     static_cast<typename Store<DT>::T*>(dst));
  return hipGetLastError();
}

template <int DT>
hipError_t irprep_dt(const DevPlan& P, const float* taps, int32_t n_taps, int32_t M, void* dst, hipStream_t s) {
  switch (P.L) {
    case 64: return irprep_l<64, DT>(P, taps, n_taps, M, dst, s);
    case 128: return irprep_l<128, DT>(P, taps, n_taps, M, dst, s);
    case 256: return irprep_l<256, DT>(P, taps, n_taps, M, dst, s);
    case 512: return irprep_l<512, DT>(P, taps, n_taps, M, dst, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fwd(const DevPlan& P, int dtype, const float* in, int64_t in_stride, float* hist, void* fdl,
                      const uint64_t* counter, hipStream_t s) {
  switch (dtype) {
    case 0: return fwd_dt<0>(P, in, in_stride, hist, fdl, counter, s);
    case 1: return fwd_dt<1>(P, in, in_stride, hist, fdl, counter, s);
    case 2: return fwd_dt<2>(P, in, in_stride, hist, fdl, counter, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mac(const DevPlan& P, int dtype, const MacShape& shape, const WorkItem* items, int n_items,
                      const void* bank, const void* fdl, const int32_t* sel, float2* ypart,
                      const uint64_t* counter, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (dtype) {
    case 0: return mac_v<0>(P, shape, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 1: return mac_v<1>(P, shape, items, n_items, bank, fdl, sel, ypart, counter, s);
    case 2: return mac_v<2>(P, shape, items, n_items, bank, fdl, sel, ypart, counter, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_inv(const DevPlan& P, int tile_width, const float2* ypart, const int32_t* rows_ptr,
                      const int32_t* rows, float* ola, float* out, int64_t out_stride, const int32_t* sel_in,
                      int32_t* sel_store, uint64_t* counter, hipStream_t s) {
  switch (P.L) {
    case 64: return inv_l<64>(P, tile_width, ypart, rows_ptr, rows, ola, out, out_stride, sel_in, sel_store, counter, s);
    case 128: return inv_l<128>(P, tile_width, ypart, rows_ptr, rows, ola, out, out_stride, sel_in, sel_store, counter, s);
    case 256: return inv_l<256>(P, tile_width, ypart, rows_ptr, rows, ola, out, out_stride, sel_in, sel_store, counter, s);
    case 512: return inv_l<512>(P, tile_width, ypart, rows_ptr, rows, ola, out, out_stride, sel_in, sel_store, counter, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_irprep(const DevPlan& P, int dtype, const float* taps, int32_t n_taps, int32_t M, void* dst,
                         hipStream_t s) {
  switch (dtype) {
    case 0: return irprep_dt<0>(P, taps, n_taps, M, dst, s);
    case 1: return irprep_dt<1>(P, taps, n_taps, M, dst, s);
    case 2: return irprep_dt<2>(P, taps, n_taps, M, dst, s);
    default: return hipErrorInvalidValue;
  }
}

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

}  // namespace tvx
