// LDS-resident FFT building blocks for gfx950 (device code only).
//
// A 4L-point real DFT (Sec. 2, eq. 4 and 6) is computed as an N = 2L point
// complex FFT of z(n) = x(2n) + i x(2n+1) followed by a split pass; the inverse
// (eq. 9) runs the split backwards and reuses the forward FFT on conjugated
// data. The complex FFT is a Stockham autosort FFT with radix-8/4 stages and
// one LDS ping-pong (and one barrier) per stage, run by T threads.
//
// Stored spectra are packed: 2L complex values, slot 0 = (Re X(0), Re X(2L)),
// slots 1 .. 2L-1 = X(k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvx {
namespace fft {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }  // a * (-i)
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }  // a * (+i)
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Small forward DFTs (sign -1).
template <int R> __device__ __forceinline__ void dft(float2 (&v)[R]);

template <> __device__ __forceinline__ void dft<4>(float2 (&v)[4]) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]));
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
  o[1] = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));   // * exp(-i pi/4)
  o[2] = cmul_mi(o[2]);                                                 // * exp(-i pi/2)
  o[3] = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));  // * exp(-3i pi/4)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// One radix-R stage of an N-point FFT by T threads; NS = product of the
// earlier radices; tw = exp(-2 pi i t / 2N) for t < 2N (in LDS).
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

// N-point forward complex FFT of `a` (LDS), `b` scratch. Callers synchronise
// before; returns the buffer holding the result, synchronised.
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
  } else if constexpr (N == 1024) {
    stage<1024, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<1024, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage<1024, 4, 64, T>(a, b, tw, tid); __syncthreads();
    stage<1024, 4, 256, T>(b, a, tw, tid); __syncthreads();
    return a;
  } else {
    static_assert(N == 2048, "unsupported FFT size");
    stage<2048, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage<2048, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage<2048, 8, 64, T>(a, b, tw, tid); __syncthreads();
    stage<2048, 4, 512, T>(b, a, tw, tid); __syncthreads();
    return a;
  }
}

// The same stages with a twiddle table of the transform's own length:
// tw[t] = exp(-2 pi i t / N) for t < N. The table of a 4L-point transform is
// the real-transform table of hop L, so a workgroup holding that table can
// run one complex 4L-point transform of two real signals at once.
template <int N, int R, int NS, int T>
__device__ __forceinline__ void stage_nat(const float2* __restrict__ src, float2* __restrict__ dst,
                                          const float2* __restrict__ tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
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
template <int N, int T>
__device__ __forceinline__ float2* fft_nat(float2* a, float2* b, const float2* tw, int tid) {
  if constexpr (N == 256) {
    stage_nat<256, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage_nat<256, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage_nat<256, 4, 64, T>(a, b, tw, tid); __syncthreads();
    return b;
  } else if constexpr (N == 512) {
    stage_nat<512, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage_nat<512, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage_nat<512, 8, 64, T>(a, b, tw, tid); __syncthreads();
    return b;
  } else if constexpr (N == 1024) {
    stage_nat<1024, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage_nat<1024, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage_nat<1024, 4, 64, T>(a, b, tw, tid); __syncthreads();
    stage_nat<1024, 4, 256, T>(b, a, tw, tid); __syncthreads();
    return a;
  } else {
    stage_nat<2048, 8, 1, T>(a, b, tw, tid); __syncthreads();
    stage_nat<2048, 8, 8, T>(b, a, tw, tid); __syncthreads();
    stage_nat<2048, 8, 64, T>(a, b, tw, tid); __syncthreads();
    stage_nat<2048, 4, 512, T>(b, a, tw, tid); __syncthreads();
    return a;
  }
}
// Packed bin k of the real 2N-point DFT from Z = FFT_N(x(2n) + i x(2n+1)).
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

// conj(Z'(k)) where the inverse N-point FFT of Z' interleaves the even and odd
// samples of 2N times the real inverse DFT of the packed spectrum Y.
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
  return cconj(cadd(S, cmul_pi(cmul(cconj(tw[k]), D))));
}

// Copy `n` float2 from global to LDS with T threads (all loads issued first).
template <int T>
__device__ __forceinline__ void copy_to_lds(float2* __restrict__ dst, const float2* __restrict__ src, int n, int tid) {
  for (int i = tid; i < n; i += T) dst[i] = src[i];
}

}  // namespace fft
}  // namespace tvx
