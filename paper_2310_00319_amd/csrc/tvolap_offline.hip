// Offline (whole-signal) TVOLAP and its adjoint on gfx950 (Sec. 2 of Jaeger et
// al., arXiv 2310.00319, read as a linear map from (x, H) to y).
//
// Block b (b = 0 .. nblk-1) is the paper's block l = b - 1: it covers input
// samples [(b-1)L, (b+1)L) and its 4L-sample output lands at (b-1)L. Spectra
// are kept packed (2L complex values, slot 0 = (Re X(0), Re X(2L))).
//
// Forward:  X_b = DFT_4L(w . x_b)                         (eq. 1, 2, 4, 5)
//           Y_b = sum_m H_{g(b)}(m) X_{b-2m}                (eq. 8)
//           y   = overlap-add of IDFT_4L(Y_b) at hop L      (eq. 9-13)
// Adjoint (real loss, gradients written as dL/dRe + i dL/dIm):
//           G_b   = (c_k / 4L) DFT_4L(gy_b), c_k = 1 at k = 0, 2L, else 2
//           dH_s(m) = sum_{b: g(b) = s} G_b conj(X_{b-2m})
//           dX_j    = sum_m G_{j+2m} conj(H_{g(j+2m)}(m))
//           dxhat_j(n) = sum_{k <= 2L} Re(dX_j(k) e^{+i 2 pi n k / 4L}), n < 2L
//           dx(t)   = sum_j w(t - jL') dxhat_j(t - jL')     (windowed overlap-add)
// The input spectra X are recomputed from x in the backward pass instead of
// being kept from the forward pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/tvolap.h"
#include "fft_lds.hpp"

namespace tvx {
namespace off {
namespace {

using fft::cadd;
using fft::cconj;
using fft::cmul;
using fft::cscale;

constexpr int T = 256;   // threads per workgroup of the per-block kernels

struct Shape {
  int32_t L, C, K, M, nblk;
  int64_t N;
};

// Twiddles exp(-2 pi i t / 4L), evaluated in double precision and rounded to
// float, into LDS; the window (1 - cos(2 pi n / 2L)) / 2 = (1 - Re tw(2n)) / 2
// from them in float. Called by every thread of the workgroup.
template <int L>
__device__ __forceinline__ void make_tables(float2* twl, float* winl, int tid) {
  for (int t = tid; t < 4 * L; t += T) {
    double sn, cs;
    sincospi(-(double)t / (double)(2 * L), &sn, &cs);
    twl[t] = make_float2((float)cs, (float)sn);
  }
  if (winl) {
    __syncthreads();
    for (int n = tid; n < 2 * L; n += T) winl[n] = 0.5f * (1.0f - twl[2 * n].x);
  }
}

// packed product; bin 0 carries two real bins and multiplies component-wise
__device__ __forceinline__ float2 pmul(float2 a, float2 b, bool dc) {
  return dc ? make_float2(a.x * b.x, a.y * b.y) : cmul(a, b);
}
// packed product with the conjugate of b
__device__ __forceinline__ float2 pmulc(float2 a, float2 b, bool dc) {
  return dc ? make_float2(a.x * b.x, a.y * b.y) : cmul(a, cconj(b));
}

__device__ __forceinline__ int slot_of(const int32_t* sched, int b, int c, int C, int K) {
  if (!sched) return 0;
  int s = sched[(int64_t)b * C + c];
  return s < 0 ? 0 : (s >= K ? K - 1 : s);
}

// H [C][K][M][2L+1] complex -> packed Hp [C][K][M][2L]
__global__ __launch_bounds__(T) void k_pack(Shape S, const float2* __restrict__ H, float2* __restrict__ Hp) {
  const int N = 2 * S.L;
  const int64_t row = blockIdx.x;   // (c, s, m)
  const float2* src = H + row * (N + 1);
  float2* dst = Hp + row * N;
  for (int k = threadIdx.x; k < N; k += T)
    dst[k] = (k == 0) ? make_float2(src[0].x, src[N].x) : src[k];
}

// Spectra of blocks b = xb0 + blockIdx.x of x[c] (windowed, zero padded,
// transformed; packed) -> Xbuf[c][b - xb0] (xn rows per channel).
template <int L>
__global__ __launch_bounds__(T) void k_spectra(Shape S, const float* __restrict__ x, float2* __restrict__ Xbuf,
                                               int32_t xb0, int32_t xn) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int b = xb0 + (int)blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  make_tables<L>(twl, winl, tid);
  __syncthreads();
  const float* xc = x + (int64_t)c * S.N;
  const int64_t t0 = (int64_t)(b - 1) * L;
  for (int n = tid; n < L; n += T) {
    const int64_t ta = t0 + 2 * n, tb = ta + 1;
    const float s0 = (ta >= 0 && ta < S.N) ? xc[ta] : 0.f;
    const float s1 = (tb >= 0 && tb < S.N) ? xc[tb] : 0.f;
    bufA[n] = make_float2(winl[2 * n] * s0, winl[2 * n + 1] * s1);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  float2* dst = Xbuf + ((int64_t)c * xn + blockIdx.x) * N;
  for (int k = tid; k < N; k += T) dst[k] = fft::real_fwd_post<N>(Z, k, twl);
}

// y_b = IDFT_4L(sum_m H_{g(b)}(m) X_{b-2m}) for blocks b = bb0 + blockIdx.x ->
// yb[c][b - bb0][4L]. H is read in the caller's layout [C][K][M][2L+1]; the
// packed bin 0 product takes Re H(0) and Re H(2L). Xbuf holds the spectra of
// blocks xb0 .. xb0 + xn - 1 of each channel, which covers every b - 2m >= 0.
template <int L>
__global__ __launch_bounds__(T) void k_fwd_blocks(Shape S, const float2* __restrict__ H,
                                                  const float2* __restrict__ Xbuf, int32_t xb0, int32_t xn,
                                                  const int32_t* __restrict__ sched, float* __restrict__ yb,
                                                  int32_t bb0, int32_t bn) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float2 Y[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int b = bb0 + (int)blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  make_tables<L>(twl, nullptr, tid);
  const int s = slot_of(sched, b, c, S.C, S.K);
  const float2* Hc = H + (((int64_t)c * S.K + s) * S.M) * (N + 1);
  const float2* X = Xbuf + ((int64_t)c * xn - xb0) * N;
  for (int k = tid; k < N; k += T) {
    float2 acc = make_float2(0.f, 0.f);
    for (int m = 0; m < S.M && b - 2 * m >= 0; ++m) {
      const float2* h = Hc + (int64_t)m * (N + 1);
      const float2 hk = (k == 0) ? make_float2(h[0].x, h[N].x) : h[k];
      acc = cadd(acc, pmul(hk, X[(int64_t)(b - 2 * m) * N + k], k == 0));
    }
    Y[k] = acc;
  }
  __syncthreads();
  for (int k = tid; k < N; k += T) bufA[k] = fft::real_inv_pre_conj<N>(Y, k, twl);
  __syncthreads();
  const float2* R = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  constexpr float scale = 1.0f / (float)(4 * L);
  float* dst = yb + ((int64_t)c * bn + blockIdx.x) * 4 * L;
  for (int n = tid; n < 4 * L; n += T) {
    const float2 z = R[n >> 1];
    dst[n] = ((n & 1) ? -z.y : z.x) * scale;
  }
}

// y[c][t] for t in [t0, t1) = sum over the (up to four) blocks whose output
// covers t, oldest first; yb holds blocks bb0 .. bb0 + bn - 1, which covers
// every block that meets [t0, t1).
__global__ __launch_bounds__(T) void k_ola(Shape S, const float* __restrict__ yb, int32_t bb0, int32_t bn,
                                           int64_t t0, int64_t t1, float* __restrict__ y) {
  const int c = blockIdx.y;
  const int L = S.L;
  for (int64_t t = t0 + (int64_t)blockIdx.x * T + threadIdx.x; t < t1; t += (int64_t)gridDim.x * T) {
    const int64_t q = t / L;
    float acc = 0.f;
    for (int64_t b = q - 2; b <= q + 1; ++b) {
      if (b < 0 || b >= S.nblk) continue;
      const int64_t off = t - (b - 1) * L;
      if (off >= 0 && off < 4 * L) acc += yb[((int64_t)c * bn + (b - bb0)) * 4 * L + off];
    }
    y[(int64_t)c * S.N + t] = acc;
  }
}

// G_b = (c_k / 4L) DFT_4L(gy over [(b-1)L, (b+3)L)) for b = gb0 .. gb0 + gn - 1
// -> gspec[c][b - gb0][2L] (packed)
template <int L>
__global__ __launch_bounds__(T) void k_gspec(Shape S, const float* __restrict__ gy, float2* __restrict__ gspec,
                                             int32_t gb0, int32_t gn) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int b = gb0 + (int)blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  make_tables<L>(twl, nullptr, tid);
  const float* g = gy + (int64_t)c * S.N;
  const int64_t t0 = (int64_t)(b - 1) * L;
  for (int n = tid; n < N; n += T) {
    const int64_t ta = t0 + 2 * n, tb = ta + 1;
    bufA[n] = make_float2((ta >= 0 && ta < S.N) ? g[ta] : 0.f, (tb >= 0 && tb < S.N) ? g[tb] : 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  constexpr float end = 1.0f / (float)(4 * L);
  constexpr float mid = 2.0f / (float)(4 * L);
  float2* dst = gspec + ((int64_t)c * gn + blockIdx.x) * N;
  for (int k = tid; k < N; k += T) dst[k] = cscale(fft::real_fwd_post<N>(Z, k, twl), k == 0 ? end : mid);
}

// dH[c][s][m][k] (+)= sum over blocks b in [b0, b1) with g(b) = s and b - 2m >= 0
// of G_b(k) conj(X_{b-2m}(k)), written unpacked ([2L+1] bins); G_b at
// gspec[c][b - gb0], X_b at Xbuf[c][b - xb0]. acc = 0: the first segment
// writes, later ones add.
__global__ __launch_bounds__(T) void k_dH(Shape S, const float2* __restrict__ gspec, int32_t gb0, int32_t gn,
                                          const float2* __restrict__ Xbuf, int32_t xb0, int32_t xn,
                                          const int32_t* __restrict__ sched, int32_t b0, int32_t b1, int32_t acc_in,
                                          float2* __restrict__ dH) {
  const int N = 2 * S.L;
  const int64_t row = blockIdx.x;                    // (c, s, m)
  const int m = (int)(row % S.M);
  const int s = (int)((row / S.M) % S.K);
  const int c = (int)(row / ((int64_t)S.M * S.K));
  const float2* G = gspec + (int64_t)c * gn * N;
  const float2* X = Xbuf + (int64_t)c * xn * N;
  float2* dst = dH + row * (N + 1);
  for (int k = threadIdx.x; k < N; k += T) {
    float2 acc = make_float2(0.f, 0.f);
    for (int b = max(b0, 2 * m); b < b1; ++b) {
      if (slot_of(sched, b, c, S.C, S.K) != s) continue;
      acc = cadd(acc, pmulc(G[(int64_t)(b - gb0) * N + k], X[(int64_t)(b - 2 * m - xb0) * N + k], k == 0));
    }
    if (k == 0) {
      float2 d0 = make_float2(acc.x, 0.f), dn = make_float2(acc.y, 0.f);
      if (acc_in) { d0.x += dst[0].x; dn.x += dst[N].x; }
      dst[0] = d0;
      dst[N] = dn;
    } else {
      dst[k] = acc_in ? cadd(dst[k], acc) : acc;
    }
  }
}

// dxhat_j = w . (first 2L samples of the R2C adjoint of dX_j) for j = j0 ..
// j0 + jn - 1 -> dxb[c][j - j0][2L]; G_b at gspec[c][b - gb0] for every
// b = j + 2m < nblk
template <int L>
__global__ __launch_bounds__(T) void k_dx_blocks(Shape S, const float2* __restrict__ gspec, int32_t gb0, int32_t gn,
                                                 const float2* __restrict__ Hp, const int32_t* __restrict__ sched,
                                                 float* __restrict__ dxb, int32_t j0, int32_t jn) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float winl[N];
  __shared__ float2 D[N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int j = j0 + (int)blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  make_tables<L>(twl, winl, tid);
  const float2* G = gspec + (int64_t)c * gn * N;
  for (int k = tid; k < N; k += T) {
    float2 acc = make_float2(0.f, 0.f);
    for (int m = 0; m < S.M && j + 2 * m < S.nblk; ++m) {
      const int b = j + 2 * m;
      const int s = slot_of(sched, b, c, S.C, S.K);
      const float2* H = Hp + (((int64_t)c * S.K + s) * S.M + m) * N;
      acc = cadd(acc, pmulc(G[(int64_t)(b - gb0) * N + k], H[k], k == 0));
    }
    // sum_k Re(D(k) e^{+i theta}) over the 2L + 1 bins equals the normalised
    // inverse real DFT of D scaled by 4L at k = 0, 2L and by 2L elsewhere
    D[k] = (k == 0) ? cscale(acc, (float)(4 * L)) : cscale(acc, (float)(2 * L));
  }
  __syncthreads();
  for (int k = tid; k < N; k += T) bufA[k] = fft::real_inv_pre_conj<N>(D, k, twl);
  __syncthreads();
  const float2* R = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  constexpr float scale = 1.0f / (float)(4 * L);
  float* dst = dxb + ((int64_t)c * jn + blockIdx.x) * N;
  for (int n = tid; n < N; n += T) {
    const float2 z = R[n >> 1];
    dst[n] = winl[n] * ((n & 1) ? -z.y : z.x) * scale;
  }
}

// dx[c][t] for t in [t0, t1) = sum of the two windowed blocks that cover t
// (blocks q and q + 1 for t in hop q, both in dxb = blocks j0 .. j0 + jn - 1)
__global__ __launch_bounds__(T) void k_dx_ola(Shape S, const float* __restrict__ dxb, int32_t j0, int32_t jn,
                                              int64_t t0, int64_t t1, float* __restrict__ dx) {
  const int c = blockIdx.y;
  const int L = S.L;
  const int N = 2 * L;
  for (int64_t t = t0 + (int64_t)blockIdx.x * T + threadIdx.x; t < t1; t += (int64_t)gridDim.x * T) {
    const int64_t q = t / L;
    float acc = 0.f;
    for (int64_t j = q; j <= q + 1; ++j) {
      if (j < 0 || j >= S.nblk) continue;
      const int64_t off = t - (j - 1) * L;
      if (off >= 0 && off < N) acc += dxb[((int64_t)c * jn + (j - j0)) * N + off];
    }
    dx[(int64_t)c * S.N + t] = acc;
  }
}

// IR spectra for the offline path: taps [C][K][n_taps] -> H [C][K][M][2L+1]
template <int L>
__global__ __launch_bounds__(T) void k_ir_spectra(Shape S, const float* __restrict__ taps, int32_t n_taps,
                                                  float2* __restrict__ H) {
  constexpr int N = 2 * L;
  __shared__ float2 twl[2 * N];
  __shared__ float2 bufA[N];
  __shared__ float2 bufB[N];
  const int64_t row = blockIdx.x;     // (c, s, m)
  const int m = (int)(row % S.M);
  const int64_t cs = row / S.M;
  const int tid = threadIdx.x;
  make_tables<L>(twl, nullptr, tid);
  const float* h = taps + cs * n_taps;
  for (int n = tid; n < L; n += T) {
    const int t0 = N * m + 2 * n;
    bufA[n] = make_float2(t0 < n_taps ? h[t0] : 0.f, t0 + 1 < n_taps ? h[t0 + 1] : 0.f);
    bufA[n + L] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<N, T>(bufA, bufB, twl, tid);
  float2* dst = H + row * (N + 1);
  for (int k = tid; k < N; k += T) {
    const float2 v = fft::real_fwd_post<N>(Z, k, twl);
    if (k == 0) {
      dst[0] = make_float2(v.x, 0.f);
      dst[N] = make_float2(v.y, 0.f);
    } else {
      dst[k] = v;
    }
  }
}

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

// ---------------------------------------------------------------- host side

struct Workspace {
  float2* Hp;      // [C][K][M][2L]
  float2* Xbuf;    // [C][nx][2L] input spectra of one segment
  float2* Gbuf;    // [C][nx][2L] gradient spectra of one segment
  float* blk;      // [C][nq + 4][4L] forward output blocks / windowed gradient blocks of one segment
};

int64_t align_up(int64_t v) { return (v + 255) & ~(int64_t)255; }

// Hops per segment of the workspace forms: the working memory grows with the
// segment, not with the signal (a segment of nq hops holds the spectra of
// nq + 4 + 2(M - 1) blocks per channel).
constexpr int64_t kSegHops = 1024;
int64_t seg_hops(const Shape& S) { return std::min<int64_t>((int64_t)S.nblk - 1, kSegHops); }

int64_t workspace_layout(const Shape& S, Workspace* w, char* base) {
  const int N = 2 * S.L;
  const int64_t nq = seg_hops(S);
  const int64_t nx = nq + 4 + 2 * ((int64_t)S.M - 1);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const int64_t o_hp = take((int64_t)S.C * S.K * S.M * N * 8);
  const int64_t o_x = take((int64_t)S.C * nx * N * 8);
  const int64_t o_g = take((int64_t)S.C * nx * N * 8);
  const int64_t o_b = take((int64_t)S.C * (nq + 4) * 4 * S.L * 4);
  if (w && base) {
    w->Hp = reinterpret_cast<float2*>(base + o_hp);
    w->Xbuf = reinterpret_cast<float2*>(base + o_x);
    w->Gbuf = reinterpret_cast<float2*>(base + o_g);
    w->blk = reinterpret_cast<float*>(base + o_b);
  }
  return off;
}

// Forward over output segments. Segment [Q0, Q1) of hop indices writes the
// samples [Q0 L, Q1 L) of y; they are covered by blocks [Q0 - 2, Q1 + 2), whose
// products need spectra from 2(M - 1) blocks earlier. Each sample is summed by
// one thread in the same order whatever the segment length, so results do not
// depend on it.
struct Segment {
  int32_t bb0, bn, xb0, xn;
  int64_t t0, t1;
};

Segment segment(const Shape& S, int64_t Q0, int64_t nq) {
  const int64_t Q1 = std::min<int64_t>(Q0 + nq, (int64_t)S.nblk - 1);
  Segment g;
  const int64_t bb0 = std::max<int64_t>(0, Q0 - 2), bb1 = std::min<int64_t>(S.nblk, Q1 + 2);
  const int64_t xb0 = std::max<int64_t>(0, bb0 - 2 * ((int64_t)S.M - 1));
  g.bb0 = (int32_t)bb0;
  g.bn = (int32_t)(bb1 - bb0);
  g.xb0 = (int32_t)xb0;
  g.xn = (int32_t)(bb1 - xb0);
  g.t0 = Q0 * S.L;
  g.t1 = std::min<int64_t>(S.N, Q1 * S.L);
  return g;
}

// Scratch bytes of segments of nq hop indices: spectra of nq + 4 + 2(M - 1)
// blocks and 4L output samples of nq + 4 blocks per channel.
int64_t segment_bytes(const Shape& S, int64_t nq) {
  const int64_t nb = nq + 4, nx = nb + 2 * ((int64_t)S.M - 1);
  return align_up((int64_t)S.C * nx * 2 * S.L * 8) + (int64_t)S.C * nb * 4 * S.L * 4;
}

hipError_t forward_segments(const Shape& S, const float* x, const float2* H, const int32_t* sched, float* y,
                            float2* Xbuf, float* yb, int64_t nq, hipStream_t st) {
  return by_hop(S.L, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    for (int64_t Q0 = 0; Q0 < (int64_t)S.nblk - 1; Q0 += nq) {
      const Segment g = segment(S, Q0, nq);
      if (g.t0 >= g.t1) break;
      const unsigned ola_x = (unsigned)std::min<int64_t>((g.t1 - g.t0 + T - 1) / T, 65535);
      hipLaunchKernelGGL((k_spectra<L>), dim3(g.xn, S.C), dim3(T), 0, st, S, x, Xbuf, g.xb0, g.xn);
      hipLaunchKernelGGL((k_fwd_blocks<L>), dim3(g.bn, S.C), dim3(T), 0, st, S, H, Xbuf, g.xb0, g.xn, sched, yb,
                         g.bb0, g.bn);
      hipLaunchKernelGGL(k_ola, dim3(ola_x, S.C), dim3(T), 0, st, S, yb, g.bb0, g.bn, g.t0, g.t1, y);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
}

}  // namespace off
}  // namespace tvx

using tvx::off::Shape;
using tvx::off::Workspace;

// Working memory of tvolap_offline_forward_noalloc: one array per GPU, placed
// by the code-object loader and kept until the process ends. Host code never
// passes the array's name to a kernel: it is the host-side stand-in of the
// symbol; the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[TVOLAP_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local const char* g_off_err = "no error";

int off_fail(int code, const char* msg) {
  g_off_err = msg;
  return code;
}

int check_shape(const tvolap_offline_shape* sh, Shape* S) {
  if (!sh) return off_fail(TVOLAP_EINVAL, "shape is NULL");
  if (!(sh->hop == 64 || sh->hop == 128 || sh->hop == 256 || sh->hop == 512))
    return off_fail(TVOLAP_EINVAL, "hop must be 64, 128, 256 or 512");
  if (sh->n_channels < 1 || sh->n_partitions < 1 || sh->n_slots < 1 || sh->n_samples < 1)
    return off_fail(TVOLAP_EINVAL, "n_channels, n_partitions, n_slots and n_samples must be >= 1");
  if (sh->n_channels > 65535) return off_fail(TVOLAP_EINVAL, "n_channels must be <= 65535");
  const int64_t nblk = (sh->n_samples + sh->hop - 1) / sh->hop + 1;
  if (nblk > (1 << 30)) return off_fail(TVOLAP_EINVAL, "n_samples too large");
  S->L = sh->hop;
  S->C = sh->n_channels;
  S->K = sh->n_slots;
  S->M = sh->n_partitions;
  S->N = sh->n_samples;
  S->nblk = (int32_t)nblk;
  return TVOLAP_OK;
}

int prepare(const Shape& S, void* ws, int64_t ws_bytes, Workspace* w) {
  if (!ws) return off_fail(TVOLAP_EINVAL, "workspace is NULL");
  if (ws_bytes < tvx::off::workspace_layout(S, nullptr, nullptr)) return off_fail(TVOLAP_EINVAL, "workspace too small");
  tvx::off::workspace_layout(S, w, static_cast<char*>(ws));
  return TVOLAP_OK;
}

// Device address of `scratch` on the current device, looked up on the first
// call on that device (with it current) and kept per device.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;

int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return off_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return off_fail(TVOLAP_EDEVICE, "hipGetSymbolAddress of the static scratch failed");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return TVOLAP_OK;
}

}  // namespace

extern "C" {

const char* tvolap_offline_last_error(void) { return g_off_err; }

int64_t tvolap_offline_workspace_bytes(const tvolap_offline_shape* shape) {
  Shape S;
  if (check_shape(shape, &S) != TVOLAP_OK) return -1;
  return tvx::off::workspace_layout(S, nullptr, nullptr);
}

int tvolap_offline_ir_spectra(const tvolap_offline_shape* shape, const float* taps, int32_t n_taps, float* H,
                              void* stream) {
  Shape S;
  if (int rc = check_shape(shape, &S)) return rc;
  if (!taps || !H) return off_fail(TVOLAP_EINVAL, "taps or H is NULL");
  if (n_taps < 1 || n_taps > 2 * S.L * S.M) return off_fail(TVOLAP_EINVAL, "n_taps outside [1, 2L M]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = tvx::off::by_hop(S.L, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    hipLaunchKernelGGL((tvx::off::k_ir_spectra<L>), dim3((unsigned)((int64_t)S.C * S.K * S.M)), dim3(tvx::off::T),
                       0, st, S, taps, n_taps, reinterpret_cast<float2*>(H));
    return hipGetLastError();
  });
  if (e != hipSuccess) return off_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

int tvolap_offline_forward(const tvolap_offline_shape* shape, const float* x, const float* H,
                           const int32_t* schedule, float* y, void* workspace, int64_t workspace_bytes,
                           void* stream) {
  Shape S;
  if (int rc = check_shape(shape, &S)) return rc;
  if (!x || !H || !y) return off_fail(TVOLAP_EINVAL, "x, H or y is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w;
  if (int rc = prepare(S, workspace, workspace_bytes, &w)) return rc;
  const hipError_t e = tvx::off::forward_segments(S, x, reinterpret_cast<const float2*>(H), schedule, y, w.Xbuf,
                                                  w.blk, tvx::off::seg_hops(S), st);
  if (e != hipSuccess) return off_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

int tvolap_offline_backward(const tvolap_offline_shape* shape, const float* x, const float* H,
                            const int32_t* schedule, const float* gy, float* dx, float* dH, void* workspace,
                            int64_t workspace_bytes, void* stream) {
  Shape S;
  if (int rc = check_shape(shape, &S)) return rc;
  if (!x || !H || !gy) return off_fail(TVOLAP_EINVAL, "x, H or gy is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w;
  if (int rc = prepare(S, workspace, workspace_bytes, &w)) return rc;
  const unsigned rows = (unsigned)((int64_t)S.C * S.K * S.M);
  const int64_t nq = tvx::off::seg_hops(S);
  const int64_t M2 = 2 * ((int64_t)S.M - 1);
  const hipError_t e = tvx::off::by_hop(S.L, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    using namespace tvx::off;
    hipLaunchKernelGGL(k_pack, dim3(rows), dim3(T), 0, st, S, reinterpret_cast<const float2*>(H), w.Hp);
    // Segments of hops [Q0, Q1): dx over their samples (windowed blocks Q0 ..
    // Q1, each from the gradient spectra of the blocks j + 2m after it), dH
    // over the blocks [Q0, Q1) (the last segment also takes block nblk - 1),
    // with the input spectra of 2(M - 1) blocks before them recomputed from x.
    for (int64_t Q0 = 0; Q0 < (int64_t)S.nblk - 1; Q0 += nq) {
      const int64_t Q1 = std::min<int64_t>(Q0 + nq, (int64_t)S.nblk - 1);
      const int64_t hb1 = (Q1 == (int64_t)S.nblk - 1) ? S.nblk : Q1;       // dH blocks [Q0, hb1)
      const int64_t jb1 = std::min<int64_t>(S.nblk, Q1 + 1);                // dx blocks [Q0, jb1)
      const int64_t gb1 = std::min<int64_t>(S.nblk, std::max(hb1, jb1 + M2));  // gradient spectra [Q0, gb1)
      const int64_t xb0 = std::max<int64_t>(0, Q0 - M2);                     // input spectra [xb0, hb1)
      const int32_t gn = (int32_t)(gb1 - Q0), xn = (int32_t)(hb1 - xb0), jn = (int32_t)(jb1 - Q0);
      hipLaunchKernelGGL((k_gspec<L>), dim3(gn, S.C), dim3(T), 0, st, S, gy, w.Gbuf, (int32_t)Q0, gn);
      if (dH) {
        hipLaunchKernelGGL((k_spectra<L>), dim3(xn, S.C), dim3(T), 0, st, S, x, w.Xbuf, (int32_t)xb0, xn);
        hipLaunchKernelGGL(k_dH, dim3(rows), dim3(T), 0, st, S, w.Gbuf, (int32_t)Q0, gn, w.Xbuf, (int32_t)xb0, xn,
                           schedule, (int32_t)Q0, (int32_t)hb1, (int32_t)(Q0 > 0), reinterpret_cast<float2*>(dH));
      }
      if (dx) {
        const int64_t t0 = Q0 * S.L, t1 = std::min<int64_t>(S.N, Q1 * S.L);
        const unsigned ola_x = (unsigned)std::min<int64_t>((t1 - t0 + T - 1) / T, 65535);
        hipLaunchKernelGGL((k_dx_blocks<L>), dim3(jn, S.C), dim3(T), 0, st, S, w.Gbuf, (int32_t)Q0, gn, w.Hp,
                           schedule, w.blk, (int32_t)Q0, jn);
        hipLaunchKernelGGL(k_dx_ola, dim3(ola_x, S.C), dim3(T), 0, st, S, w.blk, (int32_t)Q0, jn, t0, t1, dx);
      }
      const hipError_t le = hipGetLastError();
      if (le != hipSuccess) return le;
    }
    return hipSuccess;
  });
  if (e != hipSuccess) return off_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

int tvolap_offline_forward_noalloc(const tvolap_offline_shape* shape, const float* x, const float* H,
                                   const int32_t* schedule, float* y, void* stream) {
  Shape S;
  if (int rc = check_shape(shape, &S)) return rc;
  if (!x || !H || !y) return off_fail(TVOLAP_EINVAL, "x, H or y is NULL");
  const int64_t cap = TVOLAP_NOALLOC_SCRATCH_BYTES;
  if (tvx::off::segment_bytes(S, 1) > cap)
    return off_fail(TVOLAP_EINVAL,
                    "shape too large for the static scratch: one hop per segment needs C (2M + 8) 16L bytes, "
                    "more than TVOLAP_NOALLOC_SCRATCH_BYTES");
  // the longest segment that fits
  int64_t lo = 1, hi = (int64_t)S.nblk - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (tvx::off::segment_bytes(S, mid) <= cap) lo = mid; else hi = mid - 1;
  }
  const int64_t nq = lo;
  void* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  const int64_t nx = nq + 4 + 2 * ((int64_t)S.M - 1);
  float2* Xbuf = static_cast<float2*>(base);
  float* yb = reinterpret_cast<float*>(static_cast<char*>(base) +
                                       tvx::off::align_up((int64_t)S.C * nx * 2 * S.L * 8));
  const hipError_t e = tvx::off::forward_segments(S, x, reinterpret_cast<const float2*>(H), schedule, y, Xbuf, yb,
                                                  nq, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return off_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

}  // extern "C"
