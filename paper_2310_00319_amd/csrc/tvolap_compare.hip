// The comparison algorithms of Sec. 3 (Jaeger et al., arXiv 2310.00319) on
// gfx950, offline over whole signals, on the same LDS transforms as TVOLAP:
// block convolution by overlap-add (OLA) and overlap-save (OLS), weighted
// overlap-add (WOLA) with block B = N_IR (FFT 2B), and the cross-faded direct
// time-domain convolution (CF-TDC).
//
// Block methods, per (channel, block):
//   OLA   x[jB, (j+1)B) zero padded to 2B         -> 2B samples added at jB
//   OLS   x[(j-1)B, (j+1)B)                        -> last B samples at jB
//   WOLA  analysis window . x[jR, jR + B), R = B/2 -> synthesis window, at jR
//         (rectangular synthesis: all 2B samples; square-root Hann: the first
//         B samples weighted, the rest dropped)
// each multiplied in the frequency domain with the 2B-point spectrum of the
// response active in the block, then summed per output sample over the blocks
// that cover it, oldest first.
// CF-TDC: sum_s c_s(t) (x * h_s)(t), c_s the Hann cross-fade of L samples on
// TVOLAP's block grid, the convolutions evaluated directly (FP32 sums).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "../../include/tvolap.h"
#include "fft_lds.hpp"

namespace tvx {
namespace cmpk {
namespace {

using fft::cmul;

constexpr int T = 256;

struct CShape {
  int32_t method, B, C, K, n_taps, analysis, synthesis, nblk;
  int64_t N;
};

// exp(-2 pi i t / 2B) for t < 2B, from double precision
template <int B>
__global__ __launch_bounds__(T) void k_cmp_tw(float2* __restrict__ tw) {
  for (int t = threadIdx.x; t < 2 * B; t += T) {
    double sn, cs;
    sincospi(-(double)t / (double)B, &sn, &cs);
    tw[t] = make_float2((float)cs, (float)sn);
  }
}

// Window value at n < B from the twiddle table: Hann (1 - cos(2 pi n / B)) / 2
// = (1 - Re tw[2n]) / 2; square-root Hann sin(pi n / B) = -Im tw[n].
template <int B>
__device__ __forceinline__ float win(int kind, int n, const float2* twl) {
  if (kind == TVOLAP_WIN_HANN) return 0.5f * (1.0f - twl[2 * n].x);
  if (kind == TVOLAP_WIN_SQRT_HANN) return -twl[n].y;
  return 1.0f;
}

// Packed 2B-point spectra of the responses: Hp[c][s][B] from taps[c][s][n_taps].
template <int B>
__global__ __launch_bounds__(T) void k_cmp_spectra(CShape S, const float* __restrict__ taps,
                                                   const float2* __restrict__ tw, float2* __restrict__ Hp) {
  __shared__ float2 twl[2 * B];
  __shared__ float2 bufA[B];
  __shared__ float2 bufB[B];
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;    // (c, s)
  for (int t = tid; t < 2 * B; t += T) twl[t] = tw[t];
  const float* h = taps + row * S.n_taps;
  for (int n = tid; n < B; n += T) {
    const int t0 = 2 * n, t1 = 2 * n + 1;
    bufA[n] = make_float2(t0 < S.n_taps ? h[t0] : 0.f, t1 < S.n_taps ? h[t1] : 0.f);
  }
  __syncthreads();
  const float2* Z = fft::fft_fwd<B, T>(bufA, bufB, twl, tid);
  for (int k = tid; k < B; k += T) Hp[row * B + k] = fft::real_fwd_post<B>(Z, k, twl);
}

// One block of one channel: input segment, transform, product with the active
// response's spectrum, inverse, synthesis; yb[c][b][0 .. 2B).
template <int B>
__global__ __launch_bounds__(T) void k_cmp_blocks(CShape S, const float* __restrict__ x,
                                                  const float2* __restrict__ Hp, const int32_t* __restrict__ sched,
                                                  const float2* __restrict__ tw, float* __restrict__ yb) {
  __shared__ float2 twl[2 * B];
  __shared__ float2 bufA[B];
  __shared__ float2 bufB[B];
  __shared__ float2 Y[B];
  const int tid = threadIdx.x;
  const int b = blockIdx.x, c = blockIdx.y;
  for (int t = tid; t < 2 * B; t += T) twl[t] = tw[t];
  __syncthreads();
  const float* xc = x + (int64_t)c * S.N;
  // input start and length: OLA x[jB, jB + B); OLS x[(j-1)B, (j+1)B); WOLA
  // x[jR, jR + B) with j = b - 1 (blocks start at -R)
  int64_t t0;
  int len;
  if (S.method == TVOLAP_CMP_OLA) { t0 = (int64_t)b * B; len = B; }
  else if (S.method == TVOLAP_CMP_OLS) { t0 = (int64_t)(b - 1) * B; len = 2 * B; }
  else { t0 = (int64_t)(b - 1) * (B / 2); len = B; }
  const bool wola = S.method == TVOLAP_CMP_WOLA;
  for (int n = tid; n < B; n += T) {
    float v[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = 2 * n + e;
      const int64_t t = t0 + i;
      float s = (i < len && t >= 0 && t < S.N) ? xc[t] : 0.f;
      if (wola && i < B) s *= win<B>(S.analysis, i, twl);
      v[e] = s;
    }
    bufA[n] = make_float2(v[0], v[1]);
  }
  __syncthreads();
  int s = sched ? sched[(int64_t)b * S.C + c] : 0;
  s = s < 0 ? 0 : (s >= S.K ? S.K - 1 : s);
  const float2* H = Hp + ((int64_t)c * S.K + s) * B;
  const float2* Z = fft::fft_fwd<B, T>(bufA, bufB, twl, tid);
  for (int k = tid; k < B; k += T) {
    const float2 X = fft::real_fwd_post<B>(Z, k, twl);
    const float2 h = H[k];
    Y[k] = (k == 0) ? make_float2(X.x * h.x, X.y * h.y) : cmul(X, h);
  }
  __syncthreads();
  for (int k = tid; k < B; k += T) bufA[k] = fft::real_inv_pre_conj<B>(Y, k, twl);
  __syncthreads();
  const float2* R = fft::fft_fwd<B, T>(bufA, bufB, twl, tid);
  constexpr float scale = 1.0f / (float)(2 * B);
  float* dst = yb + ((int64_t)c * S.nblk + b) * 2 * B;
  for (int i = tid; i < 2 * B; i += T) {
    const float2 z = R[i >> 1];
    const float v = ((i & 1) ? -z.y : z.x) * scale;
    if (S.method == TVOLAP_CMP_OLS) {
      if (i >= B) dst[i - B] = v;                     // the samples free of wrap-around
    } else if (wola && S.synthesis == TVOLAP_WIN_SQRT_HANN) {
      dst[i] = (i < B) ? v * win<B>(TVOLAP_WIN_SQRT_HANN, i, twl) : 0.f;
    } else {
      dst[i] = v;
    }
  }
}

// y[c][t] = sum over the blocks that cover t, oldest first.
__global__ __launch_bounds__(T) void k_cmp_ola(CShape S, const float* __restrict__ yb, float* __restrict__ y) {
  const int c = blockIdx.y;
  const int B = S.B;
  int hop, span, first;   // block b starts at (b + first) * hop and covers span samples
  if (S.method == TVOLAP_CMP_OLA) { hop = B; span = 2 * B; first = 0; }
  else if (S.method == TVOLAP_CMP_OLS) { hop = B; span = B; first = 0; }
  else { hop = B / 2; span = (S.synthesis == TVOLAP_WIN_RECT) ? 2 * B : B; first = -1; }
  for (int64_t t = (int64_t)blockIdx.x * T + threadIdx.x; t < S.N; t += (int64_t)gridDim.x * T) {
    const int64_t q = t / hop;                         // latest block index j that starts at or before t
    float acc = 0.f;
    for (int64_t j = q - (span / hop - 1); j <= q; ++j) {
      const int64_t b = j - first;
      if (b < 0 || b >= S.nblk) continue;
      const int64_t off = t - j * hop;
      acc += yb[((int64_t)c * S.nblk + b) * 2 * B + off];
    }
    y[(int64_t)c * S.N + t] = acc;
  }
}

// CF-TDC: output tile of T samples per workgroup; the input window and the
// taps are staged through LDS in chunks of TAPS.
constexpr int TAPS = 1024;

__global__ __launch_bounds__(T) void k_cftdc(int32_t L, int32_t C, int32_t K, int64_t N, int32_t n_taps,
                                             const float* __restrict__ x, const float* __restrict__ taps,
                                             const int32_t* __restrict__ sched, float* __restrict__ y) {
  __shared__ float xs[TAPS + T];
  const int tid = threadIdx.x;
  const int c = blockIdx.y;
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int64_t t = t0 + tid;
  const int64_t q = t / L;
  const int n = (int)(t - q * L);
  // blocks q - 1 (second half of its window) and q (first half); schedule row
  // b is block b - 1
  const int64_t nb = (N + L - 1) / L + 1;
  auto slot = [&](int64_t row) {
    if (!sched || row < 0 || row >= nb) return 0;
    const int v = sched[row * C + c];
    return v < 0 ? 0 : (v >= K ? K - 1 : v);
  };
  const int sa = slot(q), sb = slot(q + 1);
  const float* ha = taps + ((int64_t)c * K + sa) * n_taps;
  const float* hb = taps + ((int64_t)c * K + sb) * n_taps;
  const float* xc = x + (int64_t)c * N;
  float za0 = 0.f, za1 = 0.f, zb0 = 0.f, zb1 = 0.f;
  for (int d0 = 0; d0 < n_taps; d0 += TAPS) {
    // xs[i] = x[t0 - d0 - TAPS + 1 + i] for i < TAPS + T - 1
    __syncthreads();
    for (int i = tid; i < TAPS + T - 1; i += T) {
      const int64_t u = t0 - d0 - TAPS + 1 + i;
      xs[i] = (u >= 0 && u < N) ? xc[u] : 0.f;
    }
    __syncthreads();
    const int dn = min(TAPS, n_taps - d0);
    // x[t - d] = xs[tid + TAPS - 1 - (d - d0)]
    int d = 0;
    for (; d + 1 < dn; d += 2) {
      const float x0 = xs[tid + TAPS - 1 - d], x1 = xs[tid + TAPS - 2 - d];
      za0 = fmaf(ha[d0 + d], x0, za0);
      za1 = fmaf(ha[d0 + d + 1], x1, za1);
      zb0 = fmaf(hb[d0 + d], x0, zb0);
      zb1 = fmaf(hb[d0 + d + 1], x1, zb1);
    }
    for (; d < dn; ++d) {
      const float x0 = xs[tid + TAPS - 1 - d];
      za0 = fmaf(ha[d0 + d], x0, za0);
      zb0 = fmaf(hb[d0 + d], x0, zb0);
    }
  }
  if (t < N) {
    // Hann window of length 2L (amplitude 1/2): block q - 1 at offset L + n,
    // block q at offset n
    const float wb = 0.5f * (1.0f - cospif((float)n / (float)L));
    const float wa = 1.0f - wb;
    y[(int64_t)c * N + t] = wa * (za0 + za1) + wb * (zb0 + zb1);
  }
}

template <typename F>
hipError_t by_block(int B, F&& f) {
  switch (B) {
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    case 2048: return f(std::integral_constant<int, 2048>{});
    default: return hipErrorInvalidValue;
  }
}

int64_t align_up(int64_t v) { return (v + 255) & ~(int64_t)255; }

// workspace: twiddles [2B] | packed spectra [C][K][B] | block outputs [C][nblk][2B]
int64_t layout(const CShape& S, float2** tw, float2** Hp, float** yb, char* base) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const int64_t o_tw = take((int64_t)2 * S.B * 8);
  const int64_t o_h = take((int64_t)S.C * S.K * S.B * 8);
  const int64_t o_y = take((int64_t)S.C * S.nblk * 2 * S.B * 4);
  if (base) {
    *tw = reinterpret_cast<float2*>(base + o_tw);
    *Hp = reinterpret_cast<float2*>(base + o_h);
    *yb = reinterpret_cast<float*>(base + o_y);
  }
  return off;
}

}  // namespace
}  // namespace cmpk
}  // namespace tvx

using tvx::cmpk::CShape;

namespace {

thread_local const char* g_cmp_err = "no error";

int cmp_fail(int code, const char* msg) {
  g_cmp_err = msg;
  return code;
}

int check_cmp(const tvolap_cmp_shape* sh, CShape* S) {
  if (!sh) return cmp_fail(TVOLAP_EINVAL, "shape is NULL");
  if (sh->method < TVOLAP_CMP_OLA || sh->method > TVOLAP_CMP_WOLA) return cmp_fail(TVOLAP_EINVAL, "unknown method");
  if (!(sh->block == 128 || sh->block == 256 || sh->block == 512 || sh->block == 1024 || sh->block == 2048))
    return cmp_fail(TVOLAP_EINVAL, "block must be 128, 256, 512, 1024 or 2048");
  if (sh->n_channels < 1 || sh->n_channels > 65535 || sh->n_slots < 1 || sh->n_samples < 1)
    return cmp_fail(TVOLAP_EINVAL, "n_channels in [1, 65535], n_slots >= 1 and n_samples >= 1");
  if (sh->n_taps < 1 || sh->n_taps > sh->block) return cmp_fail(TVOLAP_EINVAL, "n_taps must be in [1, block]");
  if (sh->method == TVOLAP_CMP_WOLA) {
    if (sh->analysis != TVOLAP_WIN_HANN && sh->analysis != TVOLAP_WIN_SQRT_HANN)
      return cmp_fail(TVOLAP_EINVAL, "WOLA analysis window must be Hann or square-root Hann");
    if (sh->synthesis != TVOLAP_WIN_RECT && sh->synthesis != TVOLAP_WIN_SQRT_HANN)
      return cmp_fail(TVOLAP_EINVAL, "WOLA synthesis window must be rectangular or square-root Hann");
  }
  const int64_t hop = sh->method == TVOLAP_CMP_WOLA ? sh->block / 2 : sh->block;
  const int64_t nblk = (sh->n_samples + hop - 1) / hop + (sh->method == TVOLAP_CMP_WOLA ? 1 : 0);
  if (nblk > (1 << 30)) return cmp_fail(TVOLAP_EINVAL, "n_samples too large");
  S->method = sh->method;
  S->B = sh->block;
  S->C = sh->n_channels;
  S->K = sh->n_slots;
  S->n_taps = sh->n_taps;
  S->analysis = sh->analysis;
  S->synthesis = sh->synthesis;
  S->N = sh->n_samples;
  S->nblk = (int32_t)nblk;
  return TVOLAP_OK;
}

}  // namespace

extern "C" {

const char* tvolap_cmp_last_error(void) { return g_cmp_err; }

int64_t tvolap_cmp_blocks(const tvolap_cmp_shape* shape) {
  CShape S;
  if (check_cmp(shape, &S) != TVOLAP_OK) return -1;
  return S.nblk;
}

int64_t tvolap_cmp_workspace_bytes(const tvolap_cmp_shape* shape) {
  CShape S;
  if (check_cmp(shape, &S) != TVOLAP_OK) return -1;
  return tvx::cmpk::layout(S, nullptr, nullptr, nullptr, nullptr);
}

int tvolap_cmp_forward(const tvolap_cmp_shape* shape, const float* x, const float* taps, const int32_t* schedule,
                       float* y, void* workspace, int64_t workspace_bytes, void* stream) {
  CShape S;
  if (int rc = check_cmp(shape, &S)) return rc;
  if (!x || !taps || !y) return cmp_fail(TVOLAP_EINVAL, "x, taps or y is NULL");
  if (!workspace) return cmp_fail(TVOLAP_EINVAL, "workspace is NULL");
  if (workspace_bytes < tvx::cmpk::layout(S, nullptr, nullptr, nullptr, nullptr))
    return cmp_fail(TVOLAP_EINVAL, "workspace too small");
  float2* tw = nullptr;
  float2* Hp = nullptr;
  float* yb = nullptr;
  tvx::cmpk::layout(S, &tw, &Hp, &yb, static_cast<char*>(workspace));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned ola_x = (unsigned)std::min<int64_t>((S.N + tvx::cmpk::T - 1) / tvx::cmpk::T, 65535);
  const hipError_t e = tvx::cmpk::by_block(S.B, [&](auto Bc) {
    constexpr int B = decltype(Bc)::value;
    using namespace tvx::cmpk;
    hipLaunchKernelGGL((k_cmp_tw<B>), dim3(1), dim3(T), 0, st, tw);
    hipLaunchKernelGGL((k_cmp_spectra<B>), dim3((unsigned)(S.C * S.K)), dim3(T), 0, st, S, taps, tw, Hp);
    hipLaunchKernelGGL((k_cmp_blocks<B>), dim3(S.nblk, S.C), dim3(T), 0, st, S, x, Hp, schedule, tw, yb);
    hipLaunchKernelGGL(k_cmp_ola, dim3(ola_x, S.C), dim3(T), 0, st, S, yb, y);
    return hipGetLastError();
  });
  if (e != hipSuccess) return cmp_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

int tvolap_cftdc_forward(int32_t hop, int32_t n_channels, int32_t n_slots, int64_t n_samples, int32_t n_taps,
                         const float* x, const float* taps, const int32_t* schedule, float* y, void* stream) {
  if (hop < 1 || hop > 65536) return cmp_fail(TVOLAP_EINVAL, "hop must be in [1, 65536]");
  if (n_channels < 1 || n_channels > 65535 || n_slots < 1 || n_samples < 1 || n_taps < 1)
    return cmp_fail(TVOLAP_EINVAL, "n_channels in [1, 65535]; n_slots, n_samples, n_taps >= 1");
  if (!x || !taps || !y) return cmp_fail(TVOLAP_EINVAL, "x, taps or y is NULL");
  const int64_t tiles = (n_samples + tvx::cmpk::T - 1) / tvx::cmpk::T;
  if (tiles > INT32_MAX) return cmp_fail(TVOLAP_EINVAL, "n_samples too large");
  hipLaunchKernelGGL(tvx::cmpk::k_cftdc, dim3((unsigned)tiles, n_channels), dim3(tvx::cmpk::T), 0,
                     static_cast<hipStream_t>(stream), hop, n_channels, n_slots, n_samples, n_taps, x, taps, schedule,
                     y);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cmp_fail(TVOLAP_EDEVICE, hipGetErrorString(e));
  return TVOLAP_OK;
}

}  // extern "C"
