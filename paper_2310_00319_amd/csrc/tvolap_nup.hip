// TVOLAP with non-uniform partitions on gfx950: a head convolver of short
// partitions (hop L1, latency 2 L1) and a tail convolver of long partitions
// (hop L2 = r L1) whose output joins D = 2 L1 M1 samples later (Sec. 2 applied
// to each part of the response; non-uniform partitioning as in Sec. 1). The
// two parts run on two TVOLAP handles sharing one stream; these kernels move
// samples between them: each call's input into a ring that the tail reads r
// hops at a time, and the tail's output, one hop per call, into the output.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>

#include "../../include/tvolap.h"
#include "tvolap_internal.h"

namespace tvx {
namespace nupk {
namespace {

// ring[i][slot * L1 + n] = in[i * in_stride + n], n < L1
__global__ __launch_bounds__(256) void k_nup_stage(const float* __restrict__ in, int64_t in_stride,
                                                   float* __restrict__ ring, int64_t ring_stride, int32_t slot,
                                                   int32_t L1, int32_t I) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)I * L1) return;
  const int i = (int)(k / L1), n = (int)(k % L1);
  ring[i * ring_stride + (int64_t)slot * L1 + n] = in[i * in_stride + n];
}

// out[c * out_stride + n] += stage[c * L2 + off + n], n < L1
__global__ __launch_bounds__(256) void k_nup_add(float* __restrict__ out, int64_t out_stride,
                                                 const float* __restrict__ stage, int32_t L2, int32_t off, int32_t L1,
                                                 int32_t C) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)C * L1) return;
  const int c = (int)(k / L1), n = (int)(k % L1);
  out[c * out_stride + n] += stage[(int64_t)c * L2 + off + n];
}

// dst[c] = src[c], c < C
__global__ __launch_bounds__(256) void k_nup_copy_sel(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                      int32_t C) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c < C) dst[c] = src[c];
}

}  // namespace
}  // namespace nupk
}  // namespace tvx

struct tvolap_nup {
  tvolap_t* head = nullptr;
  tvolap_t* tail = nullptr;
  hipStream_t stream = nullptr;
  int32_t L1 = 0, L2 = 0, r = 1, M1 = 0, D = 0, C = 0, I = 0, K = 0, max_taps = 0;
  int32_t ring_slots = 0;     // hops of input kept per input (a multiple of r)
  float* d_ring = nullptr;    // [I][ring_slots * L1]
  float* d_stage = nullptr;   // [C][L2] output of the latest tail call
  int32_t* d_sel = nullptr;   // [C] latest device selection passed to a call
  bool dev_sel = false;       // the tail takes d_sel (else the handles' selection)
  int64_t calls = 0;          // calls issued (host side; graph replays keep the phase)
  bool capturing = false;
  int64_t capture_start = 0;
  std::string err = "no error";
};

namespace {

thread_local std::string g_nup_create_error = "no error";

int nfail(tvolap_nup_t* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_nup_create_error = msg;
  return code;
}

void nfree(tvolap_nup_t* h) {
  if (h->head) tvolap_destroy(h->head);
  if (h->tail) tvolap_destroy(h->tail);
  if (h->d_ring) (void)hipFree(h->d_ring);
  if (h->d_stage) (void)hipFree(h->d_stage);
  if (h->d_sel) (void)hipFree(h->d_sel);
  h->head = h->tail = nullptr;
  h->d_ring = h->d_stage = nullptr;
  h->d_sel = nullptr;
}

// head call index of tail call c2: r (c2 - 1) + 2 M1 + 1
int64_t first_tail_call(const tvolap_nup_t* h) { return 2LL * h->M1 + 1 - h->r; }

}  // namespace

extern "C" {

int tvolap_nup_create(const tvolap_nup_config* cfg, tvolap_nup_t** out) {
  if (!out) return nfail(nullptr, TVOLAP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return nfail(nullptr, TVOLAP_EINVAL, "cfg is NULL");
  const tvolap_config& b = cfg->base;
  const int r = cfg->tail_ratio;
  if (r < 1 || (r & (r - 1)) != 0) return nfail(nullptr, TVOLAP_EINVAL, "tail_ratio must be a power of two >= 1");
  const int64_t L2 = (int64_t)b.hop * r;
  if (!(b.hop == 64 || b.hop == 128 || b.hop == 256 || b.hop == 512) || L2 > 512)
    return nfail(nullptr, TVOLAP_EINVAL, "hop and hop * tail_ratio must be 64, 128, 256 or 512");
  if (cfg->head_partitions < 1 || cfg->head_partitions < r - 1)
    return nfail(nullptr, TVOLAP_EINVAL, "head_partitions must be >= max(1, tail_ratio - 1)");
  if (b.taps_of_channel) return nfail(nullptr, TVOLAP_EINVAL, "taps_of_channel must be NULL (one length for all)");
  if (b.n_outputs != 0) return nfail(nullptr, TVOLAP_EINVAL, "n_outputs must be 0");
  const int64_t D = 2LL * b.hop * cfg->head_partitions;
  if (D > INT32_MAX || b.max_taps < 1) return nfail(nullptr, TVOLAP_EINVAL, "head too long or max_taps < 1");
  tvolap_nup_t* h = new (std::nothrow) tvolap_nup_t();
  if (!h) return nfail(nullptr, TVOLAP_ENOMEM, "host allocation failed");
  h->L1 = b.hop;
  h->L2 = (int32_t)L2;
  h->r = r;
  h->M1 = cfg->head_partitions;
  h->D = (int32_t)D;
  h->C = b.n_channels;
  h->I = b.n_inputs;
  h->K = b.n_slots;
  h->max_taps = b.max_taps;
  h->stream = static_cast<hipStream_t>(b.stream);
  tvolap_config hc = b;
  hc.max_taps = (int32_t)D;
  hc.max_batch = 0;
  int rc = tvolap_create(&hc, &h->head);
  if (rc == TVOLAP_OK) {
    tvolap_config tc = b;
    tc.hop = (int32_t)L2;
    tc.max_taps = b.max_taps > D ? (int32_t)(b.max_taps - D) : 1;
    tc.max_batch = 0;
    rc = tvolap_create(&tc, &h->tail);
  }
  if (rc != TVOLAP_OK) {
    g_nup_create_error = tvolap_last_error(nullptr);
    nfree(h);
    delete h;
    return rc;
  }
  // the tail reads hops r c2 .. r c2 + r - 1 at head call r (c2 - 1) + 2 M1 + 1:
  // keep 2 M1 + 1 hops, rounded up to a multiple of r
  const int need = 2 * h->M1 + 1;
  h->ring_slots = ((need + r - 1) / r) * r;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->d_ring), (size_t)h->I * h->ring_slots * h->L1 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->d_stage), (size_t)h->C * h->L2 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->d_sel), (size_t)h->C * sizeof(int32_t));
  if (e == hipSuccess) e = tvx::launch_fill_zero(h->d_ring, (size_t)h->I * h->ring_slots * h->L1 * sizeof(float), h->stream);
  if (e == hipSuccess) e = tvx::launch_fill_zero(h->d_stage, (size_t)h->C * h->L2 * sizeof(float), h->stream);
  if (e == hipSuccess) e = tvx::launch_fill_zero(h->d_sel, (size_t)h->C * sizeof(int32_t), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    g_nup_create_error = std::string("device buffers: ") + hipGetErrorString(e);
    const int code = (e == hipErrorOutOfMemory) ? TVOLAP_ENOMEM : TVOLAP_EDEVICE;
    (void)hipGetLastError();
    nfree(h);
    delete h;
    return code;
  }
  *out = h;
  return TVOLAP_OK;
}

int tvolap_nup_destroy(tvolap_nup_t* h) {
  if (!h) return TVOLAP_OK;
  if (h->capturing) (void)tvolap_capture_end(h->head);
  (void)hipStreamSynchronize(h->stream);
  nfree(h);
  delete h;
  return TVOLAP_OK;
}

int tvolap_nup_set_ir(tvolap_nup_t* h, int32_t channel, int32_t slot, const float* taps, int32_t n_taps,
                      int32_t taps_on_device) {
  if (!h) return TVOLAP_EINVAL;
  if (channel < 0 || channel >= h->C) return nfail(h, TVOLAP_EINVAL, "channel out of range");
  if (slot < 0 || slot >= h->K) return nfail(h, TVOLAP_EINVAL, "slot out of range");
  if (n_taps < 0 || n_taps > h->max_taps) return nfail(h, TVOLAP_EINVAL, "n_taps outside [0, max_taps]");
  if (n_taps > 0 && !taps) return nfail(h, TVOLAP_EINVAL, "taps is NULL");
  const int32_t nh = n_taps < h->D ? n_taps : h->D;
  int rc = tvolap_set_ir(h->head, channel, slot, taps, nh, taps_on_device);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  rc = n_taps > h->D ? tvolap_set_ir(h->tail, channel, slot, taps + h->D, n_taps - h->D, taps_on_device)
                     : tvolap_set_ir(h->tail, channel, slot, nullptr, 0, taps_on_device);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->tail));
  return TVOLAP_OK;
}

int tvolap_nup_select_ir(tvolap_nup_t* h, const int32_t* slot_of_channel) {
  if (!h) return TVOLAP_EINVAL;
  int rc = tvolap_select_ir(h->head, slot_of_channel);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  rc = tvolap_select_ir(h->tail, slot_of_channel);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->tail));
  h->dev_sel = false;
  return TVOLAP_OK;
}

int tvolap_nup_process_block(tvolap_nup_t* h, const float* in, int64_t in_stride, float* out, int64_t out_stride,
                             const int32_t* slot_of_channel_dev) {
  if (!h) return TVOLAP_EINVAL;
  if (!in || !out) return nfail(h, TVOLAP_EINVAL, "in or out is NULL");
  if (in_stride < h->L1 || out_stride < h->L1) return nfail(h, TVOLAP_EINVAL, "stride smaller than hop");
  const int64_t c = h->calls;
  const int32_t slot = (int32_t)(c % h->ring_slots);
  const int64_t ring_stride = (int64_t)h->ring_slots * h->L1;
  hipLaunchKernelGGL(tvx::nupk::k_nup_stage, dim3((unsigned)(((int64_t)h->I * h->L1 + 255) / 256)), dim3(256), 0,
                     h->stream, in, in_stride, h->d_ring, ring_stride, slot, h->L1, h->I);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return nfail(h, TVOLAP_EDEVICE, hipGetErrorString(e));
  if (slot_of_channel_dev) {
    hipLaunchKernelGGL(tvx::nupk::k_nup_copy_sel, dim3((unsigned)((h->C + 255) / 256)), dim3(256), 0, h->stream,
                       h->d_sel, slot_of_channel_dev, h->C);
    e = hipGetLastError();
    if (e != hipSuccess) return nfail(h, TVOLAP_EDEVICE, hipGetErrorString(e));
    h->dev_sel = true;
  }
  int rc = tvolap_process_block(h->head, in, in_stride, out, out_stride, slot_of_channel_dev);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  const int64_t c0 = first_tail_call(h);
  if (c >= c0 && (c - c0) % h->r == 0) {
    // tail call c2 = (c - c0) / r reads input hops r c2 .. r c2 + r - 1
    const int64_t c2 = (c - c0) / h->r;
    const int32_t s0 = (int32_t)((c2 * h->r) % h->ring_slots);
    rc = tvolap_process_block(h->tail, h->d_ring + (int64_t)s0 * h->L1, ring_stride, h->d_stage, h->L2,
                              h->dev_sel ? h->d_sel : nullptr);
    if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->tail));
  }
  if (c >= c0) {
    const int32_t off = (int32_t)(((c - c0) % h->r) * h->L1);
    hipLaunchKernelGGL(tvx::nupk::k_nup_add, dim3((unsigned)(((int64_t)h->C * h->L1 + 255) / 256)), dim3(256), 0,
                       h->stream, out, out_stride, h->d_stage, h->L2, off, h->L1, h->C);
    e = hipGetLastError();
    if (e != hipSuccess) return nfail(h, TVOLAP_EDEVICE, hipGetErrorString(e));
  }
  h->calls = c + 1;
  return TVOLAP_OK;
}

int tvolap_nup_reset(tvolap_nup_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return nfail(h, TVOLAP_ESTATE, "reset during capture");
  int rc = tvolap_reset(h->head);
  if (rc == TVOLAP_OK) rc = tvolap_reset(h->tail);
  if (rc != TVOLAP_OK) return nfail(h, rc, "reset of a part failed");
  hipError_t e = tvx::launch_fill_zero(h->d_ring, (size_t)h->I * h->ring_slots * h->L1 * sizeof(float), h->stream);
  if (e == hipSuccess) e = tvx::launch_fill_zero(h->d_stage, (size_t)h->C * h->L2 * sizeof(float), h->stream);
  if (e != hipSuccess) return nfail(h, TVOLAP_EDEVICE, hipGetErrorString(e));
  h->calls = 0;
  return TVOLAP_OK;
}

int tvolap_nup_autotune(tvolap_nup_t* h, int32_t iters) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return nfail(h, TVOLAP_ESTATE, "cannot autotune during graph capture");
  int rc = tvolap_autotune(h->head, iters, nullptr);
  if (rc == TVOLAP_OK) rc = tvolap_autotune(h->tail, iters, nullptr);
  if (rc != TVOLAP_OK) return nfail(h, rc, "autotune of a part failed");
  return tvolap_nup_reset(h);
}

int tvolap_nup_period(const tvolap_nup_t* h) { return h ? h->ring_slots : TVOLAP_EINVAL; }

int tvolap_nup_capture_begin(tvolap_nup_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return nfail(h, TVOLAP_ESTATE, "capture already active");
  if (h->calls % h->ring_slots != 0)
    return nfail(h, TVOLAP_ESTATE, "capture must start at a call count that is a multiple of the period");
  int rc = tvolap_capture_begin(h->head);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  h->capturing = true;
  h->capture_start = h->calls;
  return TVOLAP_OK;
}

int tvolap_nup_capture_end(tvolap_nup_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (!h->capturing) return nfail(h, TVOLAP_ESTATE, "no capture active");
  h->capturing = false;
  int rc = tvolap_capture_end(h->head);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  if ((h->calls - h->capture_start) % h->ring_slots != 0)
    return nfail(h, TVOLAP_ESTATE, "a graph must hold a multiple of the period's calls");
  return TVOLAP_OK;
}

int tvolap_nup_graph_launch(tvolap_nup_t* h) {
  if (!h) return TVOLAP_EINVAL;
  int rc = tvolap_graph_launch(h->head);
  if (rc != TVOLAP_OK) return nfail(h, rc, tvolap_last_error(h->head));
  return TVOLAP_OK;
}

const char* tvolap_nup_last_error(const tvolap_nup_t* h) { return h ? h->err.c_str() : g_nup_create_error.c_str(); }

}  // extern "C"
