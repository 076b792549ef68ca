// Host runtime behind include/tvolap.h: validation, plan construction, device
// buffers and the per-block launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tvolap.h"
#include "tvolap_internal.h"

using tvx::DevPlan;
using tvx::MacShape;
using tvx::WorkItem;

namespace {

thread_local std::string g_create_error = "no error";

constexpr int kTimingRing = 64;

struct TimingSet {
  hipEvent_t ev[4];
  bool pending = false;
};

}  // namespace

struct tvolap {
  // configuration
  int32_t L = 0, C = 0, I = 0, K = 0, dtype = 0, max_taps = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<int32_t> ch_input, ch_taps, ch_M, in_M;
  std::vector<int64_t> ch_bank_off, in_fdl_off;
  int64_t bank_elems = 0, fdl_elems = 0;
  size_t store_bytes = 8;  // bytes per stored complex value

  // device buffers
  void* d_bank = nullptr;
  void* d_fdl = nullptr;
  float* d_hist = nullptr;      // [2][I][L]
  float* d_ola = nullptr;       // [C][3L]
  int32_t* d_sel = nullptr;     // [C]
  uint64_t* d_counter = nullptr;
  float2* d_tw = nullptr;       // [4L]
  float* d_win = nullptr;       // [2L]
  int32_t* d_ch_input = nullptr;
  int32_t* d_ch_M = nullptr;
  int64_t* d_ch_bank_off = nullptr;
  int32_t* d_in_M = nullptr;
  int64_t* d_in_fdl_off = nullptr;
  float* d_taps = nullptr;      // [max_taps] staging for host taps

  // MAC work list
  MacShape shape{2, 1, 4};
  int32_t tile_width = 128;
  int32_t chunk = 0;
  std::vector<WorkItem> items;
  WorkItem* d_items = nullptr;
  int32_t n_rows = 0;
  float2* d_ypart = nullptr;    // [n_rows][tile_width]
  int32_t* d_rows_ptr = nullptr;
  int32_t* d_rows = nullptr;

  // pinned staging ring for host slot selections
  static constexpr int kSelRing = 16;
  int32_t* h_sel_ring = nullptr;   // [kSelRing][C], hipHostMalloc
  hipEvent_t sel_ev[kSelRing];
  bool sel_ev_used[kSelRing] = {};
  bool sel_ev_made = false;
  int sel_next = 0;

  // timing
  bool timing = false;
  TimingSet tsets[kTimingRing];
  int tnext = 0;
  double ms_in = 0, ms_mac = 0, ms_out = 0;
  int64_t t_blocks = 0;
  bool events_made = false;

  std::string err = "no error";
  DevPlan plan() const {
    DevPlan P;
    P.L = L; P.C = C; P.I = I; P.K = K;
    P.ch_input = d_ch_input; P.ch_M = d_ch_M; P.ch_bank_off = d_ch_bank_off;
    P.in_M = d_in_M; P.in_fdl_off = d_in_fdl_off; P.tw = d_tw; P.win = d_win;
    return P;
  }
};

namespace {

int fail(tvolap_t* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

int hip_fail(tvolap_t* h, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, TVOLAP_EDEVICE, m);
}

#define HIP_TRY(h, expr)                                   \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}

void free_all(tvolap_t* h) {
  void* bufs[] = {h->d_bank, h->d_fdl, h->d_hist, h->d_ola, h->d_sel, h->d_counter, h->d_tw, h->d_win,
                  h->d_ch_input, h->d_ch_M, h->d_ch_bank_off, h->d_in_M, h->d_in_fdl_off, h->d_taps,
                  h->d_items, h->d_ypart, h->d_rows_ptr, h->d_rows};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (h->events_made)
    for (auto& t : h->tsets)
      for (auto& e : t.ev) (void)hipEventDestroy(e);
  if (h->sel_ev_made)
    for (auto& e : h->sel_ev) (void)hipEventDestroy(e);
  if (h->h_sel_ring) (void)hipHostFree(h->h_sel_ring);
}

bool supported_hop(int L) { return L == 64 || L == 128 || L == 256 || L == 512; }

// Build the MAC work list: channels grouped by input (up to G per item), the
// 2L bins cut into tiles of 64*V, the partitions into chunks.
void build_work(tvolap_t* h, int chunk_override) {
  const int N = 2 * h->L;
  const int V = (h->dtype == 0) ? 2 : std::min(4, N / 64);
  h->shape.V = V;
  h->tile_width = 64 * V;
  const int T = N / h->tile_width;

  std::vector<std::vector<int>> by_input(h->I);
  for (int c = 0; c < h->C; ++c) by_input[h->ch_input[c]].push_back(c);
  int fan = 1;
  for (auto& v : by_input) fan = std::max<int>(fan, (int)v.size());
  const int G = fan >= 4 ? 4 : (fan >= 2 ? 2 : 1);
  h->shape.G = G;

  struct Sub { int input; std::vector<int> ch; int M; };
  std::vector<Sub> subs;
  for (int i = 0; i < h->I; ++i) {
    auto& v = by_input[i];
    for (size_t j = 0; j < v.size(); j += G) {
      Sub s;
      s.input = i;
      int Ms = 0;
      for (size_t k = j; k < std::min(v.size(), j + G); ++k) {
        s.ch.push_back(v[k]);
        Ms = std::max(Ms, h->ch_M[v[k]]);
      }
      s.M = Ms;
      subs.push_back(s);
    }
  }
  int64_t units = 0;
  for (auto& s : subs) units += (int64_t)s.M * T;
  int S = chunk_override;
  if (S <= 0) {
    // about four workgroups per compute unit of a 256-CU device
    const int64_t target = 1024;
    S = (int)std::max<int64_t>(8, (units + target - 1) / target);
  }
  h->chunk = S;

  struct Tmp { WorkItem w; int size; };
  std::vector<Tmp> tmp;
  for (auto& s : subs)
    for (int t = 0; t < T; ++t)
      for (int m0 = 0; m0 < s.M; m0 += S) {
        WorkItem w{};
        w.input = s.input;
        w.n_ch = (int)s.ch.size();
        w.m0 = m0;
        w.m1 = std::min(s.M, m0 + S);
        w.tile = t;
        for (int g = 0; g < 4; ++g) w.ch[g] = g < w.n_ch ? s.ch[g] : 0;
        tmp.push_back({w, w.m1 - w.m0});
      }
  // largest items first so that the tail of the launch is made of small ones
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.size > b.size; });
  h->items.clear();
  int row = 0;
  for (auto& t : tmp) {
    t.w.row = row;
    row += t.w.n_ch;
    h->items.push_back(t.w);
  }
  h->n_rows = row;
}

int upload_work(tvolap_t* h) {
  const int N = 2 * h->L;
  const int T = N / h->tile_width;
  // rows of every (channel, tile) in item order
  std::vector<std::vector<int32_t>> lists((size_t)h->C * T);
  for (auto& w : h->items)
    for (int g = 0; g < w.n_ch; ++g) lists[(size_t)w.ch[g] * T + w.tile].push_back(w.row + g);
  std::vector<int32_t> ptr((size_t)h->C * T + 1, 0), rows;
  for (size_t k = 0; k < lists.size(); ++k) {
    // sum partial spectra in increasing partition order (fixed, deterministic)
    std::sort(lists[k].begin(), lists[k].end(), [&](int32_t a, int32_t b) { return a < b; });
    ptr[k + 1] = ptr[k] + (int32_t)lists[k].size();
    rows.insert(rows.end(), lists[k].begin(), lists[k].end());
  }
  HIP_TRY(h, dalloc(&h->d_items, h->items.size() * sizeof(WorkItem)));
  HIP_TRY(h, dalloc(&h->d_ypart, (size_t)h->n_rows * h->tile_width * sizeof(float2)));
  HIP_TRY(h, dalloc(&h->d_rows_ptr, ptr.size() * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_rows, rows.size() * sizeof(int32_t)));
  HIP_TRY(h, hipMemcpy(h->d_items, h->items.data(), h->items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_rows_ptr, ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!rows.empty())
    HIP_TRY(h, hipMemcpy(h->d_rows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return TVOLAP_OK;
}

int create_impl(const tvolap_config* cfg, tvolap_t* h) {
  h->L = cfg->hop;
  h->C = cfg->n_channels;
  h->I = cfg->n_inputs;
  h->K = cfg->n_slots;
  h->dtype = cfg->spectra_dtype;
  h->max_taps = cfg->max_taps;
  h->stream = static_cast<hipStream_t>(cfg->stream);
  h->store_bytes = (h->dtype == TVOLAP_F32) ? 8 : 4;
  HIP_TRY(h, hipGetDevice(&h->device));
  const int L = h->L, N = 2 * L;

  h->ch_input.resize(h->C);
  h->ch_taps.resize(h->C);
  h->ch_M.resize(h->C);
  for (int c = 0; c < h->C; ++c) {
    h->ch_input[c] = cfg->input_of_channel ? cfg->input_of_channel[c] : c;
    h->ch_taps[c] = cfg->taps_of_channel ? cfg->taps_of_channel[c] : cfg->max_taps;
    h->ch_M[c] = (h->ch_taps[c] + N - 1) / N;
  }
  h->in_M.assign(h->I, 1);
  for (int c = 0; c < h->C; ++c) h->in_M[h->ch_input[c]] = std::max(h->in_M[h->ch_input[c]], h->ch_M[c]);
  h->ch_bank_off.resize(h->C);
  int64_t off = 0;
  for (int c = 0; c < h->C; ++c) {
    h->ch_bank_off[c] = off;
    off += (int64_t)h->K * h->ch_M[c] * N;
  }
  h->bank_elems = off;
  h->in_fdl_off.resize(h->I);
  off = 0;
  for (int i = 0; i < h->I; ++i) {
    h->in_fdl_off[i] = off;
    off += (int64_t)2 * h->in_M[i] * N;
  }
  h->fdl_elems = off;

  HIP_TRY(h, dalloc(&h->d_bank, (size_t)h->bank_elems * h->store_bytes));
  HIP_TRY(h, dalloc(&h->d_fdl, (size_t)h->fdl_elems * h->store_bytes));
  HIP_TRY(h, dalloc(&h->d_hist, (size_t)2 * h->I * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_ola, (size_t)h->C * 3 * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_sel, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_counter, sizeof(uint64_t)));
  HIP_TRY(h, dalloc(&h->d_tw, (size_t)4 * L * sizeof(float2)));
  HIP_TRY(h, dalloc(&h->d_win, (size_t)2 * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_ch_input, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_ch_M, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_ch_bank_off, (size_t)h->C * sizeof(int64_t)));
  HIP_TRY(h, dalloc(&h->d_in_M, (size_t)h->I * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_in_fdl_off, (size_t)h->I * sizeof(int64_t)));
  HIP_TRY(h, dalloc(&h->d_taps, (size_t)h->max_taps * sizeof(float)));

  // twiddles exp(-2 pi i t / 4L) and the Hann window, evaluated in double precision
  std::vector<float2> tw(4 * L);
  for (int t = 0; t < 4 * L; ++t) {
    const double a = -2.0 * M_PI * (double)t / (double)(4 * L);
    tw[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::vector<float> win(2 * L);
  for (int n = 0; n < 2 * L; ++n) win[n] = (float)(0.5 * (1.0 - std::cos(2.0 * M_PI * (double)n / (double)(2 * L))));
  HIP_TRY(h, hipMemcpy(h->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_win, win.data(), win.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_ch_input, h->ch_input.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_ch_M, h->ch_M.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_ch_bank_off, h->ch_bank_off.data(), h->C * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_in_M, h->in_M.data(), h->I * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_in_fdl_off, h->in_fdl_off.data(), h->I * sizeof(int64_t), hipMemcpyHostToDevice));

  HIP_TRY(h, hipMemsetAsync(h->d_bank, 0, (size_t)h->bank_elems * h->store_bytes, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_fdl, 0, (size_t)h->fdl_elems * h->store_bytes, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_hist, 0, (size_t)2 * h->I * L * sizeof(float), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_ola, 0, (size_t)h->C * 3 * L * sizeof(float), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_sel, 0, (size_t)h->C * sizeof(int32_t), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_counter, 0, sizeof(uint64_t), h->stream));

  HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->h_sel_ring),
                           (size_t)tvolap_t::kSelRing * h->C * sizeof(int32_t), hipHostMallocDefault));
  for (auto& e : h->sel_ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  h->sel_ev_made = true;

  build_work(h, 0);
  int rc = upload_work(h);
  if (rc != TVOLAP_OK) return rc;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return TVOLAP_OK;
}

void drain_timing(tvolap_t* h, TimingSet& t) {
  if (!t.pending) return;
  float a = 0, b = 0, c = 0;
  if (hipEventSynchronize(t.ev[3]) == hipSuccess) {
    (void)hipEventElapsedTime(&a, t.ev[0], t.ev[1]);
    (void)hipEventElapsedTime(&b, t.ev[1], t.ev[2]);
    (void)hipEventElapsedTime(&c, t.ev[2], t.ev[3]);
    h->ms_in += a;
    h->ms_mac += b;
    h->ms_out += c;
    h->t_blocks += 1;
  }
  t.pending = false;
}

}  // namespace

extern "C" {

const char* tvolap_version(void) { return "tvolap-gfx950 0.1"; }

const char* tvolap_last_error(const tvolap_t* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int tvolap_create(const tvolap_config* cfg, tvolap_t** out) {
  if (!out) return fail(nullptr, TVOLAP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, TVOLAP_EINVAL, "cfg is NULL");
  if (!supported_hop(cfg->hop)) return fail(nullptr, TVOLAP_EINVAL, "hop must be 64, 128, 256 or 512");
  if (cfg->n_channels < 1 || cfg->n_inputs < 1 || cfg->n_slots < 1 || cfg->max_taps < 1)
    return fail(nullptr, TVOLAP_EINVAL, "n_channels, n_inputs, n_slots and max_taps must be >= 1");
  if (cfg->spectra_dtype < 0 || cfg->spectra_dtype > 2)
    return fail(nullptr, TVOLAP_EINVAL, "spectra_dtype must be TVOLAP_F32, TVOLAP_BF16 or TVOLAP_F16");
  if (!cfg->input_of_channel && cfg->n_inputs != cfg->n_channels)
    return fail(nullptr, TVOLAP_EINVAL, "input_of_channel is NULL but n_inputs != n_channels");
  for (int c = 0; c < cfg->n_channels; ++c) {
    if (cfg->input_of_channel &&
        (cfg->input_of_channel[c] < 0 || cfg->input_of_channel[c] >= cfg->n_inputs))
      return fail(nullptr, TVOLAP_EINVAL, "input_of_channel value out of range");
    if (cfg->taps_of_channel && (cfg->taps_of_channel[c] < 1 || cfg->taps_of_channel[c] > cfg->max_taps))
      return fail(nullptr, TVOLAP_EINVAL, "taps_of_channel value outside [1, max_taps]");
  }
  {
    const int64_t M = (cfg->max_taps + 2LL * cfg->hop - 1) / (2LL * cfg->hop);
    const int64_t worst = (int64_t)cfg->n_channels * cfg->n_slots * M * 2 * cfg->hop;
    if (worst > (int64_t)1 << 40) return fail(nullptr, TVOLAP_ENOMEM, "IR bank larger than 2^40 elements");
    if (M > (1 << 24)) return fail(nullptr, TVOLAP_EINVAL, "max_taps too large");
  }
  tvolap_t* h = new (std::nothrow) tvolap_t();
  if (!h) return fail(nullptr, TVOLAP_ENOMEM, "host allocation failed");
  int rc = create_impl(cfg, h);
  if (rc != TVOLAP_OK) {
    g_create_error = h->err;
    if (rc == TVOLAP_EDEVICE && h->err.find("out of memory") != std::string::npos) rc = TVOLAP_ENOMEM;
    (void)hipGetLastError();
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return TVOLAP_OK;
}

int tvolap_destroy(tvolap_t* h) {
  if (!h) return TVOLAP_OK;
  (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
  return TVOLAP_OK;
}

int tvolap_set_ir(tvolap_t* h, int32_t channel, int32_t slot, const float* taps, int32_t n_taps,
                  int32_t taps_on_device) {
  if (!h) return TVOLAP_EINVAL;
  if (channel < 0 || channel >= h->C) return fail(h, TVOLAP_EINVAL, "channel out of range");
  if (slot < 0 || slot >= h->K) return fail(h, TVOLAP_EINVAL, "slot out of range");
  if (n_taps < 0 || n_taps > h->ch_taps[channel])
    return fail(h, TVOLAP_EINVAL, "n_taps outside [0, taps of the channel]");
  if (n_taps > 0 && !taps) return fail(h, TVOLAP_EINVAL, "taps is NULL");
  const float* src = taps;
  if (n_taps > 0 && !taps_on_device) {
    // Wait for earlier users of the staging buffer, then copy: the host array
    // may be reused as soon as this call returns.
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->d_taps, taps, (size_t)n_taps * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    src = h->d_taps;
  }
  if (n_taps == 0) src = h->d_taps;
  const int N = 2 * h->L;
  const int M = h->ch_M[channel];
  char* dst = static_cast<char*>(h->d_bank) +
              (size_t)(h->ch_bank_off[channel] + (int64_t)slot * M * N) * h->store_bytes;
  HIP_TRY(h, tvx::launch_irprep(h->plan(), h->dtype, src, n_taps, M, dst, h->stream));
  return TVOLAP_OK;
}

int tvolap_select_ir(tvolap_t* h, const int32_t* slot_of_channel) {
  if (!h) return TVOLAP_EINVAL;
  if (!slot_of_channel) return fail(h, TVOLAP_EINVAL, "slot_of_channel is NULL");
  for (int c = 0; c < h->C; ++c)
    if (slot_of_channel[c] < 0 || slot_of_channel[c] >= h->K) return fail(h, TVOLAP_EINVAL, "slot out of range");
  // Copy into a pinned ring slot whose previous transfer has completed, then
  // transfer in stream order; the caller's array is free on return.
  const int k = h->sel_next;
  if (h->sel_ev_used[k]) HIP_TRY(h, hipEventSynchronize(h->sel_ev[k]));
  int32_t* slot = h->h_sel_ring + (size_t)k * h->C;
  std::memcpy(slot, slot_of_channel, (size_t)h->C * sizeof(int32_t));
  HIP_TRY(h, hipMemcpyAsync(h->d_sel, slot, (size_t)h->C * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipEventRecord(h->sel_ev[k], h->stream));
  h->sel_ev_used[k] = true;
  h->sel_next = (k + 1) % tvolap_t::kSelRing;
  return TVOLAP_OK;
}

int tvolap_process_block(tvolap_t* h, const float* in, int64_t in_stride, float* out, int64_t out_stride,
                         const int32_t* slot_of_channel_dev) {
  if (!h) return TVOLAP_EINVAL;
  if (!in || !out) return fail(h, TVOLAP_EINVAL, "in or out is NULL");
  if (in_stride < h->L || out_stride < h->L) return fail(h, TVOLAP_EINVAL, "stride smaller than hop");
  const DevPlan P = h->plan();
  const int32_t* sel = slot_of_channel_dev ? slot_of_channel_dev : h->d_sel;
  TimingSet* ts = nullptr;
  if (h->timing) {
    ts = &h->tsets[h->tnext];
    h->tnext = (h->tnext + 1) % kTimingRing;
    drain_timing(h, *ts);
  }
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[0], h->stream));
  HIP_TRY(h, tvx::launch_fwd(P, h->dtype, in, in_stride, h->d_hist, h->d_fdl, h->d_counter, h->stream));
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[1], h->stream));
  HIP_TRY(h, tvx::launch_mac(P, h->dtype, h->shape, h->d_items, (int)h->items.size(), h->d_bank, h->d_fdl, sel,
                                h->d_ypart, h->d_counter, h->stream));
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[2], h->stream));
  HIP_TRY(h, tvx::launch_inv(P, h->tile_width, h->d_ypart, h->d_rows_ptr, h->d_rows, h->d_ola, out, out_stride,
                                slot_of_channel_dev, h->d_sel, h->d_counter, h->stream));
  if (ts) {
    HIP_TRY(h, hipEventRecord(ts->ev[3], h->stream));
    ts->pending = true;
  }
  return TVOLAP_OK;
}

int tvolap_reset(tvolap_t* h) {
  if (!h) return TVOLAP_EINVAL;
  HIP_TRY(h, tvx::launch_fill_zero(h->d_fdl, (size_t)h->fdl_elems * h->store_bytes, h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_hist, (size_t)2 * h->I * h->L * sizeof(float), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_ola, (size_t)h->C * 3 * h->L * sizeof(float), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_counter, sizeof(uint64_t), h->stream));
  return TVOLAP_OK;
}

int tvolap_get_info(const tvolap_t* h, tvolap_info* info) {
  if (!h || !info) return TVOLAP_EINVAL;
  std::memset(info, 0, sizeof(*info));
  const int N = 2 * h->L;
  info->hop = h->L;
  info->n_channels = h->C;
  info->n_inputs = h->I;
  info->n_slots = h->K;
  info->spectra_dtype = h->dtype;
  info->bins = N;
  int64_t sm = 0, si = 0;
  for (int c = 0; c < h->C; ++c) sm += h->ch_M[c];
  for (int i = 0; i < h->I; ++i) si += h->in_M[i];
  info->sum_partitions = sm;
  info->sum_input_partitions = si;
  // The MAC reads the M_c active partition spectra of every channel and, per
  // input, the M_i same-parity delay-line spectra (shared by the channels of
  // that input).
  info->mac_bytes_per_block = (sm + si) * N * (int64_t)h->store_bytes;
  info->block_bytes = info->mac_bytes_per_block + (int64_t)h->I * N * h->store_bytes +
                      (int64_t)(h->I + h->C) * h->L * 4;
  info->bank_bytes = h->bank_elems * (int64_t)h->store_bytes;
  info->delay_line_bytes = h->fdl_elems * (int64_t)h->store_bytes;
  info->workspace_bytes = (int64_t)h->n_rows * h->tile_width * 8;
  info->n_work_items = (int32_t)h->items.size();
  info->mac_chunk = h->chunk;
  info->mac_waves = h->shape.NW;
  info->mac_grid = (int32_t)h->items.size();
  return TVOLAP_OK;
}

int tvolap_get_partitions(const tvolap_t* h, int32_t* m_of_channel) {
  if (!h || !m_of_channel) return TVOLAP_EINVAL;
  for (int c = 0; c < h->C; ++c) m_of_channel[c] = h->ch_M[c];
  return TVOLAP_OK;
}

int tvolap_set_timing(tvolap_t* h, int32_t enable) {
  if (!h) return TVOLAP_EINVAL;
  if (enable && !h->events_made) {
    for (auto& t : h->tsets)
      for (auto& e : t.ev) HIP_TRY(h, hipEventCreate(&e));
    h->events_made = true;
  }
  h->timing = enable != 0;
  return TVOLAP_OK;
}

int tvolap_get_timing(tvolap_t* h, double* ms_in, double* ms_mac, double* ms_out, int64_t* n_blocks) {
  if (!h) return TVOLAP_EINVAL;
  if (h->events_made)
    for (int k = 0; k < kTimingRing; ++k) drain_timing(h, h->tsets[(h->tnext + k) % kTimingRing]);
  if (ms_in) *ms_in = h->ms_in;
  if (ms_mac) *ms_mac = h->ms_mac;
  if (ms_out) *ms_out = h->ms_out;
  if (n_blocks) *n_blocks = h->t_blocks;
  h->ms_in = h->ms_mac = h->ms_out = 0;
  h->t_blocks = 0;
  return TVOLAP_OK;
}

}  // extern "C"
