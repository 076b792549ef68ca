// Host runtime behind include/tvolap.h: validation, plan construction, device
// buffers, the per-block launch sequence, the MAC autotuner and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tvolap.h"
#include "tvolap_internal.h"

using tvx::BatchArgs;
using tvx::BlockArgs;
using tvx::DevPlan;
using tvx::MacShape;
using tvx::WorkItem;

namespace {

thread_local std::string g_create_error = "no error";

constexpr int kTimingRing = 64;
constexpr int kSelRing = 16;

struct TimingSet {
  hipEvent_t ev[4];
  bool pending = false;
  int mode = 0;     // launch mode of the recorded call (see MacChoice::fused)
  int blocks = 1;   // blocks covered by the recorded call
};

// fused: 0 = three launches per block (transform-in, MAC, transform-out);
// 1 = one launch (the last work item of a channel transforms back);
// 2 = two launches (transform-in fused into the MAC, then transform-out).
// vec: complex bins per lane for 16-bit storage (2 or 4; f32 always uses 2).
struct MacChoice {
  int32_t chunk = 0, waves = 4, grid = 0, fused = 1, vec = 4;
};

// Schedule of the time-blocked MAC of batched calls: partitions per item,
// complex bins per lane, waves per tile, blocks per time group, channels per
// item (0 = automatic for each) and engine (1 = vector ALU, 2 = matrix cores).
struct BatchChoice {
  int32_t chunk = 0, vec = 0, waves = 0, time_block = 0, group = 0, engine = 0;
};

// Autotuner results, keyed by the handle's shape (hop, channels, inputs,
// dtype, input map and partition counts).
std::mutex g_tune_mu;
std::map<std::string, MacChoice> g_tune_cache;
std::map<std::string, BatchChoice> g_btune_cache;

}  // namespace

struct tvolap {
  // configuration
  int32_t L = 0, C = 0, I = 0, K = 0, dtype = 0, max_taps = 0;
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  std::vector<int32_t> ch_input, ch_taps, ch_M;
  std::vector<int32_t> in_M;      // delay-line ring length per parity: M_i + ring_extra
  std::vector<int32_t> in_Mdata;  // M_i = max M_c over the channels of input i
  int32_t max_batch = 16, ring_extra = 7;
  std::vector<int64_t> ch_bank_off, in_fdl_off;
  int64_t bank_elems = 0, fdl_elems = 0;
  int32_t bank_pad_rows = 0;    // zero partition rows allocated after the bank
  size_t bank_alloc_bytes = 0;  // bank and padding; the delay line follows in the same allocation
  size_t store_bytes = 8;  // bytes per stored complex value

  // device buffers
  void* d_bank = nullptr;
  void* d_fdl = nullptr;
  float* d_hist = nullptr;      // [2][I][L]
  float* d_ola = nullptr;       // [n_out][3L]
  float2* d_ybus = nullptr;     // [n_out][2L] bus spectra of one block (mixdown)
  int32_t n_out = 0;            // output buses (C without a mixdown)
  bool mixdown = false;
  std::vector<int32_t> out_ptr, out_ch;   // bus e: channels out_ch[out_ptr[e] .. out_ptr[e+1])
  int32_t* d_out_ptr = nullptr;
  int32_t* d_out_ch = nullptr;
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
  int32_t* d_arrive = nullptr;  // [C]
  int32_t* d_done = nullptr;    // [1]
  float* d_zero_in = nullptr;   // [I][L] zeros (autotuner input)
  float* d_tune_out = nullptr;  // [C][L] autotuner output
  int32_t* d_tune_sel = nullptr;  // [K][C] autotuner selections (row k: every channel in slot k)
  int32_t* d_in_ch_ptr = nullptr; // [I+1]
  int32_t* d_in_ch = nullptr;     // [C]
  int32_t* d_part_base = nullptr; // [C+1] prefix sums of the partition counts
  int32_t* d_ch_taps = nullptr;   // [C] taps per channel

  // MAC work list
  MacShape shape{2, 1, 4};
  MacChoice choice;
  int32_t tile_width = 128;
  int32_t chunk = 0;
  std::vector<WorkItem> items;    // n_spec spectrum items, then n_mac MAC items
  int32_t n_spec = 0, n_mac = 0;
  std::vector<int32_t> ch_row_base, ch_nchunks, needed;
  int32_t n_rows = 0;
  WorkItem* d_items = nullptr;
  float2* d_ypart = nullptr;    // [n_rows][tile_width]
  int32_t* d_ch_row_base = nullptr;
  int32_t* d_ch_nchunks = nullptr;
  int32_t* d_needed = nullptr;

  // batched blocks: time-blocked MAC work list (partitions from 0)
  MacShape bshape{2, 1, 4};
  BatchChoice bchoice;
  int32_t b_tile_width = 512, b_chunk = 0, n_bmac = 0, n_brows = 0, b_tb = 8;
  std::vector<WorkItem> bitems;
  std::vector<int32_t> b_row_base, b_nchunks;
  WorkItem* d_bitems = nullptr;
  int32_t* d_brow_base = nullptr;
  int32_t* d_bnchunks = nullptr;
  float2* d_bypart = nullptr;     // [max_batch][n_brows][b_tile_width]
  int32_t* d_defer = nullptr;     // [1 + units]: count, then units the matrix-core MAC defers
  int32_t* d_tune_bsel = nullptr; // [max_batch][C] autotuner schedule (slot = block mod K)

  // pinned staging ring for host slot selections
  int32_t* h_sel_ring = nullptr;  // [kSelRing][C], hipHostMalloc
  hipEvent_t sel_ev[kSelRing];
  bool sel_ev_used[kSelRing] = {};
  bool sel_ev_made = false;
  int sel_next = 0;

  // graph capture
  bool capturing = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  // timing
  bool timing = false;
  TimingSet tsets[kTimingRing];
  int tnext = 0;
  double ms_in = 0, ms_mac = 0, ms_out = 0;
  int64_t t_blocks = 0, t_calls = 0;
  bool events_made = false;

  std::string err = "no error";

  DevPlan plan() const {
    DevPlan P;
    P.L = L; P.C = C; P.I = I; P.K = K;
    P.ch_input = d_ch_input; P.ch_M = d_ch_M; P.ch_bank_off = d_ch_bank_off;
    P.in_M = d_in_M; P.in_fdl_off = d_in_fdl_off; P.tw = d_tw; P.win = d_win;
    P.ch_row_base = d_ch_row_base; P.ch_nchunks = d_ch_nchunks; P.tile_width = tile_width;
    P.in_ch_ptr = d_in_ch_ptr; P.in_ch = d_in_ch;
    P.n_out = n_out; P.out_ptr = d_out_ptr; P.out_ch = d_out_ch; P.ybus = d_ybus;
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

#define RC_TRY(expr)                  \
  do {                                \
    int _rc = (expr);                 \
    if (_rc != TVOLAP_OK) return _rc; \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_work(tvolap_t* h) {
  dfree(h->d_items);
  dfree(h->d_ypart);
  dfree(h->d_ch_row_base);
  dfree(h->d_ch_nchunks);
  dfree(h->d_needed);
}

void free_batch_work(tvolap_t* h) {
  dfree(h->d_bitems);
  dfree(h->d_brow_base);
  dfree(h->d_bnchunks);
  dfree(h->d_bypart);
  dfree(h->d_defer);
}

void free_all(tvolap_t* h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
  free_work(h);
  free_batch_work(h);
  dfree(h->d_bank); h->d_fdl = nullptr; dfree(h->d_ybus); dfree(h->d_hist); dfree(h->d_ola); dfree(h->d_sel);
  dfree(h->d_out_ptr); dfree(h->d_out_ch);
  dfree(h->d_counter); dfree(h->d_tw); dfree(h->d_win); dfree(h->d_ch_input); dfree(h->d_ch_M);
  dfree(h->d_ch_bank_off); dfree(h->d_in_M); dfree(h->d_in_fdl_off); dfree(h->d_taps);
  dfree(h->d_arrive); dfree(h->d_done); dfree(h->d_zero_in); dfree(h->d_tune_out); dfree(h->d_tune_sel);
  dfree(h->d_in_ch_ptr); dfree(h->d_in_ch); dfree(h->d_part_base); dfree(h->d_ch_taps); dfree(h->d_tune_bsel);
  if (h->events_made)
    for (auto& t : h->tsets)
      for (auto& e : t.ev) (void)hipEventDestroy(e);
  if (h->sel_ev_made)
    for (auto& e : h->sel_ev) (void)hipEventDestroy(e);
  if (h->h_sel_ring) (void)hipHostFree(h->h_sel_ring);
  h->h_sel_ring = nullptr;
}

bool supported_hop(int L) { return L == 64 || L == 128 || L == 256 || L == 512; }

// Build the MAC work list: channels grouped by input (up to G per item), the
// 2L bins cut into tiles of 64 V, each channel group's partition range cut
// into chunks of `S` partitions. The partial-spectrum rows of a channel are
// contiguous in (tile, chunk) order, so the channel's spectrum is the sum over
// chunks of rows base + tile * nchunks + chunk.
void build_work(tvolap_t* h, int S_req, int waves, int vec) {
  const int N = 2 * h->L;
  const int V = (h->dtype == 0) ? 2 : std::min(vec == 2 ? 2 : 4, N / 64);
  h->shape.V = V;
  h->shape.NW = (waves == 8) ? 8 : 4;
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
      s.M = 0;
      for (size_t k = j; k < std::min(v.size(), j + (size_t)G); ++k) {
        s.ch.push_back(v[k]);
        s.M = std::max(s.M, h->ch_M[v[k]]);
      }
      subs.push_back(s);
    }
  }
  // MAC items cover partitions m >= 1; the m = 0 term is added when a channel
  // is completed, from the spectrum computed in the same block.
  int64_t units = 0;
  for (auto& s : subs) units += (int64_t)(s.M - 1) * T;
  int S = S_req;
  if (S <= 0) {
    // about four workgroups per compute unit
    const int64_t target = 4LL * h->n_cu;
    S = (int)std::max<int64_t>(4, (units + target - 1) / target);
  }
  h->chunk = S;

  h->ch_row_base.assign(h->C, 0);
  h->ch_nchunks.assign(h->C, 0);
  h->needed.assign(h->C, 0);
  int row = 0;
  // every channel has at least one MAC item (possibly over no partitions), so
  // that in batched mode each (block, channel) pair has an item that completes it
  auto chunks_of = [&](const Sub& s) { return std::max(1, (s.M - 1 + S - 1) / S); };
  for (auto& s : subs) {
    const int nch = chunks_of(s);
    for (int c : s.ch) {
      h->ch_row_base[c] = row;
      h->ch_nchunks[c] = nch;
      h->needed[c] = nch * T + 1;   // MAC items + the input's spectrum item
      row += nch * T;
    }
  }
  h->n_rows = row;

  struct Tmp { WorkItem w; int size; };
  std::vector<Tmp> tmp;
  for (auto& s : subs) {
    const int nch = chunks_of(s);
    for (int t = 0; t < T; ++t)
      for (int j = 0; j < nch; ++j) {
        WorkItem w{};
        w.kind = 0;
        w.input = s.input;
        w.n_ch = (int)s.ch.size();
        w.m0 = std::min(s.M, 1 + j * S);
        w.m1 = std::min(s.M, 1 + (j + 1) * S);
        w.tile = t;
        w.chunk = j;
        w.nch = nch;
        for (int g = 0; g < 4; ++g) {
          const int c = g < w.n_ch ? s.ch[g] : s.ch[0];
          w.ch[g] = c;
          w.row[g] = h->ch_row_base[c] + t * nch + j;
        }
        tmp.push_back({w, w.m1 - w.m0});
      }
  }
  // largest items first, so that the launch ends with small ones
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.size > b.size; });
  h->items.clear();
  for (int i = 0; i < h->I; ++i) {
    WorkItem w{};
    w.kind = 1;
    w.input = i;
    h->items.push_back(w);
  }
  for (auto& t : tmp) h->items.push_back(t.w);
  h->n_spec = h->I;
  h->n_mac = (int32_t)tmp.size();
}

// Work list of the time-blocked MAC (batched calls): channels grouped by
// input (up to 2 per item), the 2L bins cut into tiles of 64 V NW (16 NW for
// the matrix-core engine), each
// group's partitions [0, M) cut into chunks of S. The partial rows of a
// channel are contiguous in (tile, chunk) order. Each item runs once per
// time group (a parity class of up to b_tb (8 or 16) blocks of the call).
// The matrix-core MAC addresses the partition spectra of an item's channels
// and the delay line of its input with 32-bit byte offsets from one base.
bool mfma_offsets_fit(const tvolap_t* h) {
  const int64_t N = 2 * h->L, lim = (int64_t)1 << 32;
  for (int c = 0; c < h->C; ++c) {
    // channel c and every later channel of the same input (pairs are formed in increasing order)
    for (int c2 = c; c2 < h->C; ++c2) {
      if (h->ch_input[c2] != h->ch_input[c]) continue;
      const int64_t span = h->ch_bank_off[c2] - h->ch_bank_off[c] + (int64_t)h->K * h->ch_M[c2] * N +
                           (int64_t)h->bank_pad_rows * N;
      if (span * 8 >= lim) return false;
    }
  }
  if ((int64_t)h->bank_alloc_bytes + h->fdl_elems * 8 >= lim) return false;   // delay line from the bank base
  return true;
}

void build_batch_work(tvolap_t* h, const BatchChoice& bc) {
  const int N = 2 * h->L;
  // time groups of 16 blocks (one bin per lane) when calls can hold 32 blocks
  int V = (bc.vec == 1) ? 1 : 2;
  int TB = bc.time_block == 16 ? 16 : (bc.time_block == 8 ? 8 : (h->max_batch >= 32 ? 16 : 8));
  const int engine = bc.engine == 2 ? 2 : 1;
  h->bshape.E = (engine == 2 && mfma_offsets_fit(h)) ? 1 : 0;   // else 32-bit byte offsets do not reach
  // bins per lane (vector ALU), or per lane group as 16-bin sub-tiles (matrix cores)
  const int bins = h->bshape.E == 1 ? 16 : 64;
  if (h->bshape.E == 1) {
    // matrix cores: time groups of 16 or 32 blocks, 16 bins per wave, 4 waves
    TB = bc.time_block == 16 ? 16 : (bc.time_block == 32 || h->max_batch >= 64 ? 32 : 16);
    V = 1;
  } else {
    if (TB == 16 && bc.vec == 0) V = 1;
    if (TB == 16 && V != 1) TB = 8;
  }
  h->b_tb = TB;
  while (bins * V > N && V > 1) V /= 2;
  int NW = bc.waves > 0 ? bc.waves : 4;
  NW = NW >= 4 ? 4 : (NW >= 2 ? 2 : 1);
  // matrix cores: 4 or 8 waves (tiles of 64 or 128 bins, which the vector-ALU
  // MAC of deferred units takes with 1 or 2 waves)
  if (h->bshape.E == 1) NW = (bc.waves == 8 && N >= 128) ? 8 : 4;
  while (bins * V * NW > N && NW > 1) NW /= 2;
  h->bshape.V = V;
  h->bshape.NW = NW;
  h->b_tile_width = bins * V * NW;
  const int T = N / h->b_tile_width;

  std::vector<std::vector<int>> by_input(h->I);
  for (int c = 0; c < h->C; ++c) by_input[h->ch_input[c]].push_back(c);
  int fan = 1;
  for (auto& v : by_input) fan = std::max<int>(fan, (int)v.size());
  const int G = (fan >= 2 && bc.group != 1) ? 2 : 1;
  h->bshape.G = G;
  struct Sub { int input; std::vector<int> ch; int M; };
  std::vector<Sub> subs;
  for (int i = 0; i < h->I; ++i) {
    auto& v = by_input[i];
    for (size_t j = 0; j < v.size(); j += G) {
      Sub sb;
      sb.input = i;
      sb.M = 0;
      for (size_t k = j; k < std::min(v.size(), j + (size_t)G); ++k) {
        sb.ch.push_back(v[k]);
        sb.M = std::max(sb.M, h->ch_M[v[k]]);
      }
      subs.push_back(sb);
    }
  }
  int S = bc.chunk;
  if (S <= 0) {
    // about two workgroups per compute unit for a 16-block batch (two time groups)
    int64_t units = 0;
    for (auto& sb : subs) units += (int64_t)sb.M * T;
    const int64_t target = h->n_cu;
    S = (int)std::max<int64_t>(4, (units + target - 1) / target);
  }
  h->b_chunk = S;
  h->b_row_base.assign(h->C, 0);
  h->b_nchunks.assign(h->C, 0);
  int row = 0;
  auto chunks_of = [&](const Sub& sb) { return std::max(1, (sb.M + S - 1) / S); };
  for (auto& sb : subs) {
    const int nch = chunks_of(sb);
    for (int c : sb.ch) {
      h->b_row_base[c] = row;
      h->b_nchunks[c] = nch;
      row += nch * T;
    }
  }
  h->n_brows = row;
  struct Tmp { WorkItem w; int size; };
  std::vector<Tmp> tmp;
  for (auto& sb : subs) {
    const int nch = chunks_of(sb);
    for (int t = 0; t < T; ++t)
      for (int j = 0; j < nch; ++j) {
        WorkItem w{};
        w.kind = 0;
        w.input = sb.input;
        w.n_ch = (int)sb.ch.size();
        w.m0 = std::min(sb.M, j * S);
        w.m1 = std::min(sb.M, (j + 1) * S);
        w.tile = t;
        w.chunk = j;
        w.nch = nch;
        for (int g = 0; g < 4; ++g) {
          const int c = g < w.n_ch ? sb.ch[g] : sb.ch[0];
          w.ch[g] = c;
          w.row[g] = h->b_row_base[c] + t * nch + j;
        }
        tmp.push_back({w, w.m1 - w.m0});
      }
  }
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.size > b.size; });
  h->bitems.clear();
  for (auto& t : tmp) h->bitems.push_back(t.w);
  h->n_bmac = (int32_t)h->bitems.size();
}

int upload_work(tvolap_t* h) {
  free_work(h);
  HIP_TRY(h, dalloc(&h->d_items, h->items.size() * sizeof(WorkItem)));
  HIP_TRY(h, dalloc(&h->d_ypart, (size_t)h->n_rows * h->tile_width * sizeof(float2)));
  HIP_TRY(h, dalloc(&h->d_ch_row_base, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_ch_nchunks, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_needed, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, hipMemcpy(h->d_items, h->items.data(), h->items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_ch_row_base, h->ch_row_base.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_ch_nchunks, h->ch_nchunks.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_needed, h->needed.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  return TVOLAP_OK;
}

int upload_batch_work(tvolap_t* h) {
  free_batch_work(h);
  HIP_TRY(h, dalloc(&h->d_bitems, h->bitems.size() * sizeof(WorkItem)));
  HIP_TRY(h, dalloc(&h->d_brow_base, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_bnchunks, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_bypart, (size_t)h->max_batch * h->n_brows * h->b_tile_width * sizeof(float2)));
  {
    // work units of a full call: 8-aligned (item, class) pairs times time groups
    // (in the vector-ALU MAC's index space: time groups of 16)
    const int64_t groups = ((h->max_batch + 1) / 2 + 15) / 16;
    const int64_t units = 8 * (int64_t)((2 * h->n_bmac + 7) / 8) * groups;
    HIP_TRY(h, dalloc(&h->d_defer, (size_t)(1 + units) * sizeof(int32_t)));
    HIP_TRY(h, hipMemset(h->d_defer, 0, sizeof(int32_t)));
  }
  HIP_TRY(h, hipMemcpy(h->d_bitems, h->bitems.data(), h->bitems.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_brow_base, h->b_row_base.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_bnchunks, h->b_nchunks.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  return TVOLAP_OK;
}

int apply_batch_choice(tvolap_t* h, const BatchChoice& c) {
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  build_batch_work(h, c);
  RC_TRY(upload_batch_work(h));
  h->bchoice.chunk = h->b_chunk;
  h->bchoice.vec = h->bshape.V;
  h->bchoice.waves = h->bshape.NW;
  h->bchoice.time_block = h->b_tb;
  h->bchoice.group = h->bshape.G;
  h->bchoice.engine = h->bshape.E == 1 ? 2 : 1;
  return TVOLAP_OK;
}

int apply_choice(tvolap_t* h, const MacChoice& c) {
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  build_work(h, c.chunk, c.waves, c.vec);
  RC_TRY(upload_work(h));
  h->choice = c;
  h->choice.chunk = h->chunk;
  h->choice.waves = h->shape.NW;
  h->choice.vec = h->shape.V;
  return TVOLAP_OK;
}

int grid_of(const tvolap_t* h) {
  const int n = (int)h->items.size();
  if (h->choice.grid <= 0 || h->choice.grid > n) return n;
  return h->choice.grid;
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
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
      h->n_cu = cus;
  }
  const int L = h->L, N = 2 * L;

  h->ch_input.resize(h->C);
  h->ch_taps.resize(h->C);
  h->ch_M.resize(h->C);
  for (int c = 0; c < h->C; ++c) {
    h->ch_input[c] = cfg->input_of_channel ? cfg->input_of_channel[c] : c;
    h->ch_taps[c] = cfg->taps_of_channel ? cfg->taps_of_channel[c] : cfg->max_taps;
    h->ch_M[c] = (h->ch_taps[c] + N - 1) / N;
  }
  h->max_batch = cfg->max_batch > 0 ? cfg->max_batch : 16;
  h->ring_extra = (h->max_batch - 1) / 2;
  // output buses
  h->mixdown = cfg->n_outputs > 0;
  h->n_out = h->mixdown ? cfg->n_outputs : h->C;
  h->out_ptr.assign(h->n_out + 1, 0);
  h->out_ch.clear();
  for (int e = 0; e < h->n_out; ++e) {
    for (int c = 0; c < h->C; ++c)
      if ((h->mixdown ? cfg->output_of_channel[c] : c) == e) h->out_ch.push_back(c);
    h->out_ptr[e + 1] = (int32_t)h->out_ch.size();
  }
  h->in_Mdata.assign(h->I, 1);
  for (int c = 0; c < h->C; ++c)
    h->in_Mdata[h->ch_input[c]] = std::max(h->in_Mdata[h->ch_input[c]], h->ch_M[c]);
  h->in_M.resize(h->I);
  for (int i = 0; i < h->I; ++i) h->in_M[i] = h->in_Mdata[i] + h->ring_extra;
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

  // zero rows after the last channel: the matrix-core MAC loads partition rows
  // up to 16 ahead of the one it multiplies, and a channel shorter than the
  // other channel of its item up to the other's partition count (the values
  // are masked; the addresses must stay inside the allocation)
  {
    int maxM = 1;
    for (int c = 0; c < h->C; ++c) maxM = std::max(maxM, h->ch_M[c]);
    h->bank_pad_rows = maxM + 32;
  }
  // one allocation holds the bank (with its padding) and then the delay line,
  // so one base and 32-bit offsets reach both
  h->bank_alloc_bytes = (((size_t)(h->bank_elems + (int64_t)h->bank_pad_rows * N) * h->store_bytes + 255) / 256) * 256;
  HIP_TRY(h, dalloc(&h->d_bank, h->bank_alloc_bytes + (size_t)h->fdl_elems * h->store_bytes));
  h->d_fdl = static_cast<char*>(h->d_bank) + h->bank_alloc_bytes;
  HIP_TRY(h, dalloc(&h->d_hist, (size_t)2 * h->I * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_ola, (size_t)h->n_out * 3 * L * sizeof(float)));
  if (h->mixdown) HIP_TRY(h, dalloc(&h->d_ybus, (size_t)h->n_out * 2 * L * sizeof(float2)));
  HIP_TRY(h, dalloc(&h->d_out_ptr, (size_t)(h->n_out + 1) * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_out_ch, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, hipMemcpy(h->d_out_ptr, h->out_ptr.data(), (h->n_out + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_out_ch, h->out_ch.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
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
  HIP_TRY(h, dalloc(&h->d_arrive, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_done, sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_zero_in, (size_t)h->I * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_tune_out, (size_t)h->C * L * sizeof(float)));
  HIP_TRY(h, dalloc(&h->d_tune_sel, (size_t)h->K * h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_tune_bsel, (size_t)h->max_batch * h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_in_ch_ptr, (size_t)(h->I + 1) * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_in_ch, (size_t)h->C * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_part_base, (size_t)(h->C + 1) * sizeof(int32_t)));
  HIP_TRY(h, dalloc(&h->d_ch_taps, (size_t)h->C * sizeof(int32_t)));
  {
    std::vector<int32_t> ts((size_t)h->K * h->C);
    for (int k = 0; k < h->K; ++k)
      for (int c = 0; c < h->C; ++c) ts[(size_t)k * h->C + c] = k;
    HIP_TRY(h, hipMemcpy(h->d_tune_sel, ts.data(), ts.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    std::vector<int32_t> tb((size_t)h->max_batch * h->C);
    for (int j = 0; j < h->max_batch; ++j)
      for (int c = 0; c < h->C; ++c) tb[(size_t)j * h->C + c] = j % h->K;
    HIP_TRY(h, hipMemcpy(h->d_tune_bsel, tb.data(), tb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    std::vector<int32_t> ptr(h->I + 1, 0), chs;
    for (int i = 0; i < h->I; ++i) {
      for (int c = 0; c < h->C; ++c)
        if (h->ch_input[c] == i) chs.push_back(c);
      ptr[i + 1] = (int32_t)chs.size();
    }
    HIP_TRY(h, hipMemcpy(h->d_in_ch_ptr, ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_in_ch, chs.data(), chs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    std::vector<int32_t> pb(h->C + 1, 0);
    for (int c = 0; c < h->C; ++c) pb[c + 1] = pb[c] + h->ch_M[c];
    HIP_TRY(h, hipMemcpy(h->d_part_base, pb.data(), pb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_ch_taps, h->ch_taps.data(), h->C * sizeof(int32_t), hipMemcpyHostToDevice));
  }

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

  HIP_TRY(h, hipMemsetAsync(h->d_bank, 0, (size_t)(h->bank_elems + (int64_t)h->bank_pad_rows * N) * h->store_bytes,
                            h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_fdl, 0, (size_t)h->fdl_elems * h->store_bytes, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_hist, 0, (size_t)2 * h->I * L * sizeof(float), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_ola, 0, (size_t)h->n_out * 3 * L * sizeof(float), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_sel, 0, (size_t)h->C * sizeof(int32_t), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_counter, 0, sizeof(uint64_t), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_arrive, 0, (size_t)h->C * sizeof(int32_t), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_done, 0, sizeof(int32_t), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_zero_in, 0, (size_t)h->I * L * sizeof(float), h->stream));

  HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->h_sel_ring), (size_t)kSelRing * h->C * sizeof(int32_t),
                           hipHostMallocDefault));
  for (auto& e : h->sel_ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  h->sel_ev_made = true;

  MacChoice c;
  if (h->mixdown) c.fused = 0;   // bus sums run in the separate transform-out launch
  RC_TRY(apply_choice(h, c));
  RC_TRY(apply_batch_choice(h, BatchChoice{}));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return TVOLAP_OK;
}

void drain_timing(tvolap_t* h, TimingSet& t) {
  if (!t.pending) return;
  float a = 0, b = 0, c = 0;
  if (hipEventSynchronize(t.ev[3]) == hipSuccess) {
    if (t.mode == 1) {
      (void)hipEventElapsedTime(&b, t.ev[0], t.ev[3]);
    } else if (t.mode == 2) {
      (void)hipEventElapsedTime(&b, t.ev[0], t.ev[2]);
      (void)hipEventElapsedTime(&c, t.ev[2], t.ev[3]);
    } else {
      (void)hipEventElapsedTime(&a, t.ev[0], t.ev[1]);
      (void)hipEventElapsedTime(&b, t.ev[1], t.ev[2]);
      (void)hipEventElapsedTime(&c, t.ev[2], t.ev[3]);
    }
    h->ms_in += a;
    h->ms_mac += b;
    h->ms_out += c;
    h->t_blocks += t.blocks;
    h->t_calls += 1;
  }
  t.pending = false;
}

// Enqueue one block. Timing events are recorded only outside graph capture.
// sel_dev: this block's slots (device) or NULL for the handle's selection;
// copy_sel: make sel_dev the handle's selection.
int enqueue_block(tvolap_t* h, const float* in, int64_t in_stride, float* out, int64_t out_stride,
                  const int32_t* sel_dev, bool copy_sel) {
  const DevPlan P = h->plan();
  const int32_t* sel = sel_dev ? sel_dev : h->d_sel;
  TimingSet* ts = nullptr;
  if (h->timing && !h->capturing) {
    ts = &h->tsets[h->tnext];
    h->tnext = (h->tnext + 1) % kTimingRing;
    drain_timing(h, *ts);
    ts->mode = h->choice.fused;
    ts->blocks = 1;
  }
  if (h->choice.fused) {
    BlockArgs A;
    A.P = P;
    A.items = h->d_items;
    A.n_items = (int32_t)h->items.size();
    A.bank = h->d_bank;
    A.fdl = h->d_fdl;
    A.sel = sel;
    A.sel_store = h->d_sel;
    A.copy_sel = copy_sel ? 1 : 0;
    A.in = in;
    A.in_stride = in_stride;
    A.hist = h->d_hist;
    A.ypart = h->d_ypart;
    A.arrive = h->d_arrive;
    A.needed = h->d_needed;
    A.done = h->d_done;
    A.ola = h->d_ola;
    A.out = out;
    A.out_stride = out_stride;
    A.counter = h->d_counter;
    A.inverse_inline = h->choice.fused == 1 ? 1 : 0;
    if (ts) HIP_TRY(h, hipEventRecord(ts->ev[0], h->stream));
    HIP_TRY(h, tvx::launch_block(A, h->dtype, h->shape, grid_of(h), h->stream));
    if (h->choice.fused == 2) {
      if (ts) HIP_TRY(h, hipEventRecord(ts->ev[2], h->stream));
      HIP_TRY(h, tvx::launch_inv(P, h->dtype, h->d_ypart, h->d_bank, h->d_fdl, sel, h->d_ola, out, out_stride,
                                 copy_sel ? 1 : 0, h->d_sel, h->d_done, h->d_counter, h->stream));
    }
    if (ts) {
      HIP_TRY(h, hipEventRecord(ts->ev[3], h->stream));
      ts->pending = true;
    }
    return TVOLAP_OK;
  }
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[0], h->stream));
  HIP_TRY(h, tvx::launch_fwd(P, h->dtype, in, in_stride, h->d_hist, h->d_fdl, h->d_counter, h->stream));
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[1], h->stream));
  HIP_TRY(h, tvx::launch_mac(P, h->dtype, h->shape, h->d_items + h->n_spec, h->n_mac, h->d_bank, h->d_fdl, sel,
                             h->d_ypart, h->d_counter, h->stream));
  if (ts) HIP_TRY(h, hipEventRecord(ts->ev[2], h->stream));
  HIP_TRY(h, tvx::launch_inv(P, h->dtype, h->d_ypart, h->d_bank, h->d_fdl, sel, h->d_ola, out, out_stride,
                             copy_sel ? 1 : 0, h->d_sel, h->d_done, h->d_counter, h->stream));
  if (ts) {
    HIP_TRY(h, hipEventRecord(ts->ev[3], h->stream));
    ts->pending = true;
  }
  return TVOLAP_OK;
}

int enqueue_blocks(tvolap_t* h, const float* in, int64_t in_stride, int32_t n_blocks, float* out,
                   int64_t out_stride, const int32_t* slots_dev, int64_t slots_stride, bool copy_sel);

int reset_state(tvolap_t* h) {
  HIP_TRY(h, tvx::launch_fill_zero(h->d_fdl, (size_t)h->fdl_elems * h->store_bytes, h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_hist, (size_t)2 * h->I * h->L * sizeof(float), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_ola, (size_t)h->n_out * 3 * h->L * sizeof(float), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_counter, sizeof(uint64_t), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_arrive, (size_t)h->C * sizeof(int32_t), h->stream));
  HIP_TRY(h, tvx::launch_fill_zero(h->d_done, sizeof(int32_t), h->stream));
  return TVOLAP_OK;
}

std::string tune_key(const tvolap_t* h) {
  std::string k = std::to_string(h->L) + "/" + std::to_string(h->C) + "/" + std::to_string(h->I) + "/" +
                  std::to_string(h->dtype) + "/" + std::to_string(h->n_cu) + ":";
  uint64_t hash = 1469598103934665603ull;
  for (int c = 0; c < h->C; ++c) {
    hash = (hash ^ (uint64_t)h->ch_M[c]) * 1099511628211ull;
    hash = (hash ^ (uint64_t)h->ch_input[c]) * 1099511628211ull;
  }
  return k + std::to_string(hash);
}

}  // namespace

extern "C" {

const char* tvolap_version(void) { return "tvolap-gfx950 0.2"; }

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
  if (cfg->max_batch < 0 || cfg->max_batch > 1024)
    return fail(nullptr, TVOLAP_EINVAL, "max_batch must be in [0, 1024]");
  if (!cfg->input_of_channel && cfg->n_inputs != cfg->n_channels)
    return fail(nullptr, TVOLAP_EINVAL, "input_of_channel is NULL but n_inputs != n_channels");
  if (cfg->n_outputs < 0 || cfg->n_outputs > cfg->n_channels)
    return fail(nullptr, TVOLAP_EINVAL, "n_outputs must be in [0, n_channels]");
  if (cfg->n_outputs > 0) {
    if (!cfg->output_of_channel) return fail(nullptr, TVOLAP_EINVAL, "output_of_channel is NULL");
    std::vector<int> used(cfg->n_outputs, 0);
    for (int c = 0; c < cfg->n_channels; ++c) {
      const int e = cfg->output_of_channel[c];
      if (e < 0 || e >= cfg->n_outputs) return fail(nullptr, TVOLAP_EINVAL, "output_of_channel value out of range");
      used[e] = 1;
    }
    for (int e = 0; e < cfg->n_outputs; ++e)
      if (!used[e]) return fail(nullptr, TVOLAP_EINVAL, "every output needs at least one channel");
  }
  for (int c = 0; c < cfg->n_channels; ++c) {
    if (cfg->input_of_channel &&
        (cfg->input_of_channel[c] < 0 || cfg->input_of_channel[c] >= cfg->n_inputs))
      return fail(nullptr, TVOLAP_EINVAL, "input_of_channel value out of range");
    if (cfg->taps_of_channel && (cfg->taps_of_channel[c] < 1 || cfg->taps_of_channel[c] > cfg->max_taps))
      return fail(nullptr, TVOLAP_EINVAL, "taps_of_channel value outside [1, max_taps]");
  }
  {
    const int64_t M = (cfg->max_taps + 2LL * cfg->hop - 1) / (2LL * cfg->hop);
    if (M > (1 << 24)) return fail(nullptr, TVOLAP_EINVAL, "max_taps too large");
    const int64_t worst = (int64_t)cfg->n_channels * cfg->n_slots * M * 2 * cfg->hop;
    if (worst > ((int64_t)1 << 40)) return fail(nullptr, TVOLAP_ENOMEM, "IR bank larger than 2^40 elements");
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
  if (h->capturing) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h->stream, &g);
    if (g) (void)hipGraphDestroy(g);
  }
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
  if (h->capturing && n_taps > 0 && !taps_on_device)
    return fail(h, TVOLAP_ESTATE, "host taps cannot be loaded during graph capture");
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

int tvolap_set_irs(tvolap_t* h, int32_t slot, const float* taps_dev, int64_t taps_stride) {
  if (!h) return TVOLAP_EINVAL;
  if (slot < 0 || slot >= h->K) return fail(h, TVOLAP_EINVAL, "slot out of range");
  if (!taps_dev) return fail(h, TVOLAP_EINVAL, "taps is NULL");
  if (taps_stride < 1) return fail(h, TVOLAP_EINVAL, "taps_stride must be >= 1");
  int64_t total = 0;
  for (int c = 0; c < h->C; ++c) total += h->ch_M[c];
  if (total > INT32_MAX) return fail(h, TVOLAP_EINVAL, "too many partitions");
  HIP_TRY(h, tvx::launch_irprep_all(h->plan(), h->dtype, h->d_part_base, (int32_t)total, h->d_ch_taps, taps_dev,
                                    taps_stride, slot, h->d_bank, h->stream));
  return TVOLAP_OK;
}

int tvolap_select_ir(tvolap_t* h, const int32_t* slot_of_channel) {
  if (!h) return TVOLAP_EINVAL;
  if (!slot_of_channel) return fail(h, TVOLAP_EINVAL, "slot_of_channel is NULL");
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "host selections cannot be recorded in a graph");
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
  h->sel_next = (k + 1) % kSelRing;
  return TVOLAP_OK;
}

int tvolap_process_block(tvolap_t* h, const float* in, int64_t in_stride, float* out, int64_t out_stride,
                         const int32_t* slot_of_channel_dev) {
  if (!h) return TVOLAP_EINVAL;
  if (!in || !out) return fail(h, TVOLAP_EINVAL, "in or out is NULL");
  if (in_stride < h->L || out_stride < h->L) return fail(h, TVOLAP_EINVAL, "stride smaller than hop");
  return enqueue_block(h, in, in_stride, out, out_stride, slot_of_channel_dev, slot_of_channel_dev != nullptr);
}

int tvolap_process_blocks(tvolap_t* h, const float* in, int64_t in_stride, int32_t n_blocks, float* out,
                          int64_t out_stride, const int32_t* slots_dev, int64_t slots_stride) {
  if (!h) return TVOLAP_EINVAL;
  if (!in || !out) return fail(h, TVOLAP_EINVAL, "in or out is NULL");
  if (n_blocks < 1 || n_blocks > h->max_batch) return fail(h, TVOLAP_EINVAL, "n_blocks outside [1, max_batch]");
  if (in_stride < (int64_t)n_blocks * h->L && h->I > 1)
    return fail(h, TVOLAP_EINVAL, "in_stride smaller than n_blocks * hop");
  if (out_stride < (int64_t)n_blocks * h->L && h->n_out > 1)
    return fail(h, TVOLAP_EINVAL, "out_stride smaller than n_blocks * hop");
  if (slots_dev && slots_stride < h->C) return fail(h, TVOLAP_EINVAL, "slots_stride smaller than n_channels");
  return enqueue_blocks(h, in, in_stride, n_blocks, out, out_stride, slots_dev, slots_stride, slots_dev != nullptr);
}

}  // extern "C"

namespace {

// Enqueue a batched call (arguments already checked). copy_sel: the last
// block's slots become the handle's selection.
int enqueue_blocks(tvolap_t* h, const float* in, int64_t in_stride, int32_t n_blocks, float* out,
                   int64_t out_stride, const int32_t* slots_dev, int64_t slots_stride, bool copy_sel) {
  BatchArgs B;
  B.P = h->plan();
  B.items = h->d_bitems;
  B.n_mac = h->n_bmac;
  B.n_blocks = n_blocks;
  B.n_rows = h->n_brows;
  B.tile_width = h->b_tile_width;
  B.time_block = h->b_tb;
  B.row_base = h->d_brow_base;
  B.nchunks = h->d_bnchunks;
  B.bank = h->d_bank;
  B.fdl = h->d_fdl;
  B.sel = slots_dev ? slots_dev : h->d_sel;
  B.sel_stride = slots_dev ? slots_stride : 0;
  B.sel_store = h->d_sel;
  B.copy_sel = (slots_dev && copy_sel) ? 1 : 0;
  B.ypart = h->d_bypart;
  B.ola_state = h->d_ola;
  B.done = h->d_done;
  B.counter = h->d_counter;
  B.bus_rows = h->mixdown ? 1 : 0;
  B.defer_count = h->d_defer;
  B.defer_list = h->d_defer + 1;
  B.from_list = 0;
  const int groups = ((n_blocks + 1) / 2 + h->b_tb - 1) / h->b_tb;
  const int grid = 8 * ((2 * h->n_bmac + 7) / 8) * groups;   // k_tmac's XCD-aware index space
  TimingSet* ts = nullptr;
  if (h->timing && !h->capturing) {
    ts = &h->tsets[h->tnext];
    h->tnext = (h->tnext + 1) % kTimingRing;
    drain_timing(h, *ts);
    ts->mode = 0;          // three phases: spectra, MAC, overlap-add
    ts->blocks = n_blocks;
  }
  HIP_TRY(h, tvx::launch_batch(B, h->dtype, h->bshape, grid, in, in_stride, h->d_hist, h->d_ola, out, out_stride,
                               h->stream, ts ? ts->ev : nullptr));
  if (ts) ts->pending = true;
  return TVOLAP_OK;
}

}  // namespace

extern "C" {

int tvolap_reset(tvolap_t* h) {
  if (!h) return TVOLAP_EINVAL;
  return reset_state(h);
}

int tvolap_configure(tvolap_t* h, int32_t fused, int32_t chunk, int32_t waves, int32_t grid) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "cannot reconfigure during graph capture");
  if (chunk < 0 || grid < 0) return fail(h, TVOLAP_EINVAL, "chunk and grid must be >= 0");
  if (waves != 0 && waves != 4 && waves != 8) return fail(h, TVOLAP_EINVAL, "waves must be 0, 4 or 8");
  if (fused < 0 || fused > 2) return fail(h, TVOLAP_EINVAL, "fused must be 0, 1 or 2");
  if (h->mixdown && fused != 0) return fail(h, TVOLAP_EINVAL, "a mixdown runs with fused = 0");
  MacChoice c;
  c.fused = fused;
  c.chunk = chunk;
  c.waves = waves == 0 ? 4 : waves;
  c.grid = grid;
  return apply_choice(h, c);
}

int tvolap_configure_batch(tvolap_t* h, int32_t chunk, int32_t vec, int32_t waves, int32_t time_block,
                           int32_t group, int32_t engine) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "cannot reconfigure during graph capture");
  if (chunk < 0) return fail(h, TVOLAP_EINVAL, "chunk must be >= 0");
  if (vec != 0 && vec != 1 && vec != 2) return fail(h, TVOLAP_EINVAL, "vec must be 0, 1 or 2");
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(h, TVOLAP_EINVAL, "waves must be 0, 1, 2, 4 or 8 (8: matrix cores only)");
  if (time_block != 0 && time_block != 8 && time_block != 16 && time_block != 32)
    return fail(h, TVOLAP_EINVAL, "time_block must be 0, 8, 16 or 32");
  if (time_block == 32 && engine != 2) return fail(h, TVOLAP_EINVAL, "time_block 32 needs the matrix-core engine");
  if (time_block == 16 && vec == 2) return fail(h, TVOLAP_EINVAL, "time_block 16 needs vec 1");
  if (group != 0 && group != 1 && group != 2) return fail(h, TVOLAP_EINVAL, "group must be 0, 1 or 2");
  if (engine < 0 || engine > 2) return fail(h, TVOLAP_EINVAL, "engine must be 0, 1 or 2");
  if (engine == 2 && (vec == 2 || time_block == 8))
    return fail(h, TVOLAP_EINVAL, "the matrix-core engine runs vec 1 and time groups of 16");
  BatchChoice c;
  c.engine = engine;
  c.chunk = chunk;
  c.vec = vec;
  c.waves = waves;
  c.time_block = time_block;
  c.group = group;
  return apply_batch_choice(h, c);
}

int tvolap_autotune_batch(tvolap_t* h, int32_t iters, float* best_us) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "cannot autotune during graph capture");
  if (iters < 1) return fail(h, TVOLAP_EINVAL, "iters must be >= 1");
  const std::string key = "batch/" + std::to_string(h->max_batch) + "/" + std::to_string(h->K) + "/" + tune_key(h);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_btune_cache.find(key);
    if (it != g_btune_cache.end()) {
      RC_TRY(apply_batch_choice(h, it->second));
      if (best_us) *best_us = -1.f;
      return reset_state(h);
    }
  }
  const int N = 2 * h->L;
  const int nb = h->max_batch;
  // candidate chunks: about 1/2 to 8 workgroups per compute unit for a full batch
  int64_t units = 0;
  {
    std::vector<int> maxM(h->I, 0);
    for (int c = 0; c < h->C; ++c) maxM[h->ch_input[c]] = std::max(maxM[h->ch_input[c]], h->ch_M[c]);
    for (int i = 0; i < h->I; ++i) units += maxM[i];
  }
  std::vector<int> tbs = {8};
  if (nb >= 32) tbs.push_back(16);
  if (nb >= 64) tbs.push_back(32);   // matrix cores only
  // zero input and scratch output of one full batch, for the timing only.
  // Every exit goes through `finish`: buffers and events are released, and on
  // an error the schedule in force before the call is applied again.
  const BatchChoice prev = h->bchoice;
  float* tin = nullptr;
  float* tout = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timing_was = h->timing;
  auto finish = [&](int rc) {
    (void)hipStreamSynchronize(h->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(tin);
    dfree(tout);
    h->timing = timing_was;
    if (rc != TVOLAP_OK) {
      const std::string msg = h->err;
      (void)apply_batch_choice(h, prev);
      (void)reset_state(h);
      h->err = msg;
    }
    return rc;
  };
  if (dalloc(&tin, (size_t)h->I * nb * h->L * sizeof(float)) != hipSuccess ||
      dalloc(&tout, (size_t)h->C * nb * h->L * sizeof(float)) != hipSuccess)
    return finish(fail(h, TVOLAP_ENOMEM, "autotuner buffers"));
  if (tvx::launch_fill_zero(tin, (size_t)h->I * nb * h->L * sizeof(float), h->stream) != hipSuccess)
    return finish(fail(h, TVOLAP_EDEVICE, "autotuner buffers"));
  const int64_t ist = (int64_t)nb * h->L;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return finish(fail(h, TVOLAP_EDEVICE, "hipEventCreate"));
  h->timing = false;
  BatchChoice best;
  float best_t = 1e30f;
  int rc = TVOLAP_OK;
  const std::vector<int> vecs = {1, 2};
  int fan = 1;
  {
    std::vector<int> cnt(h->I, 0);
    for (int c = 0; c < h->C; ++c) fan = std::max(fan, ++cnt[h->ch_input[c]]);
  }
  std::vector<int> groups = {fan >= 2 ? 2 : 1};
  if (fan >= 2) groups.push_back(1);
  const std::vector<int> engines = {1, 2};
  for (int eng : engines)
  for (int grp : groups)
  for (int tb : tbs)
  for (int vec : vecs) {
    if (eng == 1 && ((tb == 16 && vec != 1) || tb == 32)) continue;
    if (eng == 2 && (tb == 8 || vec != 1)) continue;
    const int tgroups = 2 * (((nb + 1) / 2 + tb - 1) / tb);
    for (int nw : {1, 2, 4, 8}) {
      if ((eng == 2) != (nw >= 4)) continue;   // matrix cores: 4 or 8 waves; vector ALU: up to 4
      const int tw = (eng == 2 ? 16 : 64) * vec * nw;
      if (tw > N) continue;
      const int tiles = N / tw;
      std::vector<int> chunks;
      for (int half_per_cu : {1, 2, 4, 8, 16}) {
        const int64_t target = (int64_t)half_per_cu * h->n_cu / 2;
        const int64_t work = units * tiles * tgroups;
        const int S = (int)std::max<int64_t>(2, (work + target - 1) / target);
        if (std::find(chunks.begin(), chunks.end(), S) == chunks.end()) chunks.push_back(S);
      }
      for (int S : chunks) {
        BatchChoice c;
        c.chunk = S;
        c.vec = vec;
        c.waves = nw;
        c.time_block = tb;
        c.group = grp;
        c.engine = eng;
        rc = apply_batch_choice(h, c);
        if (rc != TVOLAP_OK) break;
        // every block of the batch selects slot (block mod K), as a switching
        // stream does; the handle's own selection is left as it was
        rc = enqueue_blocks(h, tin, ist, nb, tout, ist, h->d_tune_bsel, h->C, false);
        if (rc != TVOLAP_OK) break;
        if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(h, TVOLAP_EDEVICE, "event record"); break; }
        for (int k = 0; k < iters && rc == TVOLAP_OK; ++k)
          rc = enqueue_blocks(h, tin, ist, nb, tout, ist, h->d_tune_bsel, h->C, false);
        if (rc != TVOLAP_OK) break;
        if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(h, TVOLAP_EDEVICE, "event synchronize");
          break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = 1e3f * ms / (float)(iters * nb);
        if (us < best_t) {
          best_t = us;
          best = h->bchoice;
        }
      }
      if (rc != TVOLAP_OK) break;
    }
    if (rc != TVOLAP_OK) break;
  }
  if (rc == TVOLAP_OK && best_t >= 1e30f) rc = fail(h, TVOLAP_EDEVICE, "autotuner found no candidate");
  if (rc == TVOLAP_OK) rc = apply_batch_choice(h, best);
  if (rc != TVOLAP_OK) return finish(rc);
  (void)finish(TVOLAP_OK);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_btune_cache[key] = best;
  }
  if (best_us) *best_us = best_t;
  return reset_state(h);
}

int tvolap_autotune(tvolap_t* h, int32_t iters, float* best_us) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "cannot autotune during graph capture");
  if (iters < 1) return fail(h, TVOLAP_EINVAL, "iters must be >= 1");
  const std::string key = tune_key(h);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      RC_TRY(apply_choice(h, it->second));
      if (best_us) *best_us = -1.f;
      return reset_state(h);
    }
  }
  // candidate chunk sizes: about 1 to 16 work items per CU
  const int N = 2 * h->L;
  const int V = (h->dtype == 0) ? 2 : std::min(4, N / 64);
  const int T = N / (64 * V);
  int64_t units = 0;
  {
    std::vector<int> maxM(h->I, 0);
    for (int c = 0; c < h->C; ++c) maxM[h->ch_input[c]] = std::max(maxM[h->ch_input[c]], h->ch_M[c]);
    for (int i = 0; i < h->I; ++i) units += (int64_t)maxM[i] * T;
  }
  std::vector<int> chunks;
  for (int per_cu : {1, 2, 4, 8, 16}) {
    const int64_t target = (int64_t)per_cu * h->n_cu;
    const int S = (int)std::max<int64_t>(2, (units + target - 1) / target);
    if (std::find(chunks.begin(), chunks.end(), S) == chunks.end()) chunks.push_back(S);
  }
  // on an error the schedule in force before the call is applied again
  const MacChoice prev = h->choice;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timing_was = h->timing;
  auto restore = [&](int rc) {
    (void)hipStreamSynchronize(h->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    h->timing = timing_was;
    const std::string msg = h->err;
    (void)apply_choice(h, prev);
    (void)reset_state(h);
    h->err = msg;
    return rc;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return restore(fail(h, TVOLAP_EDEVICE, "hipEventCreate"));
  h->timing = false;
  MacChoice best;
  float best_t = 1e30f;
  int rc = TVOLAP_OK;
  const std::vector<int> vecs = h->dtype == 0 ? std::vector<int>{2} : std::vector<int>{2, 4};
  const std::vector<int> modes = h->mixdown ? std::vector<int>{0} : std::vector<int>{1, 2};
  for (int vec : vecs)
  for (int mode : modes)
  for (int S : chunks) {
    for (int nw : {4, 8}) {
      for (int gmul : {0, 1, 2, 4}) {
        MacChoice c;
        c.fused = mode;
        c.vec = vec;
        c.chunk = S;
        c.waves = nw;
        c.grid = gmul * h->n_cu;
        rc = apply_choice(h, c);
        if (rc != TVOLAP_OK) break;
        if (gmul > 0 && c.grid >= (int)h->items.size()) continue;
        // every block selects another slot, as a switching stream does, so the
        // timed traffic is not served from a cache that holds a single slot
        for (int k = 0; k < 2 && rc == TVOLAP_OK; ++k)
          rc = enqueue_block(h, h->d_zero_in, h->L, h->d_tune_out, h->L, h->d_tune_sel + (size_t)(k % h->K) * h->C,
                             false);
        if (rc != TVOLAP_OK) break;
        if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(h, TVOLAP_EDEVICE, "event record"); break; }
        for (int k = 0; k < iters && rc == TVOLAP_OK; ++k)
          rc = enqueue_block(h, h->d_zero_in, h->L, h->d_tune_out, h->L, h->d_tune_sel + (size_t)(k % h->K) * h->C,
                             false);
        if (rc != TVOLAP_OK) break;
        if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(h, TVOLAP_EDEVICE, "event synchronize");
          break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = 1e3f * ms / (float)iters;
        if (us < best_t) {
          best_t = us;
          best = h->choice;
          best.grid = c.grid;
        }
      }
      if (rc != TVOLAP_OK) break;
    }
    if (rc != TVOLAP_OK) break;
  }
  if (rc == TVOLAP_OK && best_t >= 1e30f) rc = fail(h, TVOLAP_EDEVICE, "autotuner found no candidate");
  if (rc == TVOLAP_OK) rc = apply_choice(h, best);
  if (rc != TVOLAP_OK) return restore(rc);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->timing = timing_was;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  if (best_us) *best_us = best_t;
  return reset_state(h);
}

int tvolap_capture_begin(tvolap_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "capture already active");
  if (!h->stream) return fail(h, TVOLAP_ESTATE, "graph capture needs a non-null stream");
  HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
  h->capturing = true;
  return TVOLAP_OK;
}

int tvolap_capture_end(tvolap_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (!h->capturing) return fail(h, TVOLAP_ESTATE, "no capture active");
  hipGraph_t g = nullptr;
  h->capturing = false;
  HIP_TRY(h, hipStreamEndCapture(h->stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(h, e, "hipGraphInstantiate");
  }
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph = g;
  h->graph_exec = ex;
  return TVOLAP_OK;
}

int tvolap_graph_launch(tvolap_t* h) {
  if (!h) return TVOLAP_EINVAL;
  if (!h->graph_exec) return fail(h, TVOLAP_ESTATE, "no captured graph");
  if (h->capturing) return fail(h, TVOLAP_ESTATE, "capture active");
  HIP_TRY(h, hipGraphLaunch(h->graph_exec, h->stream));
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
  for (int i = 0; i < h->I; ++i) si += h->in_Mdata[i];
  info->sum_partitions = sm;
  info->sum_input_partitions = si;
  // The MAC reads the M_c active partition spectra of every channel and, per
  // input, the M_i same-parity delay-line spectra (shared by the channels of
  // that input).
  info->mac_bytes_per_block = (sm + si) * N * (int64_t)h->store_bytes;
  info->block_bytes = info->mac_bytes_per_block + (int64_t)h->I * N * h->store_bytes  // new spectra
                      + (int64_t)h->I * h->L * 4 * 3                                  // input + history r/w
                      + (int64_t)h->C * h->L * 4                                      // output
                      + (int64_t)h->C * 3 * h->L * 4 * 2;                             // overlap state r/w
  info->bank_bytes = h->bank_elems * (int64_t)h->store_bytes;
  info->delay_line_bytes = h->fdl_elems * (int64_t)h->store_bytes;
  info->workspace_bytes = (int64_t)h->n_rows * h->tile_width * 8;
  info->n_work_items = (int32_t)h->items.size();
  info->mac_chunk = h->chunk;
  info->mac_waves = h->shape.NW;
  info->mac_grid = grid_of(h);
  info->fused = h->choice.fused;
  info->n_outputs = h->n_out;
  info->batch_chunk = h->b_chunk;
  info->batch_vec = h->bshape.V;
  info->batch_waves = h->bshape.NW;
  info->batch_tile_width = h->b_tile_width;
  info->batch_work_items = h->n_bmac;
  info->batch_rows = h->n_brows;
  info->batch_time_block = h->b_tb;
  info->batch_group = h->bshape.G;
  info->batch_engine = h->bshape.E == 1 ? 2 : 1;
  info->n_cu = h->n_cu;
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
  h->t_calls = 0;
  return TVOLAP_OK;
}

}  // extern "C"
