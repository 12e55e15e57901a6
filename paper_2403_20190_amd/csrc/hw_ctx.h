// hw_ctx.h -- the context object behind the C ABI and the host helpers that
// the API (hw_api.cpp) and the serving engine (hw_engine.cpp) share.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hwisard.h"
#include "hw_internal.h"

using hw::Tabs;
typedef unsigned __int128 u128;

// Online tuning of a kernel's schedule: every variant computes the same
// bits; the first launches on a context cycle through the variants between
// HIP events until each has been timed TUNE_RUNS times, then the one with the
// least time per unit of work is kept.
struct TuneState {
  int forced = -1;                 // hw_tune_set
  int chosen = -1;                 // after tuning
  std::vector<double> best;        // per variant: least ms per unit of work seen
  std::vector<int> runs;           // per variant: completed timings
  struct Pend {
    int v;
    hipEvent_t a, b;
    double work;
  };
  std::vector<Pend> pend;
};
constexpr int TUNE_RUNS = 2;

struct hw_ctx;
// the tuned kernels and their variants; nullptr past the last one
const char* tune_variant_name(const char* kernel, int v);
int tune_variants(const hw_ctx* c, const char* kernel);  // variants that exist for c's parameters
int enc_rows_per_wg(int variant);  // "encrypt_rgsw" variant -> RGSW rows per workgroup
double tune_min_work(const char* kernel);

struct hw_ctx {
  hw_params prm;
  int device;
  int logN;
  Tabs tabs;
  hw::CrtTab crt;
  hw::Cdt cdt;
  u128 Q;
  void* d_tables = nullptr;        // twiddle tables of every prime
  uint32_t* d_skhat = nullptr;     // sk_hat_words(): [nq][N] transformed key, then [nq][N] Shoup companions
  void* d_ws = nullptr;            // workspace
  size_t ws_bytes = 0;
  size_t ws_budget = 0;
  // permutations on the device, by (s, seed)
  std::map<std::pair<uint32_t, uint64_t>, uint32_t*> perms;
  // batched training: job/item tables (pinned host staging, device copy), queue counter
  void* h_btab = nullptr;
  void* d_btab = nullptr;
  size_t btab_bytes = 0;
  uint32_t* d_counter = nullptr;   // 64 bytes: word 0 the training queue, word 16 the inference queue
  // batched inference: job/item tables (pinned host staging, device copy)
  void* h_itab = nullptr;
  void* d_itab = nullptr;
  size_t itab_bytes = 0;
  // per-kernel timing
  bool prof = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
    double work;
  };
  std::vector<Rec> pending;
  struct Acc {
    double ms = 0, work = 0;
    uint64_t launches = 0;
  };
  std::map<std::string, Acc> acc;
  // schedule tuning, by kernel name
  bool tune_off = false;
  std::map<std::string, TuneState> tune;
};

// fold finished timings in; choose once every variant has TUNE_RUNS of them
void tune_settle(TuneState& S);

// launch(v) with the variant the tuner picks for `kernel`, timing it while
// tuning (not under stream capture, where the best variant so far is used)
template <class F>
static hipError_t tuned(hw_ctx* c, const char* kernel, double work, hipStream_t st, F&& launch) {
  const int n = tune_variants(c, kernel);
  TuneState& S = c->tune[kernel];
  if ((int)S.runs.size() != n) {
    S.runs.assign(n, 0);
    S.best.assign(n, 1e300);
  }
  if (S.forced >= 0) return launch(S.forced);
  if (S.chosen < 0 && (c->tune_off || n <= 1)) S.chosen = 0;
  if (S.chosen < 0) tune_settle(S);
  if (S.chosen >= 0) return launch(S.chosen);
  int best = 0;
  for (int v = 1; v < n; ++v)
    if (S.best[v] < S.best[best]) best = v;
  if (work < tune_min_work(kernel)) return launch(best);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return launch(best);
  // the variant with the fewest timings, pending ones included
  std::vector<int> cnt(S.runs);
  for (const auto& p : S.pend) cnt[p.v] += 1;
  int v = 0;
  for (int u = 1; u < n; ++u)
    if (cnt[u] < cnt[v]) v = u;
  if (cnt[v] >= TUNE_RUNS) return launch(best);  // all timed; waiting for results
  TuneState::Pend p{v, nullptr, nullptr, work};
  hipError_t e = hipEventCreate(&p.a);
  if (e == hipSuccess) e = hipEventCreate(&p.b);
  if (e == hipSuccess) e = hipEventRecord(p.a, st);
  if (e == hipSuccess) e = launch(v);
  if (e == hipSuccess) e = hipEventRecord(p.b, st);
  if (e == hipSuccess) {
    S.pend.push_back(p);
  } else {
    if (p.a) (void)hipEventDestroy(p.a);
    if (p.b) (void)hipEventDestroy(p.b);
  }
  return e;
}

// the variant `tuned` would settle on without timing anything (no events are
// created): the forced one, else the tuner's choice, else variant 0
static int settled_variant(const hw_ctx* c, const char* kernel) {
  const auto it = c->tune.find(kernel);
  if (it == c->tune.end()) return 0;
  if (it->second.forced >= 0) return it->second.forced;
  return it->second.chosen >= 0 ? it->second.chosen : 0;
}

// run `launch` between two events on `st` when profiling is on
template <class F>
static hipError_t timed(hw_ctx* c, const char* name, double work, hipStream_t st, F&& launch) {
  if (!c->prof) return launch();
  hw_ctx::Rec r{name, nullptr, nullptr, work};
  hipError_t e = hipEventCreate(&r.a);
  if (e == hipSuccess) e = hipEventCreate(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(r.b, st);
  if (e == hipSuccess) c->pending.push_back(r);
  return e;
}

static size_t rlwe_words(const hw_ctx* c) { return (size_t)2 * c->prm.nq * c->prm.N; }
static size_t rgsw_words(const hw_ctx* c) { return (size_t)2 * c->prm.digits * c->prm.nq * rlwe_words(c); }
static size_t lwe_words(const hw_ctx* c) { return (size_t)c->prm.nq * (c->prm.N + 1); }

struct Dims {
  uint32_t L, k0, k1, z;
  uint32_t kt;      // 2^z: leaves of a full RAM's IVP tree (k1 of them are model rows)
  uint32_t layout;  // 0: label-pruned rows (label bits lowest in the index); 1: class-packed rows;
                    // 2: class-packed, several RAMs per row
  uint32_t pL, pl;  // label bits at the bottom of the tree and the classes they take: (L, l)
                    // for layout 0; (0, 1) for layouts 1-2, whose tree holds tuple bits only
  uint32_t rpr;     // RAMs per model row: N / 2^(L+a) for layout 2 when that is >= 2, else 1
  uint32_t rows;    // model rows: ceil(k0 / rpr)
  uint32_t nbf;     // L + a: RAM j of layout 2 starts at coefficient (j mod rpr) 2^nbf
};

uint32_t live_rows(uint32_t z, uint32_t L, uint32_t l);
uint32_t ivp_xp(uint32_t nb, int logN, uint32_t L, uint32_t l);
uint32_t live_splits(uint32_t lev, uint32_t z, uint32_t L, uint32_t l);
uint32_t infer_slots(const Dims& d);
double infer_xp_per_sample(const hw_ctx* c, const hw_wisard_shape* sh, const Dims& d);


// error reporting: sets the calling thread's message
hw_status fail(hw_status st, const char* fmt, ...);
hw_status ok();

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? HW_ENOMEM : HW_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                              \
  } while (0)

#define CHECK(expr)            \
  do {                         \
    hw_status s_ = (expr);     \
    if (s_ != HW_OK) return s_; \
  } while (0)

hw_status check_shape(const hw_ctx* c, const hw_wisard_shape* sh, Dims* d);
// 64-bit draw `index` of stream (seed, domain) of the library's generator (Philox4x32-10)
uint64_t lib_draw64(uint64_t seed, uint32_t domain, uint64_t index);
// make the context current on this thread (HW_EINVAL for a null context)
hw_status enter(hw_ctx* c);
// grow the context's workspace to at least `bytes` (waits for the device when it reallocates)
hw_status ensure_ws(hw_ctx* c, size_t bytes);
hw_status perm_for(hw_ctx* c, const hw_wisard_shape* sh, hipStream_t st, const uint32_t** out);

// workspace bytes per sample of one training / inference call
// words of a transformed key buffer (launch_sk_hat's output): values and Shoup companions
inline size_t sk_hat_words(const hw_ctx* c) { return (size_t)2 * c->prm.nq * c->prm.N; }
size_t train_ws_per_sample(const hw_ctx* c, const Dims& d);
size_t infer_ws_per_sample(const hw_ctx* c, const hw_wisard_shape* sh, const Dims& d);

// training / inference of n samples with an explicit workspace of ws_bytes
// (at least one sample's worth) and a resolved device permutation; the
// arguments are not checked again.  `timing` records per-kernel events;
// without `tune` the training kernel runs its settled schedule and no event
// is created.
hw_status train_core(hw_ctx* c, const hw_wisard_shape* sh, const Dims& d, const uint32_t* perm,
                     const uint32_t* x, const uint32_t* y, uint64_t n, uint32_t* model, uint32_t* cnt,
                     uint32_t* ws, size_t ws_bytes, hipStream_t st, bool timing, bool tune = true);
hw_status infer_core(hw_ctx* c, const hw_wisard_shape* sh, const Dims& d, const uint32_t* perm,
                     const uint32_t* model, const uint32_t* x, uint64_t n, uint32_t* scores, uint32_t* sums,
                     uint32_t* ws, size_t ws_bytes, hipStream_t st, bool timing);
