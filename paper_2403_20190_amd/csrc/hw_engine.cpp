// hw_engine.cpp -- serving engine (continuous batching) of the C ABI.
//
// A scheduler thread owns every device call made for requests.  Requests are
// cut into chunks of `chunk` samples.  A chunk starts when one of the stream
// slots is free and its footprint fits in the arena (a first-fit allocator
// over one device allocation); its work is enqueued on the slot's stream:
// copy the chunk's bits, encrypt them (the client's step, on the device),
// train or infer against the resident model, and for inference decrypt the
// PD-act cells and copy them to pinned host memory.  An event marks the end;
// the scheduler polls the events, retires chunks and completes requests.
// Chunks start in submission order (first come, first served; slots that the
// earliest requests cannot use go to later ones).  Requests on one model
// keep their order: a training request waits for every earlier request on
// its model and has at most one chunk in flight (its chunks update the model
// one after another); inference requests behind inference requests overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "hw_ctx.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// first-fit allocator over [0, size) with coalescing of free neighbours
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        sizes_[*off] = bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t bytes = s->second;
    sizes_.erase(s);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_, sizes_;
  size_t used_ = 0, peak_ = 0;
};

struct Job {
  hw_wisard_shape sh;
  Dims d;
  const uint32_t* perm;
  uint32_t* model;
  uint32_t* cnt;
  uint64_t samples;           // trained into the model, plus those of admitted training requests
  std::deque<uint64_t> fifo;  // requests on this model, in submission order
  double xp_train, xp_infer;  // external products per sample of a training / inference request
};

struct Req {
  hw_request r;
  uint64_t seed_x = 0, seed_y = 0;  // encryption seeds of the inputs and labels (hw_request_seeds)
  int state = HW_REQ_QUEUED;
  uint64_t chunks = 0, next = 0, done = 0;
  uint32_t inflight = 0;
  bool cancel = false;
  double t_submit = 0, t_end = 0;
  std::string err;
};

struct Run {
  uint64_t req = 0, chunk = 0, off = 0, m = 0;
  size_t arena_off = 0;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  Run run;
  uint8_t* h_bits = nullptr;    // pinned staging of the chunk's bits and labels
  uint64_t* h_cells = nullptr;  // pinned landing of the decrypted cells
};

}  // namespace

struct hw_engine {
  hw_ctx* ctx = nullptr;
  const int32_t* sk = nullptr;
  uint32_t* skhat = nullptr;
  hw_engine_config cfg{};
  char* arena = nullptr;
  Arena alloc;
  std::vector<Slot> slots;
  std::vector<Job> jobs;
  std::map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;  // unfinished requests, submission order
  uint64_t next_id = 1;
  uint64_t started = 0;
  uint32_t inflight = 0, peak_inflight = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
};

static size_t chunk_bytes(const hw_engine* E, const Job& J, uint32_t kind, uint64_t m) {
  const hw_ctx* c = E->ctx;
  const size_t rg = rgsw_words(c) * 4;
  size_t b = m * (J.sh.s + J.d.L) + 256;                  // bits
  b += m * J.sh.s * rg + 256;                             // input ciphertexts
  if (kind == 0) {
    b += m * J.d.L * rg + 256;                            // label ciphertexts
    b += m * train_ws_per_sample(c, J.d) + 256;           // training workspace
  } else {
    const size_t cells = (size_t)m * J.sh.l * J.d.k0;
    b += cells * lwe_words(c) * 4 + 256;                  // PD-act LWE scores
    b += cells * 8 + 256;                                 // decrypted cells
    b += m * infer_ws_per_sample(c, &J.sh, J.d) + 256;    // inference workspace
  }
  return b;
}

static char* carve(char*& p, size_t bytes) {
  char* r = p;
  p += (bytes + 255) & ~(size_t)255;
  return r;
}

// enqueue one chunk on a slot (scheduler thread)
static hw_status launch_chunk(hw_engine* E, Slot& S, Req& R, const Job& J) {
  hw_ctx* c = E->ctx;
  const Run& run = S.run;
  const uint64_t m = run.m, o = run.off, s = J.sh.s, L = J.d.L;
  char* p = E->arena + run.arena_off;
  uint8_t* d_bits = reinterpret_cast<uint8_t*>(carve(p, m * (s + L)));
  uint32_t* xr = reinterpret_cast<uint32_t*>(carve(p, m * s * rgsw_words(c) * 4));
  memcpy(S.h_bits, R.r.bits_host + o * s, m * s);
  if (R.r.kind == 0 && L) memcpy(S.h_bits + m * s, R.r.labels_host + o * L, m * L);
  HIP_TRY(hipMemcpyAsync(d_bits, S.h_bits, m * (s + (R.r.kind == 0 ? L : 0)), hipMemcpyHostToDevice, S.st));
  hw::EncArgs A{};
  A.sk = E->sk;
  A.sk_hat = E->skhat;
  A.bits = d_bits;
  A.out = xr;
  A.seed = R.seed_x;
  A.ct0 = o * s;
  A.log_base = c->prm.log_base;
  const double rows_per_bit = 2.0 * c->prm.digits * c->prm.nq;
  HIP_TRY(tuned(c, "encrypt_rgsw", (double)m * s * rows_per_bit, S.st, [&](int v) {
    return hw::launch_enc_rgsw(c->logN, c->prm.nq, c->prm.digits, c->tabs, c->cdt, A, m * s, enc_rows_per_wg(v),
                               S.st);
  }));
  if (R.r.kind == 0) {
    uint32_t* yr = reinterpret_cast<uint32_t*>(carve(p, m * L * rgsw_words(c) * 4));
    if (L) {
      A.bits = d_bits + m * s;
      A.out = yr;
      A.seed = R.seed_y;
      A.ct0 = o * L;
      HIP_TRY(tuned(c, "encrypt_rgsw", (double)m * L * rows_per_bit, S.st, [&](int v) {
        return hw::launch_enc_rgsw(c->logN, c->prm.nq, c->prm.digits, c->tabs, c->cdt, A, m * L,
                                   enc_rows_per_wg(v), S.st);
      }));
    }
    const size_t wsb = m * train_ws_per_sample(c, J.d);
    uint32_t* ws = reinterpret_cast<uint32_t*>(carve(p, wsb));
    hw_status st = train_core(c, &J.sh, J.d, J.perm, xr, yr, m, J.model, J.cnt, ws, wsb, S.st, false);
    if (st) return st;
  } else {
    const size_t cells = (size_t)m * J.sh.l * J.d.k0;
    uint32_t* scores = reinterpret_cast<uint32_t*>(carve(p, cells * lwe_words(c) * 4));
    uint64_t* d_cells = reinterpret_cast<uint64_t*>(carve(p, cells * 8));
    const size_t wsb = m * infer_ws_per_sample(c, &J.sh, J.d);
    uint32_t* ws = reinterpret_cast<uint32_t*>(carve(p, wsb));
    hw_status st = infer_core(c, &J.sh, J.d, J.perm, J.model, xr, m, scores, nullptr, ws, wsb, S.st, false);
    if (st) return st;
    HIP_TRY(hw::launch_dec_lwe(c->logN, c->prm.nq, c->tabs, c->crt, E->sk, scores, cells, d_cells, S.st));
    HIP_TRY(hipMemcpyAsync(S.h_cells, d_cells, cells * 8, hipMemcpyDeviceToHost, S.st));
  }
  HIP_TRY(hipEventRecord(S.ev, S.st));
  return HW_OK;
}

static void finish_request(hw_engine* E, uint64_t id, Req& R, int state) {
  R.state = state;
  R.t_end = now_ms();
  Job& J = E->jobs[R.r.job];
  J.fifo.erase(std::remove(J.fifo.begin(), J.fifo.end(), id), J.fifo.end());
  E->active.erase(std::remove(E->active.begin(), E->active.end(), id), E->active.end());
  E->cv.notify_all();
}

// Per-model order: a training request starts only at the front of its
// model's FIFO (every earlier request, training or inference, has finished);
// an inference request starts once every request ahead of it is an
// inference (they only read the model), so it sees exactly the training
// submitted before it and no later training can change the model under it.
static bool may_start(const hw_engine* E, const Job& J, uint64_t id, const Req& R) {
  for (uint64_t f : J.fifo) {
    if (f == id) return true;
    if (R.r.kind == 0) return false;
    const auto it = E->reqs.find(f);
    if (it == E->reqs.end() || it->second.r.kind == 0) return false;
  }
  return false;
}

static void scheduler(hw_engine* E) {
  hipSetDevice(E->ctx->device);
  std::unique_lock<std::mutex> lk(E->mu);
  while (true) {
    bool progress = false;
    // retire finished chunks
    for (Slot& S : E->slots) {
      if (!S.busy) continue;
      const hipError_t q = hipEventQuery(S.ev);
      if (q == hipErrorNotReady) continue;
      Req& R = E->reqs[S.run.req];
      const Job& J = E->jobs[R.r.job];
      if (q != hipSuccess) {
        R.err = hipGetErrorString(q);
        R.cancel = true;
        R.state = HW_REQ_FAILED;
      } else if (R.r.kind == 1) {
        const size_t cells = (size_t)S.run.m * J.sh.l * J.d.k0;
        memcpy(R.r.cells_host + S.run.off * J.sh.l * J.d.k0, S.h_cells, cells * 8);
      }
      E->alloc.release(S.run.arena_off);
      S.busy = false;
      E->inflight -= 1;
      R.inflight -= 1;
      R.done += 1;
      progress = true;
      const bool all = R.done == R.chunks;
      if (R.inflight == 0 && (all || R.cancel))
        finish_request(E, S.run.req, R, R.state == HW_REQ_FAILED ? HW_REQ_FAILED
                                                                 : (all ? HW_REQ_DONE : HW_REQ_CANCELLED));
    }
    // start chunks in the configured order (submission order, or the least
    // remaining work first): a request takes every free slot it can use before
    // the next one gets one; the slots it cannot use -- a training request
    // runs one chunk at a time, a request may be waiting for an earlier one on
    // its model or for arena memory -- go to the next requests
    std::vector<uint64_t> order(E->active);
    if (E->cfg.order == HW_ORDER_SHORTEST) {
      auto left = [&](uint64_t id) {
        const Req& R = E->reqs[id];
        const Job& J = E->jobs[R.r.job];
        const uint64_t started = std::min<uint64_t>(R.r.n, R.next * E->cfg.chunk);
        return (double)(R.r.n - started) * (R.r.kind == 0 ? J.xp_train : J.xp_infer);
      };
      std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return left(a) < left(b); });
    }
    bool slots_left = true;
    for (uint64_t id : order) {
      if (!slots_left) break;
      Req& R = E->reqs[id];
      Job& J = E->jobs[R.r.job];
      if (R.state >= HW_REQ_DONE) continue;  // finished earlier in this pass
      if (R.cancel) {
        if (R.inflight == 0) finish_request(E, id, R, R.state == HW_REQ_FAILED ? HW_REQ_FAILED : HW_REQ_CANCELLED);
        continue;
      }
      if (!may_start(E, J, id, R)) continue;  // an earlier request on this model must finish first
      while (R.next < R.chunks && !R.cancel && !(R.r.kind == 0 && R.inflight > 0)) {  // training: one at a time
        Slot* free_slot = nullptr;
        for (Slot& S : E->slots)
          if (!S.busy) {
            free_slot = &S;
            break;
          }
        if (!free_slot) {
          slots_left = false;
          break;
        }
        const uint64_t off = R.next * E->cfg.chunk;
        const uint64_t m = std::min<uint64_t>(E->cfg.chunk, R.r.n - off);
        size_t ao = 0;
        if (!E->alloc.alloc(chunk_bytes(E, J, R.r.kind, m), &ao)) break;  // wait for memory
        Slot& S = *free_slot;
        S.run = Run{id, R.next, off, m, ao};
        S.busy = true;
        R.state = HW_REQ_RUNNING;
        R.next += 1;
        R.inflight += 1;
        E->inflight += 1;
        E->peak_inflight = std::max(E->peak_inflight, E->inflight);
        E->started += 1;
        progress = true;
        const hw_status st = launch_chunk(E, S, R, J);
        if (st != HW_OK) {
          // nothing of this chunk may still run: wait for the slot before reuse
          (void)hipStreamSynchronize(S.st);
          R.err = hw_last_error();
          R.state = HW_REQ_FAILED;
          R.cancel = true;
          E->alloc.release(ao);
          S.busy = false;
          E->inflight -= 1;
          R.inflight -= 1;
          if (R.inflight == 0) finish_request(E, id, R, HW_REQ_FAILED);
        }
      }
    }
    if (E->stop && E->inflight == 0) break;
    if (!progress) {
      // wake on new submissions, otherwise poll the events again shortly
      E->cv.wait_for(lk, std::chrono::microseconds(E->inflight ? 50 : 2000));
    }
  }
}

extern "C" hw_status hw_engine_create(const hw_params* params, int device, const int32_t* sk_dev,
                                      const hw_engine_config* cfg, hw_engine** out) {
  if (!params || !sk_dev || !cfg || !out) return fail(HW_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 16) return fail(HW_EINVAL, "slots must be 1..16");
  if (cfg->chunk < 1) return fail(HW_EINVAL, "chunk must be >= 1");
  if (cfg->max_s < 1 || cfg->max_cells < 1) return fail(HW_EINVAL, "max_s and max_cells must be >= 1");
  if (cfg->order > HW_ORDER_SHORTEST) return fail(HW_EINVAL, "order must be HW_ORDER_FIFO or HW_ORDER_SHORTEST");
  hw_ctx* c = nullptr;
  CHECK(hw_ctx_create(params, device, &c));
  hw_engine* E = new hw_engine();
  E->ctx = c;
  E->sk = sk_dev;
  E->cfg = *cfg;
  auto bail = [&](hw_status st) {
    hw_engine_destroy(E);
    return st;
  };
  hipError_t e = hipMalloc(&E->skhat, sizeof(uint32_t) * sk_hat_words(c));
  if (e == hipSuccess) e = hw::launch_sk_hat(c->logN, c->prm.nq, c->tabs, sk_dev, E->skhat, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMalloc(&E->arena, cfg->arena_bytes);
  if (e != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? HW_ENOMEM : HW_EDEVICE, "engine set-up: %s", hipGetErrorString(e)));
  E->alloc.reset(cfg->arena_bytes);
  E->slots.resize(cfg->slots);
  for (Slot& S : E->slots) {
    e = hipStreamCreateWithFlags(&S.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S.h_bits), (size_t)cfg->chunk * (cfg->max_s + 8));
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&S.h_cells), (size_t)cfg->chunk * cfg->max_cells * 8);
    if (e != hipSuccess) return bail(fail(HW_EDEVICE, "engine slot set-up: %s", hipGetErrorString(e)));
  }
  E->th = std::thread(scheduler, E);
  *out = E;
  return ok();
}

extern "C" void hw_engine_destroy(hw_engine* E) {
  if (!E) return;
  if (E->th.joinable()) {
    {
      std::lock_guard<std::mutex> g(E->mu);
      E->stop = true;
      for (uint64_t id : E->active) E->reqs[id].cancel = true;
    }
    E->cv.notify_all();
    E->th.join();
  }
  hipSetDevice(E->ctx ? E->ctx->device : 0);
  for (Slot& S : E->slots) {
    if (S.st) (void)hipStreamSynchronize(S.st);
    if (S.ev) (void)hipEventDestroy(S.ev);
    if (S.st) (void)hipStreamDestroy(S.st);
    if (S.h_bits) (void)hipHostFree(S.h_bits);
    if (S.h_cells) (void)hipHostFree(S.h_cells);
  }
  if (E->arena) (void)hipFree(E->arena);
  if (E->skhat) (void)hipFree(E->skhat);
  if (E->ctx) hw_ctx_destroy(E->ctx);
  delete E;
}

// the request's two encryption seeds: draws 0 and 1 of the library's
// generator in domain DOM_REQ keyed by enc_seed, so that the input and label
// streams of one request, and those of requests with different enc_seed, are
// keyed apart (no arithmetic relation between seeds makes two streams equal)
constexpr uint32_t DOM_REQ = 6;

extern "C" hw_status hw_request_seeds(uint64_t enc_seed, uint64_t* seed_x, uint64_t* seed_y) {
  if (!seed_x || !seed_y) return fail(HW_EINVAL, "null argument");
  *seed_x = lib_draw64(enc_seed, DOM_REQ, 0);
  *seed_y = lib_draw64(enc_seed, DOM_REQ, 1);
  return ok();
}

extern "C" hw_status hw_engine_add_job(hw_engine* E, const hw_wisard_shape* sh, uint32_t* model,
                                       uint32_t* cnt, uint64_t trained, uint32_t* job_id) {
  if (!E || !sh || !model || !job_id) return fail(HW_EINVAL, "null argument");
  Job J{};
  CHECK(check_shape(E->ctx, sh, &J.d));
  if (trained > E->ctx->prm.plain_mod - 1)
    return fail(HW_EINVAL, "trained = %llu: a model holds at most p - 1 = %llu samples",
                (unsigned long long)trained, (unsigned long long)(E->ctx->prm.plain_mod - 1));
  J.samples = trained;
  if (sh->s > E->cfg.max_s) return fail(HW_EINVAL, "s = %u exceeds the engine's max_s %u", sh->s, E->cfg.max_s);
  if ((uint64_t)sh->l * J.d.k0 > E->cfg.max_cells) return fail(HW_EINVAL, "l * k0 exceeds the engine's max_cells");
  if (J.d.L > 8) return fail(HW_EINVAL, "too many label bits for the engine's staging");
  HIP_TRY(hipSetDevice(E->ctx->device));
  CHECK(perm_for(E->ctx, sh, nullptr, &J.perm));
  J.sh = *sh;
  J.model = model;
  J.cnt = cnt;
  J.xp_train = 0;
  for (uint32_t j = 0; j < J.d.k0; ++j)
    J.xp_train += ivp_xp(J.d.L + std::min(sh->a, sh->s - j * sh->a), E->ctx->logN, J.d.pL, J.d.pl);
  J.xp_infer = infer_xp_per_sample(E->ctx, sh, J.d);
  std::lock_guard<std::mutex> g(E->mu);
  *job_id = (uint32_t)E->jobs.size();
  E->jobs.push_back(J);
  return ok();
}

extern "C" hw_status hw_engine_submit(hw_engine* E, const hw_request* r, uint64_t* id) {
  if (!E || !r || !id) return fail(HW_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(E->mu);
  if (r->job >= E->jobs.size()) return fail(HW_EINVAL, "unknown job %u", r->job);
  if (r->kind > 1) return fail(HW_EINVAL, "kind must be 0 (train) or 1 (infer)");
  const Job& J = E->jobs[r->job];
  if (r->n == 0) return fail(HW_EINVAL, "empty request");
  if (!r->bits_host) return fail(HW_EINVAL, "null input bits");
  if (r->kind == 0 && J.d.L && !r->labels_host) return fail(HW_EINVAL, "null label bits");
  if (r->kind == 1 && !r->cells_host) return fail(HW_EINVAL, "null output cells");
  const uint64_t m = std::min<uint64_t>(E->cfg.chunk, r->n);
  if (chunk_bytes(E, J, r->kind, m) > E->cfg.arena_bytes)
    return fail(HW_EBUSY, "a chunk of this request needs more device memory than the engine's arena");
  // Training adds Delta per sample to a cell and to the class counter, so a
  // count reaching p would wrap (Sec. 2.5.1 encoding): refuse a request that
  // could take the model past p - 1 samples.  Admitted requests count in full
  // (a cancelled one may have run some chunks).
  const uint64_t cap = E->ctx->prm.plain_mod - 1;
  if (r->kind == 0 && (J.samples > cap || r->n > cap - J.samples))
    return fail(HW_EINVAL, "training %llu more samples would take the model to %llu samples: counters hold at "
                "most p - 1 = %llu", (unsigned long long)r->n, (unsigned long long)(J.samples + r->n),
                (unsigned long long)cap);
  Req R;
  R.r = *r;
  (void)hw_request_seeds(r->enc_seed, &R.seed_x, &R.seed_y);
  if (r->kind == 0) E->jobs[r->job].samples += r->n;
  R.chunks = (r->n + E->cfg.chunk - 1) / E->cfg.chunk;
  R.t_submit = now_ms();
  *id = E->next_id++;
  E->reqs.emplace(*id, R);
  E->jobs[r->job].fifo.push_back(*id);
  E->active.push_back(*id);
  E->cv.notify_all();
  return ok();
}

static hw_status req_state(hw_engine* E, uint64_t id, int* state, double* latency) {
  auto it = E->reqs.find(id);
  if (it == E->reqs.end()) return fail(HW_EINVAL, "unknown request %llu", (unsigned long long)id);
  const Req& R = it->second;
  if (state) *state = R.state;
  if (latency) *latency = R.t_end > 0 ? R.t_end - R.t_submit : -1.0;
  if (R.state == HW_REQ_FAILED) return fail(HW_EDEVICE, "request failed: %s", R.err.c_str());
  return ok();
}

extern "C" hw_status hw_engine_poll(hw_engine* E, uint64_t id, int* state, double* latency_ms) {
  if (!E) return fail(HW_EINVAL, "null engine");
  std::lock_guard<std::mutex> g(E->mu);
  return req_state(E, id, state, latency_ms);
}

extern "C" hw_status hw_engine_wait(hw_engine* E, uint64_t id, int* state, double* latency_ms) {
  if (!E) return fail(HW_EINVAL, "null engine");
  std::unique_lock<std::mutex> lk(E->mu);
  auto it = E->reqs.find(id);
  if (it == E->reqs.end()) return fail(HW_EINVAL, "unknown request %llu", (unsigned long long)id);
  E->cv.wait(lk, [&] { return it->second.state >= HW_REQ_DONE; });
  return req_state(E, id, state, latency_ms);
}

extern "C" hw_status hw_engine_cancel(hw_engine* E, uint64_t id) {
  if (!E) return fail(HW_EINVAL, "null engine");
  std::lock_guard<std::mutex> g(E->mu);
  auto it = E->reqs.find(id);
  if (it == E->reqs.end()) return fail(HW_EINVAL, "unknown request %llu", (unsigned long long)id);
  if (it->second.state < HW_REQ_DONE) it->second.cancel = true;
  E->cv.notify_all();
  return ok();
}

extern "C" hw_status hw_engine_job_samples(hw_engine* E, uint32_t job, uint64_t* samples, uint64_t* capacity) {
  if (!E) return fail(HW_EINVAL, "null engine");
  std::lock_guard<std::mutex> g(E->mu);
  if (job >= E->jobs.size()) return fail(HW_EINVAL, "unknown job %u", job);
  if (samples) *samples = E->jobs[job].samples;
  if (capacity) *capacity = E->ctx->prm.plain_mod - 1;
  return ok();
}

extern "C" hw_status hw_engine_stats(hw_engine* E, uint64_t* chunks, uint64_t* peak_arena, uint32_t* peak_inflight) {
  if (!E) return fail(HW_EINVAL, "null engine");
  std::lock_guard<std::mutex> g(E->mu);
  if (chunks) *chunks = E->started;
  if (peak_arena) *peak_arena = E->alloc.peak();
  if (peak_inflight) *peak_inflight = E->peak_inflight;
  return ok();
}
