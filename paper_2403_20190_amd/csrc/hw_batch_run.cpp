// hw_batch_run.cpp -- batches of training and inference jobs over several
// parameter sets (hw_batch_run of the C ABI) and the persistent inference
// queue behind it.
//
// Per context, in the order of the context list: its training jobs run as one
// persistent launch (hw_batch_train), then its inference jobs as one
// persistent launch of k_infer_batch over a queue of (job, RAM, label, piece)
// items.  A kernel is compiled for one ring degree, prime count and RGSW
// gadget, so one launch never spans two contexts; the contexts' launches
// follow each other on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/hwisard.h"
#include "hw_ctx.h"
#include "hw_internal.h"

namespace {

struct IPlan {
  std::vector<hw::IJob> jobs;
  std::vector<hw::IItem> items;
  std::vector<uint32_t> cost;  // external products per item (queue order)
  uint64_t scratch_words = 0;  // per persistent workgroup
  uint32_t grid_occ[2] = {0, 0};
  uint32_t grid = 0;
  double xp = 0;
};

// Validate the inference jobs of one context and cut every (job, RAM,
// label) into pieces of consecutive samples, aimed at 1/8 of one
// workgroup's share of the batch; items longest first.
hw_status plan_infer(hw_ctx* c, const std::vector<const hw_job*>& jobs, hipStream_t st, IPlan& B) {
  for (int v = 0; v < tune_variants(c, "infer_batch"); ++v)
    HIP_TRY(hw::infer_batch_grid(c->logN, c->prm.nq, c->prm.digits, v ? 4 : 3, &B.grid_occ[v]));
  B.grid = std::max(B.grid_occ[0], B.grid_occ[1]);
  std::vector<Dims> dims(jobs.size());
  std::vector<double> unit(jobs.size(), 0.0);  // external products of one (sample, RAM, label) VP, on average
  double W = 0;
  uint32_t slots = 1;
  for (size_t j = 0; j < jobs.size(); ++j) {
    const hw_job& J = *jobs[j];
    CHECK(check_shape(c, &J.shape, &dims[j]));
    const Dims& d = dims[j];
    const uint32_t nlab = d.layout ? 1u : J.shape.l;
    unit[j] = infer_xp_per_sample(c, &J.shape, d) / ((double)d.k0 * nlab);
    W += unit[j] * (double)J.n * d.k0 * nlab;
    slots = std::max(slots, infer_slots(d));
  }
  B.scratch_words = (uint64_t)(slots + 1) * rlwe_words(c);
  const double target = std::max(1.0, W / (8.0 * std::max(1u, B.grid)));
  for (size_t j = 0; j < jobs.size(); ++j) {
    const hw_job& J = *jobs[j];
    const Dims& d = dims[j];
    const uint32_t* perm = nullptr;
    CHECK(perm_for(c, &J.shape, st, &perm));
    hw::IJob b{};
    hw::InferArgs& A = b.args;
    A.model = J.model_dev;
    A.x_rgsw = J.x_rgsw_dev;
    A.perm = perm;
    A.scores = J.ram_scores_dev;
    A.rgsw_words = rgsw_words(c);
    A.s = J.shape.s;
    A.a = J.shape.a;
    A.L = d.L;
    A.l = J.shape.l;
    A.k0 = d.k0;
    A.k1 = d.k1;
    A.slots = infer_slots(d);
    A.layout = d.layout;
    A.nlab = d.layout ? 1u : J.shape.l;
    A.rpr = d.rpr;
    A.nbf = d.layout == 2 ? d.nbf : 0u;
    b.nsmp = (uint32_t)J.n;
    b.per = (uint32_t)std::min<uint64_t>(J.n, std::max<uint64_t>(1, (uint64_t)(target / std::max(1.0, unit[j]))));
    const uint32_t pieces = (uint32_t)((J.n + b.per - 1) / b.per);
    const uint32_t jb = (uint32_t)B.jobs.size();
    for (uint32_t p = 0; p < pieces; ++p) {
      const uint64_t cnt = std::min<uint64_t>(b.per, J.n - (uint64_t)p * b.per);
      for (uint32_t r = 0; r < d.k0; ++r)
        for (uint32_t lab = 0; lab < A.nlab; ++lab) {
          B.items.push_back(hw::IItem{jb, r, lab, p});
          B.cost.push_back((uint32_t)std::min(4e9, (double)cnt * unit[j]));
          B.xp += (double)cnt * unit[j];
        }
    }
    B.jobs.push_back(b);
  }
  if (B.items.size() > 0xFFFFFFFFull) return fail(HW_EINVAL, "too many inference work items");
  std::vector<size_t> ord(B.items.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return B.cost[x] > B.cost[y]; });
  std::vector<hw::IItem> sorted(ord.size());
  for (size_t i = 0; i < ord.size(); ++i) sorted[i] = B.items[ord[i]];
  B.items.swap(sorted);
  return HW_OK;
}

hw_status run_infer(hw_ctx* c, const std::vector<const hw_job*>& jobs, hipStream_t st) {
  IPlan B;
  CHECK(plan_infer(c, jobs, st, B));
  if (B.items.empty()) return HW_OK;
  if (!c->d_counter) HIP_TRY(hipMalloc(&c->d_counter, 64));
  CHECK(ensure_ws(c, 4 * (size_t)B.grid * B.scratch_words));
  const size_t jb = B.jobs.size() * sizeof(hw::IJob), io = (jb + 255) / 256 * 256;
  const size_t need = io + B.items.size() * sizeof(hw::IItem);
  HIP_TRY(hipStreamSynchronize(st));  // an earlier batch on this stream has released the tables
  if (need > c->itab_bytes) {
    if (c->h_itab) HIP_TRY(hipHostFree(c->h_itab));
    if (c->d_itab) HIP_TRY(hipFree(c->d_itab));
    c->h_itab = c->d_itab = nullptr;
    c->itab_bytes = 0;
    HIP_TRY(hipHostMalloc(&c->h_itab, need));
    HIP_TRY(hipMalloc(&c->d_itab, need));
    c->itab_bytes = need;
  }
  char* h = static_cast<char*>(c->h_itab);
  memcpy(h, B.jobs.data(), jb);
  memcpy(h + io, B.items.data(), B.items.size() * sizeof(hw::IItem));
  HIP_TRY(hipMemcpyAsync(c->d_itab, c->h_itab, need, hipMemcpyHostToDevice, st));
  char* d = static_cast<char*>(c->d_itab);
  hw::IBatchArgs A{};
  A.jobs = reinterpret_cast<const hw::IJob*>(d);
  A.items = reinterpret_cast<const hw::IItem*>(d + io);
  A.nitems = (uint32_t)B.items.size();
  A.counter = c->d_counter + 16;
  A.ws = static_cast<uint32_t*>(c->d_ws);
  A.scratch_words = B.scratch_words;
  auto li = [&] {
    return tuned(c, "infer_batch", B.xp, st, [&](int v) {
      return hw::launch_infer_batch(c->logN, c->prm.nq, c->prm.digits, c->tabs, A, B.grid_occ[v], v ? 4 : 3, st);
    });
  };
  HIP_TRY(timed(c, "infer_batch", B.xp, st, li));
  for (const hw_job* J : jobs) {
    if (!J->class_scores_dev) continue;
    Dims dd;
    CHECK(check_shape(c, &J->shape, &dd));
    hw::SumArgs S{};
    S.scores = J->ram_scores_dev;
    S.sums = J->class_scores_dev;
    S.n = J->n;
    S.l = J->shape.l;
    S.k0 = dd.k0;
    S.N = c->prm.N;
    S.nq = c->prm.nq;
    HIP_TRY(timed(c, "class_sums", (double)J->n * J->shape.l * lwe_words(c), st,
                  [&] { return hw::launch_class_sums(c->tabs, S, st); }));
  }
  return HW_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

}  // namespace

extern "C" hw_status hw_batch_run(hw_ctx* const* ctxs, uint32_t nctx, const hw_job* jobs, uint32_t njobs,
                                  hipStream_t st) {
  if (njobs == 0) return ok();
  if (!ctxs || !jobs) return fail(HW_EINVAL, "null argument");
  // every check before anything is enqueued
  for (uint32_t j = 0; j < njobs; ++j) {
    const hw_job& J = jobs[j];
    if (J.ctx_index >= nctx || !ctxs[J.ctx_index]) return fail(HW_EINVAL, "job %u: bad ctx_index %u", j, J.ctx_index);
    if (J.kind > 1) return fail(HW_EINVAL, "job %u: kind must be 0 (train) or 1 (infer)", j);
    hw_ctx* c = ctxs[J.ctx_index];
    Dims d;
    hw_status e = check_shape(c, &J.shape, &d);
    if (e) return fail(e, "job %u: %s", j, hw_last_error());
    if (J.n == 0) continue;
    if (J.n > 0xFFFFFFFFull) return fail(HW_EINVAL, "job %u: too many samples", j);
    if (!J.x_rgsw_dev || !J.model_dev) return fail(HW_EINVAL, "job %u: null buffer", j);
    if (J.kind == 0) {
      if (J.shape.layout == 2)
        return fail(HW_EINVAL, "job %u: layout 2 rows are shared by several RAMs; batch-train layout 1 and pack", j);
      if (d.L > 0 && !J.y_rgsw_dev) return fail(HW_EINVAL, "job %u: null label ciphertexts", j);
    } else {
      if (!J.ram_scores_dev) return fail(HW_EINVAL, "job %u: null score buffer", j);
      const size_t mb = (size_t)d.rows * d.k1 * rlwe_words(c) * 4;
      const size_t sb = (size_t)J.n * J.shape.l * d.k0 * lwe_words(c) * 4;
      if (overlaps(J.ram_scores_dev, sb, J.model_dev, mb) ||
          (J.class_scores_dev && overlaps(J.class_scores_dev, (size_t)J.n * J.shape.l * lwe_words(c) * 4,
                                          J.model_dev, mb)))
        return fail(HW_EINVAL, "job %u: scores overlap the model", j);
      if ((uint64_t)d.k0 * (d.layout ? 1u : J.shape.l) * J.n > 0xFFFFFFFFull)
        return fail(HW_EINVAL, "job %u: too many (sample, RAM, label) items", j);
    }
  }
  // outputs of a job must not overlap another job's outputs, nor a model that an inference job reads
  for (uint32_t j = 0; j < njobs; ++j) {
    const hw_job& J = jobs[j];
    if (!J.n) continue;
    hw_ctx* cj = ctxs[J.ctx_index];
    Dims dj;
    (void)check_shape(cj, &J.shape, &dj);
    const size_t mj = (size_t)dj.rows * dj.k1 * rlwe_words(cj) * 4, rwj = rlwe_words(cj) * 4;
    const size_t sj = (size_t)J.n * J.shape.l * dj.k0 * lwe_words(cj) * 4;
    const size_t cj_bytes = (size_t)J.n * J.shape.l * lwe_words(cj) * 4;
    for (uint32_t i = 0; i < j; ++i) {
      const hw_job& I = jobs[i];
      if (!I.n) continue;
      hw_ctx* ci = ctxs[I.ctx_index];
      Dims di;
      (void)check_shape(ci, &I.shape, &di);
      const size_t mi = (size_t)di.rows * di.k1 * rlwe_words(ci) * 4, rwi = rlwe_words(ci) * 4;
      const size_t si = (size_t)I.n * I.shape.l * di.k0 * lwe_words(ci) * 4;
      const size_t ci_bytes = (size_t)I.n * I.shape.l * lwe_words(ci) * 4;
      bool bad = false;
      if (J.kind == 0 && I.kind == 0) {
        bad = overlaps(J.model_dev, mj, I.model_dev, mi) ||
              (J.class_count_dev && I.class_count_dev && overlaps(J.class_count_dev, rwj, I.class_count_dev, rwi));
      } else if (J.kind == 1 && I.kind == 1) {
        bad = overlaps(J.ram_scores_dev, sj, I.ram_scores_dev, si) ||
              (J.class_scores_dev && I.class_scores_dev &&
               overlaps(J.class_scores_dev, cj_bytes, I.class_scores_dev, ci_bytes));
      } else {
        const hw_job& T = J.kind == 0 ? J : I;   // the training job
        const hw_job& F = J.kind == 0 ? I : J;   // the inference job
        const size_t mt = J.kind == 0 ? mj : mi, sf = J.kind == 0 ? si : sj;
        bad = overlaps(F.ram_scores_dev, sf, T.model_dev, mt);
      }
      if (bad) return fail(HW_EINVAL, "jobs %u and %u: overlapping output buffers", i, j);
    }
  }
  for (uint32_t k = 0; k < nctx; ++k) {
    hw_ctx* c = ctxs[k];
    if (!c) continue;
    std::vector<hw_train_job> tr;
    std::vector<const hw_job*> inf;
    for (uint32_t j = 0; j < njobs; ++j) {
      const hw_job& J = jobs[j];
      if (J.ctx_index != k || J.n == 0) continue;
      if (J.kind == 0)
        tr.push_back(hw_train_job{J.shape, J.x_rgsw_dev, J.y_rgsw_dev, J.n, J.model_dev, J.class_count_dev});
      else
        inf.push_back(&J);
    }
    if (tr.empty() && inf.empty()) continue;
    CHECK(enter(c));
    if (!tr.empty()) CHECK(hw_batch_train(c, tr.data(), (uint32_t)tr.size(), st));
    if (!inf.empty()) CHECK(run_infer(c, inf, st));
  }
  return ok();
}
