// Merging of the gridded adjoints of concurrent solves into shared launches.
//
// Each solve runs on its own host thread and stream.  When a solve reaches a
// full-grid adjoint (the dirty image, or step 4 of Alg. 2) it posts a request
// and waits.  The first waiting thread that finds the device idle becomes the
// leader: it takes every pending request, orders the shared stream after each
// requester's stream, issues one batched adjoint for all of them, reads their
// maxima, and wakes them.  Requests posted while a batch runs form the next
// batch, so a job never waits for another job's iteration to finish, only for
// the launches already on the device (continuous, iteration-level batching).
// Solves in the Gram form also post the restricted adjoints of each new
// active set (point-spread sums and b = Phi_S* V for new atoms, with FP64
// totals): those of all requests in a batch run in one launch per kind and
// one for their final sums.  A request may carry its residual forward (r = V - Phi_S x by the direct
// sums, step 4 of Alg. 2): the leader then runs the residuals of all such
// requests in one shared launch over (job, visibility block) items ahead of
// the shared adjoint, which reads them.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "common.h"

namespace pc {

struct AdjRequest {
  pc_plan* p;
  const c32* vis;
  float* image;
  hipStream_t s;
  const FwdSpec* fwd = nullptr;  // residual to form first into vis (plan order)
  const std::vector<AccJob>* acc = nullptr;  // a restricted-adjoint request instead
  double max_abs = 0;
  int64_t argmax = -1;
  float ms = 0;
  bool done = false;
  std::string error;
  pc_status status = PC_OK;
};

}  // namespace pc

using namespace pc;

struct pc_batcher {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BatchCtx ctx;
  BatchCtx fctx;                       // tables of the shared residual forward
  BatchCtx actx;                       // tables of the shared restricted adjoints
  unsigned long long* keys = nullptr;  // pinned, one per request of a batch
  size_t keys_cap = 0;
  std::vector<hipEvent_t> deps;        // per-request stream-order events

  mutable std::mutex m;
  std::condition_variable cv;
  std::vector<AdjRequest*> pending;
  bool busy = false;
  pc_batcher_stats stats{};
  int64_t nfwd_ = 0;  // residual forwards of the batch being executed (leader only)
  int64_t nacc_ = 0;  // restricted-adjoint sums of that batch
  int nadj_ = 0;      // adjoints of that batch

  ~pc_batcher() {
    ctx.release();
    fctx.release();
    actx.release();
    for (hipEvent_t e : deps) (void)hipEventDestroy(e);
    if (keys) (void)hipHostFree(keys);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (stream) (void)hipStreamDestroy(stream);
  }

  // Runs one batch on the shared stream (called by the leader, without the
  // lock held).  Fills each request's result; throws on a HIP failure.
  void execute(const std::vector<AdjRequest*>& all, float* ms_out, int64_t* nvis_out) {
    const int nall = (int)all.size();
    while (deps.size() < (size_t)nall) {
      hipEvent_t e;
      PC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      deps.push_back(e);
    }
    // every requester's queued work first
    std::vector<AdjRequest*> batch;  // the adjoint requests
    std::vector<AccJob> acc;         // the restricted-adjoint requests' sums
    for (int j = 0; j < nall; ++j) {
      AdjRequest* r = all[j];
      PC_HIP(hipEventRecord(deps[j], r->s));
      PC_HIP(hipStreamWaitEvent(stream, deps[j], 0));
      if (r->acc)
        acc.insert(acc.end(), r->acc->begin(), r->acc->end());
      else
        batch.push_back(r);
    }
    adjoint_acc64_batch(actx, acc, stream);
    nacc_ = (int64_t)acc.size();
    const int n = (int)batch.size();
    if ((size_t)n > keys_cap) {
      if (keys) (void)hipHostFree(keys);
      keys = nullptr;
      keys_cap = 0;
      PC_HIP(hipHostMalloc((void**)&keys, sizeof(unsigned long long) * 2 * n));
      keys_cap = 2 * n;
    }
    std::vector<pc_plan*> plans(n);
    std::vector<const c32*> vis(n);
    std::vector<float*> images(n);
    std::vector<float> scales(n, 1.0f);
    std::vector<FwdJob> fwd;
    int64_t nvis = 0;
    for (int j = 0; j < n; ++j) {
      AdjRequest* r = batch[j];
      plans[j] = r->p;
      vis[j] = r->vis;
      images[j] = r->image;
      nvis += r->p->L;
      if (r->fwd)
        fwd.push_back(FwdJob{r->p->AB, r->p->Cw, r->fwd->atoms, r->fwd->base,
                             const_cast<c32*>(r->vis), r->p->L, r->fwd->natoms});
    }
    forward_residual_batch(fctx, fwd, stream);
    nfwd_ = (int64_t)fwd.size();
    float ms = 0;
    if (n > 0) {
      std::unique_ptr<bool[]> flags(new bool[n]);
      for (int j = 0; j < n; ++j) flags[j] = true;
      PC_HIP(hipEventRecord(e0, stream));
      adjoint_grid_batch(ctx, plans.data(), vis.data(), flags.get(), images.data(), scales.data(),
                         n, stream);
      PC_HIP(hipEventRecord(e1, stream));
      for (int j = 0; j < n; ++j)
        PC_HIP(hipMemcpyAsync(keys + j, plans[j]->maxkey, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, stream));
    }
    PC_HIP(hipStreamSynchronize(stream));
    if (n > 0) PC_HIP(hipEventElapsedTime(&ms, e0, e1));
    for (int j = 0; j < n; ++j) {
      maxkey_decode(keys[j], &batch[j]->max_abs, &batch[j]->argmax);
      batch[j]->ms = ms;
    }
    *ms_out = ms;
    *nvis_out = nvis;
    nadj_ = n;
  }

  void run(AdjRequest* r) {
    std::unique_lock<std::mutex> lk(m);
    pending.push_back(r);
    while (!r->done) {
      if (!busy) {
        busy = true;
        std::vector<AdjRequest*> batch;
        batch.swap(pending);
        lk.unlock();
        std::string err;
        pc_status st = PC_OK;
        float ms = 0;
        int64_t nvis = 0;
        try {
          PC_HIP(hipSetDevice(device));
          execute(batch, &ms, &nvis);
        } catch (const Error& e) {
          err = e.what();
          st = e.status;
        } catch (const std::exception& e) {
          err = e.what();
          st = PC_ERR_DEVICE;
        }
        lk.lock();
        if (st == PC_OK) {
          stats.forwards += nfwd_;
          stats.restricted_adjoints += nacc_;
          if (nadj_ > 0) stats.batches += 1;
          stats.requests += nadj_;
          stats.visibilities += nvis;
          stats.max_batch = std::max(stats.max_batch, (int32_t)batch.size());
          stats.seconds += ms * 1e-3;
        }
        for (AdjRequest* q : batch) {
          q->error = err;
          q->status = st;
          q->done = true;
        }
        busy = false;
        cv.notify_all();
      } else {
        cv.wait(lk);
      }
    }
  }
};

namespace pc {

void batcher_adjoint(pc_batcher* b, pc_plan* p, const c32* vis_sorted, float* image,
                     hipStream_t s, double* max_abs, int64_t* argmax, float* ms,
                     const FwdSpec* fwd) {
  PC_REQUIRE(p->device == b->device, "plan and batcher are on different devices");
  PC_REQUIRE(p->precision == PC_PREC_FP32, "batched adjoint needs an FP32 plan");
  AdjRequest r{p, vis_sorted, image, s, fwd};
  b->run(&r);
  if (r.status != PC_OK) fail(r.status, "batched adjoint: " + r.error);
  *max_abs = r.max_abs;
  *argmax = r.argmax;
  *ms = r.ms;
}

void batcher_restricted_adjoints(pc_batcher* b, pc_plan* p, hipStream_t s,
                                 const std::vector<AccJob>& sums) {
  PC_REQUIRE(p->device == b->device, "plan and batcher are on different devices");
  AdjRequest r{p, nullptr, nullptr, s};
  r.acc = &sums;
  b->run(&r);
  if (r.status != PC_OK) fail(r.status, "batched restricted adjoints: " + r.error);
}

}  // namespace pc

extern "C" {

PC_API pc_status pc_batcher_create(int32_t device, pc_batcher** out) {
  if (!out) {
    set_last_error("pc_batcher_create: out is NULL");
    return PC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  pc_batcher* b = new (std::nothrow) pc_batcher();
  if (!b) {
    set_last_error("pc_batcher_create: host allocation failed");
    return PC_ERR_OUT_OF_MEMORY;
  }
  try {
    int count = 0;
    PC_HIP(hipGetDeviceCount(&count));
    PC_REQUIRE(device >= 0 && device < count, "device index out of range");
    b->device = device;
    PC_HIP(hipSetDevice(device));
    PC_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    PC_HIP(hipEventCreate(&b->e0));
    PC_HIP(hipEventCreate(&b->e1));
  } catch (const Error& e) {
    set_last_error(std::string("pc_batcher_create: ") + e.what());
    delete b;
    return e.status;
  }
  *out = b;
  return PC_OK;
}

PC_API pc_status pc_batcher_get_stats(const pc_batcher* b, pc_batcher_stats* stats) {
  if (!b || !stats) {
    set_last_error("pc_batcher_get_stats: NULL argument");
    return PC_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(b->m);
  *stats = b->stats;
  return PC_OK;
}

PC_API void pc_batcher_destroy(pc_batcher* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  delete b;
}

}  // extern "C"
