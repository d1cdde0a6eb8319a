// Serving scheduler of libchfsi: continuous batching of eigensolves on one GPU.
//
// The evolving-matrix setting of the paper (the Hamiltonian changes at every
// step of an outer nonlinear iteration and the lowest eigenpairs are recomputed
// from the previous subspace; introduction and Section 4.2) is served as a
// stream of requests grouped into sequences.
//
//  * `slots` worker threads, each owning one HIP stream (default priority), run
//    admitted solves concurrently; their kernels overlap on the device.
//  * Admission (scheduler.h): the first pending request (submission order)
//    whose sequence is idle and whose device footprint (chfsi_workspace_bytes
//    + its blocks) fits in the remaining budget is started as soon as a slot
//    frees up.
//  * Requests of one sequence run in submission order; the sequence's last Ritz
//    vectors stay on the device and warm-start the next request.
//  * A request runs the same kernels with the same launch shapes whether alone
//    or mixed (launch shapes depend on the problem shape only and each solve
//    has its own scratch), so its result is bitwise identical either way.
//  * Device and pinned host memory come from pools (pool.h) that grow in large
//    chunks: no allocation or free call per request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/chfsi.h"
#include "internal.h"
#include "pool.h"
#include "scheduler.h"

namespace {

struct DeviceChunks {
  void* grab(size_t bytes) {
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void release(void* p) { (void)hipFree(p); }
};
struct PinnedChunks {
  void* grab(size_t bytes) {
    void* p = nullptr;
    return hipHostMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void release(void* p) { (void)hipHostFree(p); }
};

// one request and its results
struct SolveJob {
  chfsi_request r{};
  int iterations = 0;
  double max_residual = 0.0;
  std::vector<double> evals, resnorms;
};

// bytes of one n x b block of the request's vectors (complex kinds: interleaved pairs)
size_t block_bytes(const chfsi_request& r) {
  const bool cplx = r.A.kind == CHFSI_OP_DENSE_HERMITIAN || r.A.kind == CHFSI_OP_STENCIL27_BLOCH;
  return size_t(r.A.n) * size_t(r.params.block) * sizeof(double) * (cplx ? 2 : 1);
}

// device bytes a running request holds (released when it finishes): its
// context's workspace and its working block.  A sequence's warm-start block
// is charged separately, from its allocation until it is replaced or the
// server is destroyed.
size_t footprint_of(const chfsi_request& r) {
  const chfsi_operator* B = r.B.kind == CHFSI_OP_IDENTITY ? nullptr : &r.B;
  const size_t ws = chfsi_workspace_bytes(&r.A, B, &r.params);
  if (ws == 0) return 0;
  return ws + block_bytes(r);
}

// a warm-start block fits a request of the same n and block (and kind)
uint64_t shape_key(const chfsi_request& r) {
  return (uint64_t(r.A.n) << 24) | uint64_t(r.params.block);
}

thread_local std::string g_srv_err;

struct ServerExec;
using Sched = chfsi::Scheduler<ServerExec>;

struct ServerExec {
  using Job = SolveJob;
  std::vector<hipStream_t> streams;
  std::unique_ptr<chfsi::RangePool<DeviceChunks>> dev_pool;
  std::unique_ptr<chfsi::RangePool<PinnedChunks>> host_pool;
  chfsi::Allocator al{};
  std::mutex seq_mu;                                  // guards seq_x
  std::unordered_map<int64_t, double*> seq_x;         // warm-start blocks

  size_t footprint(const Job& j) const { return footprint_of(j.r); }
  int64_t sequence(const Job& j) const { return j.r.seq_id; }
  size_t seq_block(const Job& j) const { return block_bytes(j.r); }
  uint64_t seq_shape(const Job& j) const { return shape_key(j.r); }

  double* seq_block_ptr(int64_t sid) {
    std::lock_guard<std::mutex> lk(seq_mu);
    auto f = seq_x.find(sid);
    return f == seq_x.end() ? nullptr : f->second;
  }

  void run(int slot, chfsi::Ticket<Job>& t, Sched& sch) {
    hipStream_t stream = streams[slot];
    const chfsi_request& r = t.job.r;
    const int64_t n = r.A.n, b = r.params.block;
    const size_t blk = block_bytes(r);
    const uint64_t key = shape_key(r);
    chfsi_params prm = r.params;
    double* X = nullptr;
    chfsi_ctx* ctx = nullptr;
    chfsi_status st = CHFSI_OK;
    // this sequence's block: only its own (one-at-a-time) jobs touch it
    const chfsi::SequenceState ss = r.seq_id >= 0 ? sch.sequence_state(r.seq_id)
                                                  : chfsi::SequenceState{};
    double* sx = r.seq_id >= 0 ? seq_block_ptr(r.seq_id) : nullptr;
    const bool fits = sx && ss.bytes == blk && ss.shape == key;
    do {
      X = static_cast<double*>(dev_pool->alloc(blk));
      if (!X) {
        st = CHFSI_ERR_NOMEM;
        break;
      }
      const chfsi_operator* B = r.B.kind == CHFSI_OP_IDENTITY ? nullptr : &r.B;
      bool warm = false;
      if (fits) {
        if (hipMemcpyAsync(X, sx, blk, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
          st = CHFSI_ERR_DEVICE;
          break;
        }
        warm = true;
      } else if (r.X0) {
        if (hipMemcpyAsync(X, r.X0, blk, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
          st = CHFSI_ERR_DEVICE;
          break;
        }
      }
      prm.init_random = (!warm && !r.X0) ? 1 : 0;
      st = chfsi::create_with_allocator(&ctx, &r.A, B, r.d_inv, &prm, stream, &al);
      if (st != CHFSI_OK) break;
      chfsi::ctx_set_cancel_flag(ctx, &t.cancel_flag);
      t.job.evals.assign(b, 0.0);
      t.job.resnorms.assign(b, 0.0);
      chfsi_report rep;
      st = chfsi_solve(ctx, X, n, t.job.evals.data(), t.job.resnorms.data(), &rep);
      t.job.iterations = rep.iterations;
      t.job.max_residual = rep.max_residual;
      if (st == CHFSI_OK || st == CHFSI_ERR_NOCONV) {
        if (r.seq_id >= 0) {
          if (!fits) {
            // (re)place the warm-start block; its charge in the budget moves with it
            sch.recharge(r.seq_id, blk, key, [&] {
              std::lock_guard<std::mutex> lk(seq_mu);
              double*& slot_x = seq_x[r.seq_id];
              if (slot_x) dev_pool->free(slot_x);
              slot_x = static_cast<double*>(dev_pool->alloc(blk));
              sx = slot_x;
              return slot_x != nullptr;
            });
          }
          if (sx) (void)hipMemcpyAsync(sx, X, blk, hipMemcpyDeviceToDevice, stream);
        }
        if (r.X_out) (void)hipMemcpyAsync(r.X_out, X, blk, hipMemcpyDeviceToDevice, stream);
        (void)hipStreamSynchronize(stream);
      }
    } while (false);
    if (st != CHFSI_OK) g_srv_err = chfsi_last_error();
    if (ctx) chfsi_destroy(ctx);
    if (X) {
      (void)hipStreamSynchronize(stream);   // the pool may hand X to another slot next
      dev_pool->free(X);
    }
    t.status = st;
  }
};

}  // namespace

struct chfsi_server {
  chfsi_server_config cfg{};
  int device = 0;
  ServerExec ex;
  std::unique_ptr<Sched> sched;
};

extern "C" {

chfsi_status chfsi_server_create(chfsi_server** out, const chfsi_server_config* cfg) {
  if (!out || !cfg || cfg->slots < 1 || cfg->slots > 64 || cfg->queue_capacity < 1)
    return CHFSI_ERR_ARG;
  chfsi_server* s = new chfsi_server();
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete s;
    return CHFSI_ERR_DEVICE;
  }
  const size_t budget = cfg->memory_budget ? cfg->memory_budget : size_t(0.9 * double(free_b));
  // device chunks of at least 1 GiB (or a fifth of the budget, if smaller),
  // pinned host chunks of 4 MiB
  ServerExec& ex = s->ex;
  ex.dev_pool.reset(new chfsi::RangePool<DeviceChunks>(
      DeviceChunks{}, std::min<size_t>(size_t(1) << 30, std::max<size_t>(budget / 5, 1 << 20))));
  ex.host_pool.reset(new chfsi::RangePool<PinnedChunks>(PinnedChunks{}, size_t(4) << 20));
  ex.al.self = &ex;
  ex.al.dev_alloc = [](void* self, size_t bytes) -> void* {
    return static_cast<ServerExec*>(self)->dev_pool->alloc(bytes);
  };
  ex.al.dev_free = [](void* self, void* p) { static_cast<ServerExec*>(self)->dev_pool->free(p); };
  ex.al.host_alloc = [](void* self, size_t bytes) -> void* {
    return static_cast<ServerExec*>(self)->host_pool->alloc(bytes);
  };
  ex.al.host_free = [](void* self, void* p) {
    static_cast<ServerExec*>(self)->host_pool->free(p);
  };
  for (int i = 0; i < cfg->slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : ex.streams) (void)hipStreamDestroy(x);
      delete s;
      return CHFSI_ERR_DEVICE;
    }
    ex.streams.push_back(st);
  }
  s->sched.reset(new Sched(&ex, budget, cfg->queue_capacity));
  s->sched->start(cfg->slots);
  *out = s;
  return CHFSI_OK;
}

chfsi_status chfsi_submit(chfsi_server* s, const chfsi_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return CHFSI_ERR_ARG;
  SolveJob j;
  j.r = *req;
  return s->sched->submit(j, ticket);
}

chfsi_status chfsi_wait(chfsi_server* s, uint64_t ticket, int32_t timeout_ms, chfsi_result* res) {
  if (!s || !res) return CHFSI_ERR_ARG;
  return s->sched->wait(ticket, timeout_ms, [&](chfsi::Ticket<SolveJob>& q) {
    std::memset(res, 0, sizeof(*res));
    res->status = q.status;
    res->iterations = q.job.iterations;
    res->max_residual = q.job.max_residual;
    res->submit_ms = q.submit_ms;
    res->start_ms = q.start_ms;
    res->finish_ms = q.finish_ms;
    res->n = q.job.r.A.n;
    res->block = q.job.r.params.block;
    if (!q.job.evals.empty()) {
      const size_t nb = q.job.evals.size() * sizeof(double);
      res->evals = static_cast<double*>(std::malloc(nb));
      res->resnorms = static_cast<double*>(std::malloc(nb));
      if (res->evals) std::memcpy(res->evals, q.job.evals.data(), nb);
      if (res->resnorms) std::memcpy(res->resnorms, q.job.resnorms.data(), nb);
    }
  });
}

chfsi_status chfsi_cancel(chfsi_server* s, uint64_t ticket) {
  if (!s) return CHFSI_ERR_ARG;
  return s->sched->cancel(ticket);
}

void chfsi_result_free(chfsi_result* res) {
  if (!res) return;
  std::free(res->evals);
  std::free(res->resnorms);
  res->evals = nullptr;
  res->resnorms = nullptr;
}

chfsi_status chfsi_server_stats(chfsi_server* s, chfsi_server_stats_t* out) {
  if (!s || !out) return CHFSI_ERR_ARG;
  out->budget = s->sched->budget();
  out->used = s->sched->used();
  out->device_pool_chunks = s->ex.dev_pool->grow_events();
  out->host_pool_chunks = s->ex.host_pool->grow_events();
  out->sequence_bytes = s->sched->sequence_bytes();
  return CHFSI_OK;
}

void chfsi_server_destroy(chfsi_server* s) {
  if (!s) return;
  s->sched->stop();   // pending requests end as CHFSI_ERR_CANCELLED; running ones finish
  s->sched.reset();
  {
    std::lock_guard<std::mutex> lk(s->ex.seq_mu);
    for (auto& kv : s->ex.seq_x)
      if (kv.second) s->ex.dev_pool->free(kv.second);
  }
  for (auto st : s->ex.streams) (void)hipStreamDestroy(st);
  delete s;   // the pools release their chunks
}

}  // extern "C"
