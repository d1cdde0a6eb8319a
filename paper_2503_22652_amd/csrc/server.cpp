// Serving scheduler of libchfsi: continuous batching of eigensolves on one GPU.
//
// The evolving-matrix setting of the paper (the Hamiltonian changes at every
// step of an outer nonlinear iteration and the lowest eigenpairs are recomputed
// from the previous subspace; introduction and Section 4.2) is served as a
// stream of requests grouped into sequences.
//
//  * `slots` worker threads, each owning one HIP stream (default priority), run
//    admitted solves concurrently; their kernels overlap on the device.
//  * Admission: the first pending request (submission order) whose sequence is
//    idle and whose device footprint (chfsi_workspace_bytes + its blocks) fits
//    in the remaining budget is started as soon as a slot frees up.
//  * Requests of one sequence run in submission order; the sequence's last Ritz
//    vectors stay on the device and warm-start the next request.
//  * A request runs the same kernels with the same launch shapes whether alone
//    or mixed (launch shapes depend on the problem shape only and each solve
//    has its own scratch), so its result is bitwise identical either way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/chfsi.h"
#include "internal.h"

namespace {

enum State { PENDING, RUNNING, DONE };

struct Req {
  uint64_t ticket = 0;
  chfsi_request r{};
  State state = PENDING;
  bool cancel_requested = false;
  std::atomic<int> cancel_flag{0};
  chfsi_status status = CHFSI_OK;
  int iterations = 0;
  double max_residual = 0.0;
  double submit_ms = 0, start_ms = 0, finish_ms = 0;
  size_t footprint = 0;
  std::vector<double> evals, resnorms;
};

struct Seq {
  double* X = nullptr;
  int64_t n = 0, b = 0;
  size_t bytes = 0;          // size of X (complex blocks are twice a real one)
  bool busy = false;
};

// First-fit pool over large chunks (device memory from hipMalloc, or pinned
// host memory from hipHostMalloc), so that a running server makes no
// allocation or free call per request: a chunk is added only when no free
// range fits (the first requests of each new size), and chunks are released
// only by the server's destruction.  hipFree, the call avoided, synchronises
// the whole device.  Ranges are 256-byte aligned; freed ranges merge with
// their free neighbours.
class Pool {
 public:
  Pool(bool host, size_t chunk_min) : host_(host), chunk_min_(chunk_min) {}
  ~Pool() {
    for (auto& c : chunks_) {
      if (host_)
        (void)hipHostFree(c.base);
      else
        (void)hipFree(c.base);
    }
  }
  void* alloc(size_t bytes) {
    bytes = std::max<size_t>(256, (bytes + 255) / 256 * 256);
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t ci = 0; ci < chunks_.size(); ++ci) {
      auto& fr = chunks_[ci].free;
      for (auto it = fr.begin(); it != fr.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, len = it->second;
        fr.erase(it);
        if (len > bytes) fr[off + bytes] = len - bytes;
        char* p = chunks_[ci].base + off;
        live_[p] = {ci, bytes};
        return p;
      }
    }
    const size_t sz = std::max(bytes, chunk_min_);
    void* base = nullptr;
    const hipError_t e = host_ ? hipHostMalloc(&base, sz) : hipMalloc(&base, sz);
    if (e != hipSuccess) return nullptr;
    ++grow_events_;
    Chunk c;
    c.base = static_cast<char*>(base);
    c.size = sz;
    if (sz > bytes) c.free[bytes] = sz - bytes;
    chunks_.push_back(std::move(c));
    live_[static_cast<char*>(base)] = {chunks_.size() - 1, bytes};
    return base;
  }
  void free(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(static_cast<char*>(p));
    if (it == live_.end()) return;
    const size_t ci = it->second.first, len = it->second.second;
    live_.erase(it);
    auto& fr = chunks_[ci].free;
    size_t off = size_t(static_cast<char*>(p) - chunks_[ci].base), n = len;
    auto nx = fr.lower_bound(off);
    if (nx != fr.end() && nx->first == off + n) {   // merge with the next free range
      n += nx->second;
      nx = fr.erase(nx);
    }
    if (nx != fr.begin()) {                          // and with the previous one
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        n += pv->second;
        fr.erase(pv);
      }
    }
    fr[off] = n;
  }
  int grow_events() const { return grow_events_; }

 private:
  struct Chunk {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;   // offset -> length
  };
  bool host_;
  size_t chunk_min_;
  std::mutex mu_;
  std::vector<Chunk> chunks_;
  std::map<char*, std::pair<size_t, size_t>> live_;   // range start -> (chunk, length)
  int grow_events_ = 0;
};

double clock_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct chfsi_server {
  chfsi_server_config cfg{};
  int device = 0;
  size_t budget = 0, used = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> reqs;
  std::unordered_map<int64_t, Seq> seqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  uint64_t next_ticket = 1;
  bool stop = false;
  // memory of every request (contexts, blocks) and of the sequences' warm starts
  std::unique_ptr<Pool> dev_pool, host_pool;
  chfsi::Allocator al{};
};

namespace {

thread_local std::string g_srv_err;

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

// the warm-start block a finished request of this sequence will need to
// (re)allocate: 0 when the sequence already holds one of the right size
size_t seq_growth(chfsi_server* s, const chfsi_request& r) {
  if (r.seq_id < 0) return 0;
  auto f = s->seqs.find(r.seq_id);
  const size_t blk = block_bytes(r);
  if (f == s->seqs.end() || !f->second.X) return blk;
  return f->second.bytes == blk && f->second.n == r.A.n && f->second.b == r.params.block
             ? 0
             : blk;
}

// pick the first admissible pending request; called with the lock held
Req* pick(chfsi_server* s) {
  for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
    Req* q = *it;
    const int64_t sid = q->r.seq_id;
    if (sid >= 0) {
      auto f = s->seqs.find(sid);
      if (f != s->seqs.end() && f->second.busy) continue;   // predecessor still running
      // an earlier pending request of the same sequence goes first
      bool earlier = false;
      for (auto jt = s->pending.begin(); jt != it; ++jt)
        if ((*jt)->r.seq_id == sid) earlier = true;
      if (earlier) continue;
    }
    const size_t need = footprint_of(q->r);
    // room for the request and for a (re)allocated warm-start block of its sequence
    if (s->used + need + seq_growth(s, q->r) > s->budget) continue;
    q->footprint = need;
    s->used += need;
    s->pending.erase(it);
    if (sid >= 0) s->seqs[sid].busy = true;
    return q;
  }
  return nullptr;
}

void run_one(chfsi_server* s, Req* q, hipStream_t stream) {
  const chfsi_request& r = q->r;
  const int64_t n = r.A.n, b = r.params.block;
  const size_t blk = block_bytes(r);
  chfsi_params prm = r.params;
  double* X = nullptr;
  chfsi_ctx* ctx = nullptr;
  chfsi_status st = CHFSI_OK;
  Seq* seq = nullptr;
  if (r.seq_id >= 0) {
    std::lock_guard<std::mutex> lk(s->mu);
    seq = &s->seqs[r.seq_id];
  }
  do {
    X = static_cast<double*>(s->dev_pool->alloc(blk));
    if (!X) {
      st = CHFSI_ERR_NOMEM;
      break;
    }
    const chfsi_operator* B = r.B.kind == CHFSI_OP_IDENTITY ? nullptr : &r.B;
    bool warm = false;
    if (seq && seq->X && seq->n == n && seq->b == b && seq->bytes == blk) {
      if (hipMemcpyAsync(X, seq->X, blk, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
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
    st = chfsi::create_with_allocator(&ctx, &r.A, B, r.d_inv, &prm, stream, &s->al);
    if (st != CHFSI_OK) break;
    chfsi::ctx_set_cancel_flag(ctx, &q->cancel_flag);
    q->evals.assign(b, 0.0);
    q->resnorms.assign(b, 0.0);
    chfsi_report rep;
    st = chfsi_solve(ctx, X, n, q->evals.data(), q->resnorms.data(), &rep);
    q->iterations = rep.iterations;
    q->max_residual = rep.max_residual;
    if (st == CHFSI_OK || st == CHFSI_ERR_NOCONV) {
      if (seq) {
        if (!seq->X || seq->n != n || seq->b != b || seq->bytes != blk) {
          // (re)place the warm-start block and move its charge in the budget
          std::lock_guard<std::mutex> lk(s->mu);
          if (seq->X) {
            s->dev_pool->free(seq->X);
            s->used -= seq->bytes;
          }
          seq->X = static_cast<double*>(s->dev_pool->alloc(blk));
          seq->n = n;
          seq->b = b;
          seq->bytes = seq->X ? blk : 0;
          s->used += seq->bytes;
        }
        if (seq->X) hipMemcpyAsync(seq->X, X, blk, hipMemcpyDeviceToDevice, stream);
      }
      if (r.X_out) hipMemcpyAsync(r.X_out, X, blk, hipMemcpyDeviceToDevice, stream);
      hipStreamSynchronize(stream);
    }
  } while (false);
  if (st != CHFSI_OK) g_srv_err = chfsi_last_error();
  if (ctx) chfsi_destroy(ctx);
  if (X) {
    hipStreamSynchronize(stream);   // the pool may hand X to another slot next
    s->dev_pool->free(X);
  }
  q->status = st;
}

void worker_main(chfsi_server* s, int slot) {
  hipSetDevice(s->device);
  hipStream_t stream = s->streams[slot];
  for (;;) {
    Req* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || (q = pick(s)) != nullptr; });
      if (!q) return;   // stopping
      q->state = RUNNING;
      q->start_ms = clock_ms(s->t0);
    }
    run_one(s, q, stream);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      q->finish_ms = clock_ms(s->t0);
      q->state = DONE;
      s->used -= q->footprint;
      if (q->r.seq_id >= 0) s->seqs[q->r.seq_id].busy = false;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

chfsi_status chfsi_server_create(chfsi_server** out, const chfsi_server_config* cfg) {
  if (!out || !cfg || cfg->slots < 1 || cfg->slots > 64 || cfg->queue_capacity < 1)
    return CHFSI_ERR_ARG;
  chfsi_server* s = new chfsi_server();
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  hipGetDevice(&s->device);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete s;
    return CHFSI_ERR_DEVICE;
  }
  s->budget = cfg->memory_budget ? cfg->memory_budget : size_t(0.9 * double(free_b));
  // device chunks of at least 1 GiB (or a fifth of the budget, if smaller),
  // pinned host chunks of 4 MiB
  s->dev_pool.reset(new Pool(false, std::min<size_t>(size_t(1) << 30,
                                                     std::max<size_t>(s->budget / 5, 1 << 20))));
  s->host_pool.reset(new Pool(true, size_t(4) << 20));
  s->al.self = s;
  s->al.dev_alloc = [](void* self, size_t bytes) -> void* {
    return static_cast<chfsi_server*>(self)->dev_pool->alloc(bytes);
  };
  s->al.dev_free = [](void* self, void* p) { static_cast<chfsi_server*>(self)->dev_pool->free(p); };
  s->al.host_alloc = [](void* self, size_t bytes) -> void* {
    return static_cast<chfsi_server*>(self)->host_pool->alloc(bytes);
  };
  s->al.host_free = [](void* self, void* p) { static_cast<chfsi_server*>(self)->host_pool->free(p); };
  for (int i = 0; i < cfg->slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) hipStreamDestroy(x);
      delete s;
      return CHFSI_ERR_DEVICE;
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < cfg->slots; ++i) s->workers.emplace_back(worker_main, s, i);
  *out = s;
  return CHFSI_OK;
}

chfsi_status chfsi_submit(chfsi_server* s, const chfsi_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return CHFSI_ERR_ARG;
  const size_t need = footprint_of(*req) + (req->seq_id >= 0 ? block_bytes(*req) : 0);
  if (need == 0) return CHFSI_ERR_ARG;
  Req* q = new Req();
  q->r = *req;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (need > s->budget) {
      delete q;
      return CHFSI_ERR_NOMEM;
    }
    if (s->stop || int(s->pending.size()) >= s->cfg.queue_capacity) {
      delete q;
      return CHFSI_ERR_BUSY;
    }
    q->ticket = s->next_ticket++;
    q->submit_ms = clock_ms(s->t0);
    s->reqs[q->ticket] = q;
    s->pending.push_back(q);
    *ticket = q->ticket;
  }
  s->cv_work.notify_one();
  return CHFSI_OK;
}

chfsi_status chfsi_wait(chfsi_server* s, uint64_t ticket, int32_t timeout_ms, chfsi_result* res) {
  if (!s || !res) return CHFSI_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CHFSI_ERR_ARG;
  Req* q = it->second;
  auto done = [&] { return q->state == DONE; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    return CHFSI_ERR_TIMEOUT;
  }
  std::memset(res, 0, sizeof(*res));
  res->status = q->status;
  res->iterations = q->iterations;
  res->max_residual = q->max_residual;
  res->submit_ms = q->submit_ms;
  res->start_ms = q->start_ms;
  res->finish_ms = q->finish_ms;
  res->n = q->r.A.n;
  res->block = q->r.params.block;
  if (!q->evals.empty()) {
    res->evals = static_cast<double*>(std::malloc(q->evals.size() * sizeof(double)));
    res->resnorms = static_cast<double*>(std::malloc(q->resnorms.size() * sizeof(double)));
    if (res->evals) std::memcpy(res->evals, q->evals.data(), q->evals.size() * sizeof(double));
    if (res->resnorms)
      std::memcpy(res->resnorms, q->resnorms.data(), q->resnorms.size() * sizeof(double));
  }
  s->reqs.erase(it);
  const chfsi_status st = q->status;
  delete q;
  return st;
}

chfsi_status chfsi_cancel(chfsi_server* s, uint64_t ticket) {
  if (!s) return CHFSI_ERR_ARG;
  bool notify = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return CHFSI_ERR_ARG;
    Req* q = it->second;
    if (q->state == PENDING) {
      for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
        if (*p == q) {
          s->pending.erase(p);
          break;
        }
      q->state = DONE;
      q->status = CHFSI_ERR_CANCELLED;
      q->finish_ms = clock_ms(s->t0);
      notify = true;
    } else if (q->state == RUNNING) {
      q->cancel_flag.store(1);
    }
  }
  if (notify) {
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  return CHFSI_OK;
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
  std::lock_guard<std::mutex> lk(s->mu);
  out->budget = s->budget;
  out->used = s->used;
  out->device_pool_chunks = s->dev_pool->grow_events();
  out->host_pool_chunks = s->host_pool->grow_events();
  size_t seq_bytes = 0;
  for (auto& kv : s->seqs) seq_bytes += kv.second.bytes;
  out->sequence_bytes = seq_bytes;
  return CHFSI_OK;
}

void chfsi_server_destroy(chfsi_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Req* q : s->pending) {
      q->state = DONE;
      q->status = CHFSI_ERR_CANCELLED;
    }
    s->pending.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->seqs)
    if (kv.second.X) s->dev_pool->free(kv.second.X);
  for (auto& kv : s->reqs) delete kv.second;
  for (auto st : s->streams) hipStreamDestroy(st);
  delete s;   // the pools release their chunks
}

}  // extern "C"
