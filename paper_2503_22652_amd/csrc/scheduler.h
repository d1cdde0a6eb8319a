// Continuous-batching scheduler of the serving loop, kept free of device
// calls so that its logic -- admission by a byte budget, per-sequence order,
// the charges of the sequences' warm-start blocks, cancellation, waiting --
// runs unchanged in the server (executor: one eigensolve on a HIP stream per
// slot) and in a CPU test with a fake executor under the sanitizers.
//
// The executor supplies
//   using Job = ...;                              a request and its results
//   size_t footprint(const Job&) const;           bytes held while it runs (0: invalid)
//   int64_t sequence(const Job&) const;           sequence id (< 0: none)
//   size_t seq_block(const Job&) const;           bytes of its sequence's warm-start block
//   uint64_t seq_shape(const Job&) const;         identifies a compatible warm-start block
//   void run(int slot, Ticket<Job>& t, Scheduler& s);   runs the job, no lock held
// run() may (re)place its sequence's block with s.recharge(seq, bytes, shape, f),
// which moves the charge and calls f under the scheduler's lock.
//
// Admission: a worker that is free takes the first pending job (submission
// order) whose sequence is idle, that has no earlier pending job of the same
// sequence, and whose footprint -- plus a (re)allocated warm-start block for
// its sequence -- fits in what the budget has left.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/chfsi.h"

namespace chfsi {

enum class TicketState { PENDING, RUNNING, DONE };

template <typename Job>
struct Ticket {
  uint64_t id = 0;
  Job job{};
  TicketState state = TicketState::PENDING;
  std::atomic<int> cancel_flag{0};
  chfsi_status status = CHFSI_OK;
  double submit_ms = 0, start_ms = 0, finish_ms = 0;
  size_t footprint = 0;
};

struct SequenceState {
  size_t bytes = 0;      // charged warm-start block (0: none)
  uint64_t shape = 0;    // the block's shape key
  bool busy = false;     // a job of the sequence is running
};

template <typename Exec>
class Scheduler {
 public:
  using Job = typename Exec::Job;
  using T = Ticket<Job>;

  Scheduler(Exec* ex, size_t budget, int capacity)
      : ex_(ex), budget_(budget), capacity_(capacity), t0_(std::chrono::steady_clock::now()) {}
  Scheduler(const Scheduler&) = delete;
  Scheduler& operator=(const Scheduler&) = delete;
  ~Scheduler() {
    stop();
    for (auto& kv : tickets_) delete kv.second;
  }

  void start(int slots) {
    for (int i = 0; i < slots; ++i) workers_.emplace_back([this, i] { worker(i); });
  }

  // stop admitting, cancel what is pending, let running jobs finish, join
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_) return;
      stopped_ = true;
      for (T* q : pending_) {
        q->state = TicketState::DONE;
        q->status = CHFSI_ERR_CANCELLED;
      }
      pending_.clear();
    }
    cv_work_.notify_all();
    cv_done_.notify_all();
    for (auto& t : workers_) t.join();
    workers_.clear();
  }

  chfsi_status submit(const Job& job, uint64_t* id) {
    const int64_t sid = ex_->sequence(job);
    const size_t fp = ex_->footprint(job);
    if (fp == 0) return CHFSI_ERR_ARG;
    const size_t need = fp + (sid >= 0 ? ex_->seq_block(job) : 0);
    T* q = new T();
    q->job = job;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (need > budget_) {
        delete q;
        return CHFSI_ERR_NOMEM;
      }
      if (stopped_ || int(pending_.size()) >= capacity_) {
        delete q;
        return CHFSI_ERR_BUSY;
      }
      q->id = next_id_++;
      q->submit_ms = now_ms();
      tickets_[q->id] = q;
      pending_.push_back(q);
      *id = q->id;
    }
    cv_work_.notify_one();
    return CHFSI_OK;
  }

  // wait for a ticket (timeout_ms < 0: no limit), hand it to take() under the
  // lock, then forget it; returns its status (CHFSI_ERR_TIMEOUT: still running)
  template <typename F>
  chfsi_status wait(uint64_t id, int timeout_ms, F&& take) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return CHFSI_ERR_ARG;
    T* q = it->second;
    auto done = [&] { return q->state == TicketState::DONE; };
    if (timeout_ms < 0) {
      cv_done_.wait(lk, done);
    } else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
      return CHFSI_ERR_TIMEOUT;
    }
    take(*q);
    tickets_.erase(it);
    const chfsi_status st = q->status;
    delete q;
    return st;
  }

  // a pending job is dropped (CHFSI_ERR_CANCELLED); a running one is asked to stop
  chfsi_status cancel(uint64_t id) {
    bool notify = false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = tickets_.find(id);
      if (it == tickets_.end()) return CHFSI_ERR_ARG;
      T* q = it->second;
      if (q->state == TicketState::PENDING) {
        pending_.erase(std::find(pending_.begin(), pending_.end(), q));
        q->state = TicketState::DONE;
        q->status = CHFSI_ERR_CANCELLED;
        q->finish_ms = now_ms();
        notify = true;
      } else if (q->state == TicketState::RUNNING) {
        q->cancel_flag.store(1);
      }
    }
    if (notify) {
      cv_done_.notify_all();
      cv_work_.notify_all();
    }
    return CHFSI_OK;
  }

  // from Exec::run: the sequence's block changes to `bytes` (shape key `shape`);
  // f() swaps the block itself, under the lock; the charge moves with it
  template <typename F>
  void recharge(int64_t sid, size_t bytes, uint64_t shape, F&& f) {
    std::lock_guard<std::mutex> lk(mu_);
    SequenceState& sq = seqs_[sid];
    used_ -= sq.bytes;
    const bool ok = f();
    sq.bytes = ok ? bytes : 0;
    sq.shape = ok ? shape : 0;
    used_ += sq.bytes;
  }

  // the sequence's current block (bytes, shape), read by its running job
  SequenceState sequence_state(int64_t sid) {
    std::lock_guard<std::mutex> lk(mu_);
    auto f = seqs_.find(sid);
    return f == seqs_.end() ? SequenceState{} : f->second;
  }

  size_t budget() const { return budget_; }
  size_t used() {
    std::lock_guard<std::mutex> lk(mu_);
    return used_;
  }
  size_t sequence_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    size_t s = 0;
    for (auto& kv : seqs_) s += kv.second.bytes;
    return s;
  }
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_)
        .count();
  }

 private:
  // bytes a (re)allocated warm-start block of q's sequence would add
  size_t seq_growth(const T* q) const {
    const int64_t sid = ex_->sequence(q->job);
    if (sid < 0) return 0;
    const size_t blk = ex_->seq_block(q->job);
    auto f = seqs_.find(sid);
    if (f == seqs_.end() || f->second.bytes == 0) return blk;
    return f->second.bytes == blk && f->second.shape == ex_->seq_shape(q->job) ? 0 : blk;
  }

  // the first admissible pending job; called with the lock held
  T* pick() {
    for (auto it = pending_.begin(); it != pending_.end(); ++it) {
      T* q = *it;
      const int64_t sid = ex_->sequence(q->job);
      if (sid >= 0) {
        auto f = seqs_.find(sid);
        if (f != seqs_.end() && f->second.busy) continue;   // predecessor still running
        bool earlier = false;                                // an earlier job of it goes first
        for (auto jt = pending_.begin(); jt != it; ++jt)
          if (ex_->sequence((*jt)->job) == sid) earlier = true;
        if (earlier) continue;
      }
      const size_t need = ex_->footprint(q->job);
      if (used_ + need + seq_growth(q) > budget_) continue;
      q->footprint = need;
      used_ += need;
      pending_.erase(it);
      if (sid >= 0) seqs_[sid].busy = true;
      return q;
    }
    return nullptr;
  }

  void worker(int slot) {
    for (;;) {
      T* q = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_work_.wait(lk, [&] { return stopped_ || (q = pick()) != nullptr; });
        if (!q) return;   // stopping
        q->state = TicketState::RUNNING;
        q->start_ms = now_ms();
      }
      ex_->run(slot, *q, *this);
      {
        std::lock_guard<std::mutex> lk(mu_);
        q->finish_ms = now_ms();
        q->state = TicketState::DONE;
        used_ -= q->footprint;
        const int64_t sid = ex_->sequence(q->job);
        if (sid >= 0) seqs_[sid].busy = false;
      }
      cv_done_.notify_all();
      cv_work_.notify_all();
    }
  }

  Exec* ex_;
  const size_t budget_;
  const int capacity_;
  const std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<T*> pending_;
  std::unordered_map<uint64_t, T*> tickets_;
  std::unordered_map<int64_t, SequenceState> seqs_;
  std::vector<std::thread> workers_;
  uint64_t next_id_ = 1;
  size_t used_ = 0;
  bool stopped_ = false;
};

}  // namespace chfsi
