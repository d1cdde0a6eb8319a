// CPU test of the serving scheduler (scheduler.h) and the range pool (pool.h)
// with a fake executor: no device, built with the sanitizers (ASan + UBSan, or
// TSan) by tests/test_scheduler_cpu.py.  Exits non-zero on the first broken
// invariant:
//  * the bytes charged never exceed the budget;
//  * jobs of one sequence never overlap and start in submission order;
//  * every ticket ends exactly once: run, or cancelled while pending;
//  * oversized jobs are refused (CHFSI_ERR_NOMEM), a full queue is busy;
//  * a running job sees its cancel flag; stop() cancels what is pending;
//  * warm-start charges follow the sequence's block size;
//  * the pool hands out disjoint ranges and merges them back.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "pool.h"
#include "scheduler.h"

#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "CHECK failed: %s (line %d)\n", #cond, __LINE__); \
      std::exit(1);                                                          \
    }                                                                        \
  } while (0)

struct MallocChunks {
  void* grab(size_t bytes) { return std::malloc(bytes); }
  void release(void* p) { std::free(p); }
};

struct FakeJob {
  int64_t seq = -1;
  size_t fp = 0, blk = 0;
  uint64_t shape = 0;
  int work_us = 0;
  int index = 0;         // submission index within its sequence
  bool ran = false;
};

struct FakeExec;
using Sched = chfsi::Scheduler<FakeExec>;

struct FakeExec {
  using Job = FakeJob;
  chfsi::RangePool<MallocChunks> pool{MallocChunks{}, 1 << 16};
  std::mutex mu;
  std::map<int64_t, int> next_index;        // next expected index per sequence
  std::map<int64_t, int> running;           // running jobs per sequence
  std::map<int64_t, void*> blocks;          // the sequences' warm-start blocks
  std::atomic<int> runs{0}, cancelled_runs{0};

  size_t footprint(const Job& j) const { return j.fp; }
  int64_t sequence(const Job& j) const { return j.seq; }
  size_t seq_block(const Job& j) const { return j.blk; }
  uint64_t seq_shape(const Job& j) const { return j.shape; }

  void run(int, chfsi::Ticket<Job>& t, Sched& s) {
    CHECK(s.used() <= s.budget());
    if (t.job.seq >= 0) {
      std::lock_guard<std::mutex> lk(mu);
      CHECK(running[t.job.seq] == 0);
      // submission order (jobs cancelled while pending leave gaps)
      CHECK(t.job.index >= next_index[t.job.seq]);
      ++running[t.job.seq];
      next_index[t.job.seq] = t.job.index + 1;
    }
    // the job's own scratch from the pool, written end to end
    char* scratch = static_cast<char*>(pool.alloc(t.job.fp));
    CHECK(scratch != nullptr);
    std::memset(scratch, int(t.id & 0x7f), t.job.fp);
    const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(t.job.work_us);
    bool cancelled = false;
    while (std::chrono::steady_clock::now() < until) {
      if (t.cancel_flag.load()) {
        cancelled = true;
        break;
      }
      std::this_thread::yield();
    }
    for (size_t i = 0; i < t.job.fp; i += 4093) CHECK(scratch[i] == char(t.id & 0x7f));
    pool.free(scratch);
    if (t.job.seq >= 0 && !cancelled) {
      const chfsi::SequenceState ss = s.sequence_state(t.job.seq);
      if (!(ss.bytes == t.job.blk && ss.shape == t.job.shape)) {
        s.recharge(t.job.seq, t.job.blk, t.job.shape, [&] {
          std::lock_guard<std::mutex> lk(mu);
          void*& b = blocks[t.job.seq];
          pool.free(b);
          b = pool.alloc(t.job.blk);
          return b != nullptr;
        });
      }
      CHECK(s.used() <= s.budget());
    }
    if (t.job.seq >= 0) {
      std::lock_guard<std::mutex> lk(mu);
      --running[t.job.seq];
    }
    t.job.ran = true;
    ++runs;
    if (cancelled) ++cancelled_runs;
    t.status = cancelled ? CHFSI_ERR_CANCELLED : CHFSI_OK;
  }
};

static void pool_stress() {
  chfsi::RangePool<MallocChunks> pool(MallocChunks{}, 1 << 20);
  std::mt19937 rng(7);
  std::vector<std::pair<char*, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t sz = 1 + rng() % 50000;
      char* p = static_cast<char*>(pool.alloc(sz));
      CHECK(p != nullptr);
      CHECK(reinterpret_cast<uintptr_t>(p) % 256 == 0);
      std::memset(p, int(it & 0xff), sz);
      for (auto& q : live)   // disjoint from every live range
        CHECK(p + sz <= q.first || q.first + q.second <= p);
      live.push_back({p, sz});
    } else {
      const size_t k = rng() % live.size();
      pool.free(live[k].first);
      live.erase(live.begin() + long(k));
    }
  }
  for (auto& q : live) pool.free(q.first);
  CHECK(pool.live_bytes() == 0);
  CHECK(pool.all_free());
}

static void stream_of_jobs() {
  FakeExec ex;
  const size_t budget = size_t(8) << 20;
  Sched s(&ex, budget, 1 << 20);
  s.start(4);
  std::mt19937 rng(11);
  const int nseq = 12, njobs = 600;
  std::vector<int> per_seq(nseq, 0);
  std::vector<uint64_t> ids;
  std::vector<int> cancelled_pending;
  for (int i = 0; i < njobs; ++i) {
    FakeJob j;
    j.seq = (i % 5 == 4) ? -1 : int64_t(rng() % nseq);
    j.fp = (size_t(1) << 16) + rng() % (size_t(1) << 20);
    // a sequence's block size changes now and then (a new n or block)
    j.blk = j.seq >= 0 ? (size_t(1) << 14) * (1 + (per_seq[j.seq] / 7) % 3) : 0;
    j.shape = j.blk;
    j.work_us = int(rng() % 400);
    j.index = j.seq >= 0 ? per_seq[j.seq]++ : 0;
    uint64_t id = 0;
    CHECK(s.submit(j, &id) == CHFSI_OK);
    ids.push_back(id);
  }
  // cancel a few: pending ones end cancelled without running, running ones see the flag
  int ok = 0, cancelled = 0, ran_cancelled = 0;
  for (size_t k = 0; k < ids.size(); k += 37) CHECK(s.cancel(ids[k]) == CHFSI_OK);
  for (uint64_t id : ids) {
    bool ran = false;
    const chfsi_status st = s.wait(id, -1, [&](chfsi::Ticket<FakeJob>& t) { ran = t.job.ran; });
    if (st == CHFSI_OK) {
      CHECK(ran);
      ++ok;
    } else {
      CHECK(st == CHFSI_ERR_CANCELLED);
      ++cancelled;
      if (ran) ++ran_cancelled;
    }
    CHECK(s.wait(id, 0, [](chfsi::Ticket<FakeJob>&) {}) == CHFSI_ERR_ARG);   // forgotten
  }
  CHECK(ok + cancelled == njobs);
  CHECK(ex.runs.load() == ok + ran_cancelled);
  CHECK(ex.cancelled_runs.load() == ran_cancelled);
  // only the sequences' warm-start blocks stay charged
  CHECK(s.used() == s.sequence_bytes());
  s.stop();
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    for (auto& kv : ex.blocks) ex.pool.free(kv.second);
  }
  CHECK(ex.pool.all_free());
  std::printf("stream: %d done, %d cancelled (%d while running)\n", ok, cancelled, ran_cancelled);
}

static void refusals_and_stop() {
  FakeExec ex;
  Sched s(&ex, size_t(1) << 20, 4);
  FakeJob big;
  big.fp = size_t(2) << 20;
  uint64_t id = 0;
  CHECK(s.submit(big, &id) == CHFSI_ERR_NOMEM);
  FakeJob zero;
  CHECK(s.submit(zero, &id) == CHFSI_ERR_ARG);
  // no workers yet: the queue fills up, then stop() cancels everything pending
  std::vector<uint64_t> ids;
  for (int i = 0; i < 4; ++i) {
    FakeJob j;
    j.fp = 4096;
    j.work_us = 10;
    CHECK(s.submit(j, &id) == CHFSI_OK);
    ids.push_back(id);
  }
  FakeJob j;
  j.fp = 4096;
  CHECK(s.submit(j, &id) == CHFSI_ERR_BUSY);
  CHECK(s.wait(ids[0], 5, [](chfsi::Ticket<FakeJob>&) {}) == CHFSI_ERR_TIMEOUT);
  s.stop();
  for (uint64_t t : ids)
    CHECK(s.wait(t, -1, [](chfsi::Ticket<FakeJob>& q) { CHECK(!q.job.ran); }) ==
          CHFSI_ERR_CANCELLED);
  CHECK(ex.runs.load() == 0);
  CHECK(s.submit(j, &id) == CHFSI_ERR_BUSY);   // stopped
}

static void running_cancel() {
  FakeExec ex;
  Sched s(&ex, size_t(1) << 24, 16);
  s.start(1);
  FakeJob j;
  j.fp = 4096;
  j.work_us = 2000000;   // long; ends early on the cancel flag
  uint64_t id = 0;
  CHECK(s.submit(j, &id) == CHFSI_OK);
  while (ex.runs.load() == 0 && s.used() == 0) std::this_thread::yield();
  CHECK(s.cancel(id) == CHFSI_OK);
  bool ran = false;
  CHECK(s.wait(id, -1, [&](chfsi::Ticket<FakeJob>& q) { ran = q.job.ran; }) ==
        CHFSI_ERR_CANCELLED);
  CHECK(ran);
  s.stop();
}

int main() {
  pool_stress();
  refusals_and_stop();
  running_cancel();
  stream_of_jobs();
  std::printf("ok\n");
  return 0;
}
