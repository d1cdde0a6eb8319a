// First-fit pool over large chunks, so that a running server makes no
// allocation or free call per request: a chunk is added only when no free
// range fits (the first requests of each new size), and chunks are released
// only when the pool is destroyed.  Ranges are 256-byte aligned; freed ranges
// merge with their free neighbours.  Thread-safe.
//
// Backend supplies the chunks:
//   void* grab(size_t bytes);      nullptr on failure
//   void release(void* p);
// (the server: hipMalloc / hipHostMalloc and their frees -- hipFree, the call
// the pool avoids per request, synchronises the whole device; the CPU test of
// the range logic: malloc).
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

namespace chfsi {

template <typename Backend>
class RangePool {
 public:
  RangePool(Backend be, size_t chunk_min) : be_(be), chunk_min_(chunk_min) {}
  RangePool(const RangePool&) = delete;
  RangePool& operator=(const RangePool&) = delete;
  ~RangePool() {
    for (auto& c : chunks_) be_.release(c.base);
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
    void* base = be_.grab(sz);
    if (!base) return nullptr;
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
  int grow_events() {
    std::lock_guard<std::mutex> lk(mu_);
    return grow_events_;
  }
  // bytes in live ranges, and whether every chunk is one free range again
  size_t live_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    size_t s = 0;
    for (auto& kv : live_) s += kv.second.second;
    return s;
  }
  bool all_free() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& c : chunks_)
      if (c.free.size() != 1 || c.free.begin()->first != 0 || c.free.begin()->second != c.size)
        return false;
    return live_.empty();
  }

 private:
  struct Chunk {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;   // offset -> length
  };
  Backend be_;
  size_t chunk_min_;
  std::mutex mu_;
  std::vector<Chunk> chunks_;
  std::map<char*, std::pair<size_t, size_t>> live_;   // range start -> (chunk, length)
  int grow_events_ = 0;
};

}  // namespace chfsi
