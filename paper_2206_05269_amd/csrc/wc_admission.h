// Memory policy of the request server, host-only (no HIP), so that it can be driven by a fake
// executor on the CPU.
//
// The server owns one device pool of a fixed budget. Two kinds of blocks live in it:
//   count memory    a request's text, offsets and workspace while it is being counted; always
//                   returned when the count ends;
//   resident memory the compacted result table, kept until the client releases the request.
// Count blocks are taken first-fit from the low end of the pool and resident blocks from the
// high end (the highest free block that fits, its top part), so resident tables do not land in
// the holes that finished counts leave among running ones and split the space large requests
// need.
//
// Admission rules (decisions, not waits; the server waits on a condition variable when told to):
//   count:    granted when a free block fits; otherwise wait while some request holds count
//             memory (it will return it); when none does, only resident tables hold memory,
//             which only the client can release, so the request fails (WC_ENOMEM) rather than
//             wait for a release that may never come.
//   resident: asked for by a request that itself holds count memory; granted when a free
//             block fits; otherwise wait while another holder that is not itself waiting for
//             resident memory exists (it will return its count memory); otherwise fail. So two
//             holders never wait on each other, and a request fails only when no memory can
//             come back without the client.
// Deferred release: a resident table that a merge is reading is freed when the last reader
// finishes, not when the client releases it.
#ifndef WC_ADMISSION_H
#define WC_ADMISSION_H

#include <stdint.h>

#include <iterator>
#include <map>

namespace wc {

constexpr uint64_t kPoolAlign = 256;

// Free-list allocator over [0, size) that hands out blocks from either end.
class TwoEndedPool {
 public:
  void init(uint64_t size) {
    free_.clear();
    used_.clear();
    size_ = size;
    if (size) free_[0] = size;
  }
  static uint64_t round(uint64_t bytes) {
    return ((bytes ? bytes : 1) + kPoolAlign - 1) & ~(kPoolAlign - 1);
  }
  // lowest free block that fits; its low part
  bool alloc_low(uint64_t bytes, uint64_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const uint64_t o = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[o + bytes] = len - bytes;
        used_[o] = bytes;
        *off = o;
        return true;
      }
    }
    return false;
  }
  // highest free block that fits; its high part
  bool alloc_high(uint64_t bytes, uint64_t* off) {
    bytes = round(bytes);
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second >= bytes) {
        const uint64_t o = it->first, len = it->second;
        const uint64_t at = o + len - bytes;
        if (len > bytes) it->second = len - bytes;
        else free_.erase(std::next(it).base());
        used_[at] = bytes;
        *off = at;
        return true;
      }
    }
    return false;
  }
  bool release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    uint64_t len = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return true;
      }
    }
    free_[off] = len;
    return true;
  }
  uint64_t free_bytes() const {
    uint64_t s = 0;
    for (auto& f : free_) s += f.second;
    return s;
  }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  uint64_t size() const { return size_; }
  size_t n_used() const { return used_.size(); }

 private:
  uint64_t size_ = 0;
  std::map<uint64_t, uint64_t> free_, used_;
};

enum class Admit { kGranted, kWait, kFail };

// The admission state of one server; every call is made under the server's lock.
struct Admission {
  TwoEndedPool pool;
  uint32_t holders = 0;           // requests holding count memory
  uint32_t resident_waiters = 0;  // holders waiting for resident memory

  void init(uint64_t budget) {
    pool.init(budget);
    holders = 0;
    resident_waiters = 0;
  }
  // Count memory for a request that holds none yet; on kGranted the request is a holder.
  Admit try_count(uint64_t bytes, uint64_t* off) {
    if (pool.alloc_low(bytes, off)) {
      ++holders;
      return Admit::kGranted;
    }
    return holders > 0 ? Admit::kWait : Admit::kFail;
  }
  void free_count(uint64_t off) {
    pool.release(off);
    --holders;
  }
  // Resident memory for a request that holds count memory. A caller told to wait counts
  // itself in resident_waiters while it waits.
  Admit try_resident(uint64_t bytes, uint64_t* off) {
    if (pool.alloc_high(bytes, off)) return Admit::kGranted;
    return holders > resident_waiters + 1 ? Admit::kWait : Admit::kFail;
  }
  void free_resident(uint64_t off) { pool.release(off); }
};

// Life of one resident table: readers are merges that will read it; released means the client
// has released it. The memory is freed once both hold: returns true when the caller frees it.
struct ResidentLife {
  uint32_t readers = 0;
  bool released = false;
  void pin() { ++readers; }
  bool unpin() { return --readers == 0 && released; }
  bool release() {
    released = true;
    return readers == 0;
  }
};

}  // namespace wc

#endif  // WC_ADMISSION_H
