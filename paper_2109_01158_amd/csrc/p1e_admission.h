// p1e_admission.h -- the serving loop's admission bookkeeping, free of device code so that it
// runs on the CPU as well: a first-fit allocator over the request area of the caller's pool
// (free blocks kept by offset, coalesced on release) and the slot table. Requests are
// admitted in arrival order: the first one that finds no free slot or no free block large
// enough stops admission until a request retires (no overtaking); one larger than the whole
// request area can never be admitted. Not part of the public ABI.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace p1e {

class FirstFit {
 public:
  explicit FirstFit(uint64_t bytes = 0) { reset(bytes); }
  void reset(uint64_t bytes) {
    free_.clear();
    total_ = bytes;
    if (bytes) free_[0] = bytes;
  }
  // the lowest-offset free block of at least `bytes`, split; false if there is none
  bool alloc(uint64_t bytes, uint64_t &off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const uint64_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  // return a block; merged with free neighbours on either side
  void release(uint64_t off, uint64_t bytes) {
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
  uint64_t total() const { return total_; }
  const std::map<uint64_t, uint64_t> &free_blocks() const { return free_; }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  uint64_t total_ = 0;
};

enum class Admit { kAdmitted, kWait, kNever };

struct Admission {
  FirstFit pool;
  std::vector<int64_t> owner;  // request id in each slot, -1: free

  void reset(int slots, uint64_t bytes) {
    pool.reset(bytes);
    owner.assign(slots, -1);
  }
  // the lowest free slot and a first-fit block of `bytes` for request id
  Admit try_admit(int64_t id, uint64_t bytes, int &slot, uint64_t &off) {
    if (bytes > pool.total()) return Admit::kNever;
    slot = -1;
    for (int i = 0; i < (int)owner.size(); ++i)
      if (owner[i] < 0) {
        slot = i;
        break;
      }
    if (slot < 0 || !pool.alloc(bytes, off)) return Admit::kWait;
    owner[slot] = id;
    return Admit::kAdmitted;
  }
  void retire(int slot, uint64_t off, uint64_t bytes) {
    owner[slot] = -1;
    pool.release(off, bytes);
  }
};

}  // namespace p1e
