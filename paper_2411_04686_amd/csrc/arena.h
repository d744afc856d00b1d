// arena.h -- host-side bookkeeping of the solver server: a first-fit
// allocator over one caller-owned device region and the layout of one
// request inside its blocks.  Plain C++ (no HIP), so it is unit-tested on
// the host.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace gse {

// First-fit allocator of 256-byte aligned blocks inside [0, bytes).  Free
// blocks are kept by offset and merged with their neighbours on release.
class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  static constexpr uint64_t kNone = ~uint64_t(0);

  static uint64_t round_up(uint64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

  void reset(uint64_t bytes) {
    free_.clear();
    total_ = bytes / kAlign * kAlign;
    used_ = 0;
    if (total_ > 0) free_[0] = total_;
  }

  // Offset of a new block of at least `bytes`, or kNone.
  uint64_t alloc(uint64_t bytes) {
    const uint64_t need = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, size = it->second;
      free_.erase(it);
      if (size > need) free_[off + need] = size - need;
      used_ += need;
      return off;
    }
    return kNone;
  }

  // Return a block obtained from alloc(bytes) at `off`.
  void release(uint64_t off, uint64_t bytes) {
    const uint64_t need = round_up(bytes ? bytes : 1);
    used_ -= need;
    uint64_t start = off, size = need;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + need == next->first) {
      size += next->second;
      free_.erase(next);
    }
    free_[start] = size;
  }

  uint64_t total() const { return total_; }
  uint64_t used() const { return used_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  size_t fragments() const { return free_.size(); }
  const std::map<uint64_t, uint64_t>& free_blocks() const { return free_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t total_ = 0, used_ = 0;
};

// Byte offsets of one request's buffers.  The resident block lives until the
// solve ends; the transient block (the FP64 CSR copy and the encode
// workspace of a GSE request) only until its encode ends.
struct RequestLayout {
  // resident
  uint64_t row_ptr, col, head, tail1, tail2, val, tile_row;
  uint64_t b, x, r, p, q, w, hist, seg;
  uint64_t resident;
  // transient (GSE only)
  uint64_t t_col, t_val, t_ws;
  uint64_t transient;
};

// fmt 1: GSE-SEM planes; fmt 0: FP64 CSR.  pad: entries of a plane
// (nnz rounded up to 16), tile_entries: the tile table's length,
// encode_ws: the encode workspace bytes.
inline RequestLayout request_layout(int fmt, uint64_t n, uint64_t nnz, uint64_t pad,
                                    uint64_t tile_entries, uint64_t max_iter, uint64_t encode_ws) {
  RequestLayout L{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += Arena::round_up(bytes ? bytes : 1);
    return o;
  };
  const uint64_t none = Arena::kNone;
  L.row_ptr = take(4 * (n + 1));
  L.col = take(4 * pad);
  if (fmt == 1) {
    L.head = take(2 * pad);
    L.tail1 = take(2 * pad);
    L.tail2 = take(4 * pad);
    L.val = none;
  } else {
    L.head = L.tail1 = L.tail2 = none;
    L.val = take(8 * pad);
  }
  L.tile_row = take(4 * tile_entries);
  L.b = take(8 * n);
  L.x = take(8 * n);
  L.r = take(8 * n);
  L.p = take(8 * n);
  L.q = take(8 * n);
  L.w = take(8 * n);
  L.hist = take(8 * (max_iter + 2));
  L.seg = take(4 * (max_iter + 2));
  L.resident = off;
  off = 0;
  if (fmt == 1) {
    L.t_col = take(4 * (nnz ? nnz : 1));
    L.t_val = take(8 * (nnz ? nnz : 1));
    L.t_ws = take(encode_ws);
    L.transient = off;
  } else {
    L.t_col = L.t_val = L.t_ws = none;
    L.transient = 0;
  }
  return L;
}

}  // namespace gse
