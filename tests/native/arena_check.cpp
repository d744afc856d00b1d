// Host check of the solver server's arena allocator and request layout
// (arena.h): random allocate / release sequences against an explicit model,
// and the buffer layout of requests of many shapes.  Prints "ok" or the
// first violated property and exits non-zero.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.h"

using gse::Arena;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      printf("FAIL %s: ", #c);             \
      printf(__VA_ARGS__);                 \
      printf("\n");                        \
      if (++fails > 5) exit(1);            \
    }                                      \
  } while (0)

struct Block {
  uint64_t off, bytes;
};

static void check_state(const Arena& a, const std::vector<Block>& live, uint64_t total) {
  // live blocks inside the arena and pairwise disjoint
  std::vector<char> map(total / Arena::kAlign, 0);
  uint64_t used = 0;
  for (const Block& b : live) {
    const uint64_t n = Arena::round_up(b.bytes ? b.bytes : 1);
    CHECK(b.off % Arena::kAlign == 0, "offset %llu unaligned", (unsigned long long)b.off);
    CHECK(b.off + n <= total, "block past the end");
    for (uint64_t u = b.off / Arena::kAlign; u < (b.off + n) / Arena::kAlign; ++u) {
      CHECK(!map[u], "overlap at unit %llu", (unsigned long long)u);
      map[u] = 1;
    }
    used += n;
  }
  CHECK(a.used() == used, "used %llu != %llu", (unsigned long long)a.used(), (unsigned long long)used);
  // free list: exactly the complement, maximal runs (coalesced)
  uint64_t prev_end = ~uint64_t(0), free_sum = 0;
  for (const auto& kv : a.free_blocks()) {
    CHECK(kv.first != prev_end, "adjacent free blocks not merged at %llu", (unsigned long long)kv.first);
    for (uint64_t u = kv.first / Arena::kAlign; u < (kv.first + kv.second) / Arena::kAlign; ++u) {
      CHECK(!map[u], "free block overlaps a live one");
      map[u] = 2;
    }
    prev_end = kv.first + kv.second;
    free_sum += kv.second;
  }
  CHECK(free_sum + used == total, "free + used != total");
}

int main() {
  std::mt19937_64 rng(12345);
  for (int trial = 0; trial < 40; ++trial) {
    const uint64_t total = (64 + rng() % 4096) * Arena::kAlign;
    Arena a;
    a.reset(total + (rng() % Arena::kAlign));  // ragged size: rounded down
    CHECK(a.total() == total, "total");
    std::vector<Block> live;
    for (int step = 0; step < 3000; ++step) {
      if (live.empty() || rng() % 3 != 0) {
        const uint64_t bytes = (rng() % 8 == 0) ? 0 : rng() % (total / 8 + 1);
        const uint64_t off = a.alloc(bytes);
        if (off == Arena::kNone) {
          // first fit fails only if no free block is large enough
          CHECK(a.largest_free() < Arena::round_up(bytes ? bytes : 1), "spurious failure");
        } else {
          live.push_back({off, bytes});
        }
      } else {
        const size_t k = rng() % live.size();
        a.release(live[k].off, live[k].bytes);
        live.erase(live.begin() + (long)k);
      }
      if (step % 97 == 0) check_state(a, live, total);
    }
    for (const Block& b : live) a.release(b.off, b.bytes);
    live.clear();
    check_state(a, live, total);
    CHECK(a.fragments() == 1 && a.largest_free() == total, "not whole again after freeing all");
  }
  // request layouts: buffers aligned, disjoint, inside their block
  for (int fmt = 0; fmt <= 1; ++fmt)
    for (uint64_t n : {uint64_t(1), uint64_t(7), uint64_t(1000), uint64_t(123457)})
      for (uint64_t nnz : {uint64_t(0), uint64_t(1), 5 * n, 7 * n + 3})
        for (uint64_t it : {uint64_t(0), uint64_t(1), uint64_t(5000)}) {
          const uint64_t pad = (nnz + 15) / 16 * 16;
          const uint64_t tiles = (nnz + 1023) / 1024 + 2 + (nnz == 0);
          const gse::RequestLayout L = gse::request_layout(fmt, n, nnz, pad, tiles, it, 8448);
          struct Buf {
            uint64_t off, bytes;
          };
          std::vector<Buf> res = {{L.row_ptr, 4 * (n + 1)}, {L.col, 4 * pad}, {L.tile_row, 4 * tiles},
                                  {L.b, 8 * n}, {L.x, 8 * n}, {L.r, 8 * n}, {L.p, 8 * n},
                                  {L.q, 8 * n}, {L.w, 8 * n}, {L.hist, 8 * (it + 2)},
                                  {L.seg, 4 * (it + 2)}};
          if (fmt == 1) {
            res.push_back({L.head, 2 * pad});
            res.push_back({L.tail1, 2 * pad});
            res.push_back({L.tail2, 4 * pad});
          } else {
            res.push_back({L.val, 8 * pad});
          }
          for (size_t i = 0; i < res.size(); ++i) {
            CHECK(res[i].off % Arena::kAlign == 0, "unaligned buffer");
            CHECK(res[i].off + res[i].bytes <= L.resident, "buffer %zu outside the block", i);
            for (size_t j = 0; j < i; ++j)
              CHECK(res[i].off + res[i].bytes <= res[j].off || res[j].off + res[j].bytes <= res[i].off,
                    "buffers %zu and %zu overlap", i, j);
          }
          if (fmt == 1) {
            CHECK(L.t_col + 4 * nnz <= L.t_val && L.t_val + 8 * nnz <= L.t_ws &&
                      L.t_ws + 8448 <= L.transient,
                  "transient layout");
          } else {
            CHECK(L.transient == 0, "FP64 requests have no transient block");
          }
        }
  if (fails) return 1;
  printf("ok\n");
  return 0;
}
