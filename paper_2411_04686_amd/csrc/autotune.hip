// autotune.hip -- picks the SpMV schedule (tile size / lanes per row) of a
// matrix by timing the candidates on the device, with a per-process cache
// and an optional cache file (GSE_AUTOTUNE_CACHE) keyed by the matrix shape
// and a signature of its row lengths.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gse_internal.h"

namespace gse {

gse_status fail(gse_status code, const char* fmt, ...);
gse_status hip_fail(hipError_t e, const char* where);

namespace {

struct Choice {
  int32_t tile;
  int32_t rv;
  float us;
};

std::mutex g_mu;
std::map<std::string, Choice> g_cache;
bool g_file_loaded = false;

std::string key_of(int fmt, int segs, int32_t n_rows, int64_t nnz, int32_t max_row) {
  char b[160];
  snprintf(b, sizeof b, "f%d_s%d_n%d_z%lld_m%d", fmt, segs, n_rows, (long long)nnz, max_row);
  return b;
}

// Row-length signature: the share of rows, in per mille rounded, in each
// length class 0, 1, 2-3, 4-7, ... (classes under half a per mille left
// out), read from the device row pointers once per call.  Matrices of one
// size whose rows are distributed alike share a cache entry; a different
// mix of row lengths is timed anew.
hipError_t row_signature(const int32_t* row_ptr, int32_t n_rows, hipStream_t st, std::string* sig) {
  std::vector<int32_t> rp((size_t)n_rows + 1);
  hipError_t e = hipMemcpyAsync(rp.data(), row_ptr, rp.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  int64_t cls[33] = {0};
  for (int32_t r = 0; r < n_rows; ++r) {
    const uint32_t len = (uint32_t)(rp[r + 1] - rp[r]);
    ++cls[len == 0 ? 0 : 32 - __builtin_clz(len)];
  }
  std::string out = "_r";
  for (int c = 0; c < 33; ++c) {
    const long long pm = n_rows > 0 ? (cls[c] * 1000 + n_rows / 2) / n_rows : 0;
    if (pm == 0) continue;
    char b[32];
    snprintf(b, sizeof b, "%s%d.%lld", out.size() > 2 ? "-" : "", c, pm);
    out += b;
  }
  *sig = out;
  return hipSuccess;
}

void load_file() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char* path = getenv("GSE_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[512];
  int tile, rv;
  float us;
  while (fscanf(f, "%511s %d %d %f", key, &tile, &rv, &us) == 4) g_cache[key] = Choice{tile, rv, us};
  fclose(f);
}

void save_entry(const std::string& k, const Choice& c) {
  const char* path = getenv("GSE_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %.3f\n", k.c_str(), c.tile, c.rv, c.us);
  fclose(f);
}

// Median time (us) of `reps` launches of one schedule.
hipError_t time_one(int fmt, SpmvOperand op, const double* x, double* y, int reps, hipStream_t st,
                    float* us) {
  SpmvEpilogue ep{};
  ep.epi = kEpiPlain;
  hipError_t e = launch_spmv(fmt, op, x, y, ep, st);  // warm-up
  if (e != hipSuccess) return e;
  std::vector<float> t;
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch_spmv(fmt, op, x, y, ep, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    t.push_back(ms * 1000.f);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return e;
  std::sort(t.begin(), t.end());
  *us = t[t.size() / 2];
  return hipSuccess;
}

}  // namespace

gse_status autotune(int fmt, int segs, SpmvOperand op, const int32_t* row_ptr, int32_t* tile_row,
                    int32_t tile_cap, int32_t max_row, const double* x, double* y, int32_t reps,
                    hipStream_t st, int32_t* out_tile, int32_t* out_rv, int32_t* out_tiles) {
  const bool blocks = op.block_sem != nullptr;  // per-block tables
  std::string sig;
  if (hipError_t e = row_signature(row_ptr, op.n_rows, st, &sig); e != hipSuccess)
    return hip_fail(e, "autotune row signature");
  const std::string k = key_of(fmt, segs, op.n_rows, op.nnz, max_row) + sig + (blocks ? "_b" : "");
  {
    std::lock_guard<std::mutex> lock(g_mu);
    load_file();
    auto it = g_cache.find(k);
    if (it != g_cache.end()) {
      *out_tile = it->second.tile;
      *out_rv = it->second.rv;
      *out_tiles = n_tiles_for(op.nnz, *out_tile);
      hipError_t e = launch_plan(row_ptr, op.n_rows, op.nnz, *out_tile, *out_tiles, tile_row, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      return e == hipSuccess ? GSE_OK : hip_fail(e, "autotune plan");
    }
  }
  struct Cand {
    int tile, rv;
  };
  std::vector<Cand> cands;
  if (blocks) {  // the row-tile ring (short rows) or the row-vector schedule
    if (max_row <= 8 && op.nnz >= 1024) cands.push_back({1024, 0});
    for (int L : {1, 2, 4, 8, 16, 32, 64}) cands.push_back({1024, L});
  } else {
    cands = {{1024, 0}, {2048, 0}, {4096, 0}};
    if (max_row <= 64)  // row-vector widths from an eighth of the longest row up
      for (int L : {1, 2, 4, 8, 16, 32, 64})
        if (L >= max_row / 8) cands.push_back({1024, L});
  }
  Choice best{0, 0, 1e30f};
  for (const Cand& c : cands) {
    const int32_t nt = n_tiles_for(op.nnz, c.tile);
    if (tile_cap < nt + 2) continue;
    hipError_t e = launch_plan(row_ptr, op.n_rows, op.nnz, c.tile, nt, tile_row, st);
    SpmvOperand o = op;
    o.tile_row = tile_row;
    o.tile_nnz = c.tile;
    o.n_tiles = nt;
    o.rv_lanes = c.rv;
    float us = 0.f;
    if (e == hipSuccess) e = time_one(fmt, o, x, y, reps, st, &us);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (us < best.us) best = Choice{c.tile, c.rv, us};
  }
  const int32_t nt = n_tiles_for(op.nnz, best.tile);
  hipError_t e = launch_plan(row_ptr, op.n_rows, op.nnz, best.tile, nt, tile_row, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "autotune plan");
  {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[k] = best;
    save_entry(k, best);
  }
  *out_tile = best.tile;
  *out_rv = best.rv;
  *out_tiles = nt;
  return GSE_OK;
}

}  // namespace gse
