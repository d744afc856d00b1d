// serve.hip -- solver server: requests arrive at any time (host CSR + b),
// are admitted while the caller's device arena and the batch slots allow,
// encoded on the device, and join the running batch of stepped CG solves
// (batch.hip) at the next epoch boundary.  One worker thread owns the
// device work; submit / poll / stats may be called from any thread.
//
// Admission is first-come first-served: the oldest waiting request is
// admitted as soon as a slot is free and both of its blocks (the resident
// one: operator, vectors, history; the transient one: the FP64 CSR copy
// and the encode workspace, released right after the encode) fit in the
// arena; later requests never overtake it.
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "batch.h"

namespace gse {
gse_status fail(gse_status code, const char* fmt, ...);
gse_status hip_fail(hipError_t e, const char* where);
const char* last_error_text();
}  // namespace gse

using gse::Arena;
using gse::RequestLayout;

namespace {

using Clock = std::chrono::steady_clock;

enum TicketState : int { kQueued = 0, kRunning = 1, kDone = 2 };

struct Ticket {
  int state = kQueued;
  gse_request rq{};
  Clock::time_point submitted;
  gse_report rep{};
  std::string err;
  // placement while admitted
  int slot = -1;
  uint64_t res_off = Arena::kNone, res_bytes = 0;
  uint64_t tr_off = Arena::kNone, tr_bytes = 0;
  RequestLayout L{};
  gse_matrix A{};
  gse_csr M{};
};

int64_t pad16(int64_t n) { return (n + 15) / 16 * 16; }

RequestLayout layout_of(const gse_request& rq) {
  int32_t tiles = gse_tile_entries(rq.nnz);
  size_t ews = 0;
  gse_encode_workspace(rq.nnz, rq.n_rows, &ews);
  return gse::request_layout(rq.format == GSE_FMT_GSE ? 1 : 0, (uint64_t)rq.n_rows,
                             (uint64_t)rq.nnz, (uint64_t)pad16(rq.nnz), (uint64_t)tiles,
                             (uint64_t)rq.params.max_iter, (uint64_t)ews);
}

}  // namespace

struct gse_solver {
  std::mutex mu;
  std::condition_variable cv;
  std::condition_variable ready_cv;
  std::thread worker;
  bool stop = false;
  bool ready = false;
  gse_status init_status = GSE_OK;
  std::string init_err;
  gse_status fatal = GSE_OK;
  std::string fatal_err;

  char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  int device = 0;
  hipStream_t caller = nullptr;
  hipStream_t st = nullptr;

  char* pool_base = nullptr;
  Arena pool;
  gse::BatchEngine eng;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::vector<uint64_t> slot_ticket;
  uint64_t next_ticket = 1;
  // counters
  uint64_t admitted = 0, completed = 0;
  uint64_t peak_used = 0;
  int running = 0;
};

namespace {

// Device region of the batch engine inside the arena, sized for max_slots
// systems whose operators fill the rest of the arena.
void engine_caps(size_t arena_bytes, int max_slots, int64_t* tiles, int64_t* chunks) {
  *tiles = (int64_t)(arena_bytes / (12 * 1024)) + 2 * max_slots;
  *chunks = (int64_t)(arena_bytes / (48 * (size_t)gse::kChunk)) + 2 * max_slots;
}

// Copy the request to its blocks, encode (GSE) or plan (FP64), build the
// slot descriptor.  Runs on the worker thread.
gse_status place(gse_solver* s, Ticket& t, gse::BatchSlot* B, const double** eta) {
  const gse_request& rq = t.rq;
  const RequestLayout& L = t.L;
  char* res = s->pool_base + t.res_off;
  const int n = rq.n_rows;
  const int64_t nnz = rq.nnz;
  hipStream_t st = s->st;
  auto at = [&](uint64_t off) { return res + off; };
  hipError_t e = hipMemcpyAsync(at(L.row_ptr), rq.row_ptr, sizeof(int32_t) * (size_t)(n + 1),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at(L.b), rq.b, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    if (rq.x0_given)
      e = hipMemcpyAsync(at(L.x), rq.x, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, st);
    else
      e = hipMemsetAsync(at(L.x), 0, sizeof(double) * (size_t)n, st);
  }
  if (e != hipSuccess) return gse::hip_fail(e, "serve upload");
  memset(B, 0, sizeof *B);
  if (rq.format == GSE_FMT_GSE) {
    char* tr = s->pool_base + t.tr_off;
    e = hipMemcpyAsync(tr + L.t_col, rq.col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tr + L.t_val, rq.val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return gse::hip_fail(e, "serve upload");
    gse_matrix& A = t.A;
    memset(&A, 0, sizeof A);
    A.col_idx = reinterpret_cast<uint32_t*>(at(L.col));
    A.head = reinterpret_cast<uint16_t*>(at(L.head));
    A.tail1 = reinterpret_cast<uint16_t*>(at(L.tail1));
    A.tail2 = reinterpret_cast<uint32_t*>(at(L.tail2));
    A.tile_row = reinterpret_cast<int32_t*>(at(L.tile_row));
    A.tile_cap = gse_tile_entries(nnz);
    size_t ews = 0;
    gse_encode_workspace(nnz, n, &ews);
    gse_status es = gse_encode(reinterpret_cast<const int32_t*>(at(L.row_ptr)),
                               reinterpret_cast<const int32_t*>(tr + L.t_col),
                               reinterpret_cast<const double*>(tr + L.t_val), n, n, nnz,
                               rq.num_exp, nullptr, &A, tr + L.t_ws, ews, st);
    if (es != GSE_OK) return es;
    B->row_ptr = A.row_ptr;
    B->tile_row = A.tile_row;
    B->col = A.col_idx;
    B->head = A.head;
    B->tail1 = A.tail1;
    B->tail2 = A.tail2;
    B->n_tiles = A.n_tiles;
    B->fmt = 1;
    B->max_row = A.max_row_nnz;
    B->split = gse::col_split(A.idx_bits, A.idx_layout == GSE_IDX_VALUE);
    for (int k = 0; k < GSE_MAX_EXP; ++k) B->sem[k] = A.sem[k];
    B->nnz = (int32_t)A.nnz;
    B->tile_nnz = A.tile_nnz;
    B->rv_lanes = A.rv_lanes;
    *eta = t.A.eta;
  } else {
    const int64_t pad = pad16(nnz);
    e = hipMemsetAsync(at(L.col), 0, sizeof(int32_t) * (size_t)pad, st);
    if (e == hipSuccess) e = hipMemsetAsync(at(L.val), 0, sizeof(double) * (size_t)pad, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(at(L.col), rq.col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(at(L.val), rq.val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return gse::hip_fail(e, "serve upload");
    gse_csr& M = t.M;
    memset(&M, 0, sizeof M);
    M.n_rows = n;
    M.n_cols = n;
    M.nnz = nnz;
    M.row_ptr = reinterpret_cast<const int32_t*>(at(L.row_ptr));
    M.col = reinterpret_cast<const int32_t*>(at(L.col));
    M.val = reinterpret_cast<const double*>(at(L.val));
    M.tile_row = reinterpret_cast<int32_t*>(at(L.tile_row));
    M.tile_cap = gse_tile_entries(nnz);
    gse_status ps = gse_csr_plan(&M, 1024, 0, st);
    if (ps != GSE_OK) return ps;
    B->row_ptr = M.row_ptr;
    B->tile_row = M.tile_row;
    B->col = reinterpret_cast<const uint32_t*>(M.col);
    B->val = M.val;
    B->n_tiles = M.n_tiles;
    B->fmt = 0;
    B->max_row = M.max_row_nnz;
    B->split = gse::col_split(0);
    B->nnz = (int32_t)M.nnz;
    B->tile_nnz = M.tile_nnz;
    B->rv_lanes = M.rv_lanes;
    *eta = nullptr;
  }
  B->b = reinterpret_cast<const double*>(at(L.b));
  B->x = reinterpret_cast<double*>(at(L.x));
  B->r = reinterpret_cast<double*>(at(L.r));
  B->p = reinterpret_cast<double*>(at(L.p));
  B->q = reinterpret_cast<double*>(at(L.q));
  B->w = reinterpret_cast<double*>(at(L.w));
  B->hist = reinterpret_cast<double*>(at(L.hist));
  B->seg_hist = reinterpret_cast<int32_t*>(at(L.seg));
  B->n_rows = n;
  B->n_chunks = (n + gse::kChunk - 1) / gse::kChunk;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return gse::hip_fail(e, "serve encode");
  return GSE_OK;
}

// Under the lock: free a ticket's blocks.
void free_blocks(gse_solver* s, Ticket& t) {
  if (t.res_off != Arena::kNone) s->pool.release(t.res_off, t.res_bytes);
  if (t.tr_off != Arena::kNone) s->pool.release(t.tr_off, t.tr_bytes);
  t.res_off = t.tr_off = Arena::kNone;
}

void complete(gse_solver* s, uint64_t id, const gse_report& rep, const char* err) {
  Ticket& t = s->tickets[id];
  t.rep = rep;
  t.rep.time_ms = std::chrono::duration<double, std::milli>(Clock::now() - t.submitted).count();
  if (err) t.err = err;
  t.state = kDone;
  ++s->completed;
}

void worker_main(gse_solver* s) {
  hipError_t e = hipSetDevice(s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
  gse_status ist = GSE_OK;
  if (e != hipSuccess) ist = gse::hip_fail(e, "serve worker");
  if (ist == GSE_OK) {
    int64_t tiles, chunks;
    engine_caps(s->arena_bytes, s->max_slots, &tiles, &chunks);
    const size_t eb = gse::BatchEngine::region_bytes(s->max_slots, tiles, chunks);
    if (eb >= s->arena_bytes) {
      ist = gse::fail(GSE_ERR_NOMEM, "arena of %zu bytes cannot hold the batch tables (%zu)",
                      s->arena_bytes, eb);
    } else {
      ist = s->eng.init(s->arena, eb, s->max_slots, tiles, chunks, s->st, true);
      s->pool_base = s->arena + eb;
      s->pool.reset(s->arena_bytes - eb);
    }
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->init_status = ist;
    if (ist != GSE_OK) s->init_err = gse::last_error_text();
    s->ready = true;
  }
  s->ready_cv.notify_all();
  if (ist != GSE_OK) return;

  std::vector<uint64_t> admit;
  std::vector<int> done;
  for (;;) {
    admit.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto admissible = [&] {
        if (s->queue.empty() || s->running >= s->max_slots) return false;
        Ticket& t = s->tickets[s->queue.front()];
        const uint64_t ro = s->pool.alloc(t.L.resident);
        if (ro == Arena::kNone) return false;
        uint64_t to = Arena::kNone;
        if (t.L.transient > 0) {
          to = s->pool.alloc(t.L.transient);
          if (to == Arena::kNone) {
            s->pool.release(ro, t.L.resident);
            return false;
          }
        }
        t.res_off = ro;
        t.res_bytes = t.L.resident;
        t.tr_off = to;
        t.tr_bytes = t.L.transient;
        return true;
      };
      s->cv.wait(lk, [&] {
        return s->stop || s->eng.live() > 0 ||
               (!s->queue.empty() && s->running < s->max_slots);
      });
      if (s->stop) break;
      while (admissible()) {
        const uint64_t id = s->queue.front();
        s->queue.pop_front();
        s->tickets[id].state = kRunning;
        ++s->running;
        ++s->admitted;
        admit.push_back(id);
      }
      if (s->pool.used() > s->peak_used) s->peak_used = s->pool.used();
      if (admit.empty() && s->eng.live() == 0) {
        // the oldest request does not fit yet and nothing runs: it never will
        if (!s->queue.empty() && s->running == 0) {
          const uint64_t id = s->queue.front();
          s->queue.pop_front();
          gse_report rep{};
          rep.status = GSE_ERR_NOMEM;
          complete(s, id, rep, "request does not fit in the arena");
        }
        continue;
      }
    }
    for (uint64_t id : admit) {
      Ticket* t;
      {
        std::lock_guard<std::mutex> g(s->mu);
        t = &s->tickets[id];
      }
      gse::BatchSlot B;
      const double* eta = nullptr;
      gse_status ps = place(s, *t, &B, &eta);
      int slot = -1;
      if (ps == GSE_OK) {
        slot = s->eng.add(B, &t->rq.params, eta);
        if (slot < 0) ps = slot;
      }
      std::lock_guard<std::mutex> g(s->mu);
      if (t->tr_off != Arena::kNone) {
        s->pool.release(t->tr_off, t->tr_bytes);
        t->tr_off = Arena::kNone;
      }
      if (ps != GSE_OK) {
        gse_report rep{};
        rep.status = ps;
        free_blocks(s, *t);
        --s->running;
        complete(s, id, rep, gse::last_error_text());
        if (ps == GSE_ERR_HIP) {
          s->fatal = ps;
          s->fatal_err = gse::last_error_text();
        }
        continue;
      }
      t->slot = slot;
      if ((int)s->slot_ticket.size() <= slot) s->slot_ticket.resize((size_t)slot + 1, 0);
      s->slot_ticket[slot] = id;
    }
    done.clear();
    gse_status st = s->eng.step(&done);
    if (st != GSE_OK) {
      std::lock_guard<std::mutex> g(s->mu);
      s->fatal = st;
      s->fatal_err = gse::last_error_text();
      // every running ticket ends with the error
      for (auto& kv : s->tickets)
        if (kv.second.state == kRunning) {
          gse_report rep{};
          rep.status = st;
          free_blocks(s, kv.second);
          complete(s, kv.first, rep, s->fatal_err.c_str());
        }
      s->running = 0;
      break;
    }
    for (int slot : done) {
      uint64_t id;
      Ticket* t;
      {
        std::lock_guard<std::mutex> g(s->mu);
        id = s->slot_ticket[slot];
        t = &s->tickets[id];
      }
      const gse_report rep = s->eng.report(slot);
      hipError_t ce = hipMemcpyAsync(t->rq.x, s->pool_base + t->res_off + t->L.x,
                                     sizeof(double) * (size_t)t->rq.n_rows, hipMemcpyDeviceToHost, s->st);
      if (ce == hipSuccess) ce = hipStreamSynchronize(s->st);
      std::lock_guard<std::mutex> g(s->mu);
      s->eng.release(slot);
      free_blocks(s, *t);
      --s->running;
      if (ce != hipSuccess) {
        gse_report bad = rep;
        bad.status = GSE_ERR_HIP;
        complete(s, id, bad, hipGetErrorString(ce));
      } else {
        complete(s, id, rep, nullptr);
      }
    }
  }
  // drain: the engine's work is synchronous per step, nothing is in flight
}

gse_status check_request(const gse_request* rq) {
  if (!rq) return gse::fail(GSE_ERR_ARG, "request is NULL");
  if (rq->format != GSE_FMT_GSE && rq->format != GSE_FMT_CSR64)
    return gse::fail(GSE_ERR_ARG, "unknown format %d", rq->format);
  if (rq->n_rows < 1 || rq->nnz < 0) return gse::fail(GSE_ERR_ARG, "bad sizes");
  if (rq->nnz > (int64_t(1) << 31) - (int64_t(1) << 16)) return gse::fail(GSE_ERR_RANGE, "nnz too large");
  if (!rq->row_ptr || !rq->b || !rq->x || (rq->nnz > 0 && (!rq->col || !rq->val)))
    return gse::fail(GSE_ERR_ARG, "NULL request array");
  if (rq->format == GSE_FMT_GSE && (rq->num_exp < 1 || rq->num_exp > GSE_MAX_EXP))
    return gse::fail(GSE_ERR_ARG, "num_exp must be 1..64");
  // (a system wider than the column field keeps its slot index in the value)
  const gse_params& p = rq->params;
  if (!(p.tol > 0.0) || p.max_iter < 0) return gse::fail(GSE_ERR_ARG, "tol must be > 0, max_iter >= 0");
  if (p.start_segments < 1 || p.start_segments > 3 || p.fixed_segments < 0 || p.fixed_segments > 3)
    return gse::fail(GSE_ERR_ARG, "segment counts must be 1..3 (fixed: 0..3)");
  if (p.l < 0 || p.t < 1 || p.m < 0) return gse::fail(GSE_ERR_ARG, "controller needs l >= 0, t >= 1, m >= 0");
  // the CSR structure is read by the kernels: check it here
  const int32_t* rp = rq->row_ptr;
  if (rp[0] != 0 || (int64_t)rp[rq->n_rows] != rq->nnz)
    return gse::fail(GSE_ERR_ARG, "row_ptr must start at 0 and end at nnz");
  for (int i = 0; i < rq->n_rows; ++i)
    if (rp[i + 1] < rp[i]) return gse::fail(GSE_ERR_ARG, "row_ptr must be non-decreasing");
  for (int64_t j = 0; j < rq->nnz; ++j)
    if (rq->col[j] < 0 || rq->col[j] >= rq->n_rows)
      return gse::fail(GSE_ERR_ARG, "column index out of range");
  return GSE_OK;
}

}  // namespace

extern "C" {

gse_status gse_solver_create(void* arena, size_t arena_bytes, int32_t max_slots, void* stream,
                             gse_solver** out) {
  if (!out || !arena || (reinterpret_cast<uintptr_t>(arena) & 255u) || max_slots < 1 ||
      max_slots > 65536)
    return gse::fail(GSE_ERR_ARG, "bad arguments");
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && stream) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return gse::hip_fail(e, "gse_solver_create");
  gse_solver* s = new gse_solver();
  s->arena = reinterpret_cast<char*>(arena);
  s->arena_bytes = arena_bytes;
  s->max_slots = max_slots;
  s->device = dev;
  s->caller = (hipStream_t)stream;
  s->slot_ticket.assign((size_t)max_slots, 0);
  s->worker = std::thread(worker_main, s);
  std::unique_lock<std::mutex> lk(s->mu);
  s->ready_cv.wait(lk, [&] { return s->ready; });
  const gse_status ist = s->init_status;
  const std::string err = s->init_err;
  lk.unlock();
  if (ist != GSE_OK) {
    s->worker.join();
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return gse::fail(ist, "%s", err.c_str());
  }
  *out = s;
  return GSE_OK;
}

gse_status gse_solver_footprint(const gse_request* rq, size_t* resident, size_t* transient) {
  if (!rq || !resident || !transient) return gse::fail(GSE_ERR_ARG, "bad arguments");
  if (rq->n_rows < 1 || rq->nnz < 0 || rq->params.max_iter < 0 ||
      (rq->format != GSE_FMT_GSE && rq->format != GSE_FMT_CSR64))
    return gse::fail(GSE_ERR_ARG, "bad request sizes");
  const RequestLayout L = layout_of(*rq);
  *resident = (size_t)L.resident;
  *transient = (size_t)L.transient;
  return GSE_OK;
}

gse_status gse_solver_submit(gse_solver* s, const gse_request* rq, uint64_t* ticket) {
  if (!s || !ticket) return gse::fail(GSE_ERR_ARG, "bad arguments");
  gse_status c = check_request(rq);
  if (c != GSE_OK) return c;
  const RequestLayout L = layout_of(*rq);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->fatal != GSE_OK) return gse::fail(s->fatal, "server stopped: %s", s->fatal_err.c_str());
  if (L.resident + L.transient > s->pool.total())
    return gse::fail(GSE_ERR_NOMEM, "request needs %llu bytes, the arena holds %llu",
                     (unsigned long long)(L.resident + L.transient),
                     (unsigned long long)s->pool.total());
  const uint64_t id = s->next_ticket++;
  Ticket& t = s->tickets[id];
  t.rq = *rq;
  t.L = L;
  t.submitted = Clock::now();
  t.state = kQueued;
  s->queue.push_back(id);
  *ticket = id;
  s->cv.notify_all();
  return GSE_OK;
}

gse_status gse_solver_poll(gse_solver* s, uint64_t ticket, gse_report* rep) {
  if (!s || !rep) return gse::fail(GSE_ERR_ARG, "bad arguments");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return gse::fail(GSE_ERR_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second.state != kDone) return GSE_PENDING;
  *rep = it->second.rep;
  const std::string err = it->second.err;
  s->tickets.erase(it);
  if (rep->status < 0 && !err.empty()) gse::fail(rep->status, "%s", err.c_str());
  return GSE_OK;
}

gse_status gse_solver_stats(gse_solver* s, gse_server_stats* out) {
  if (!s || !out) return gse::fail(GSE_ERR_ARG, "bad arguments");
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->queued = (int64_t)s->queue.size();
  out->running = s->running;
  out->admitted = (int64_t)s->admitted;
  out->completed = (int64_t)s->completed;
  out->arena_bytes = (int64_t)s->pool.total();
  out->arena_used = (int64_t)s->pool.used();
  out->arena_peak = (int64_t)s->peak_used;
  out->arena_largest_free = (int64_t)s->pool.largest_free();
  return GSE_OK;
}

gse_status gse_solver_destroy(gse_solver* s) {
  if (!s) return gse::fail(GSE_ERR_ARG, "solver is NULL");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->st) {
    (void)hipStreamSynchronize(s->st);
    (void)hipStreamDestroy(s->st);
  }
  delete s;
  return GSE_OK;
}

}  // extern "C"
