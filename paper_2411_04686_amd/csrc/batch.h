// batch.h -- batched stepped CG: many independent systems advanced together
// by one set of kernel launches per iteration (internal to libgse).
#pragma once

#include <chrono>
#include <vector>

#include "gse_internal.h"
#include "solver_state.h"

namespace gse {

constexpr int kChunk = 2048;  // rows per vector work item

// Device descriptor of one system in the batch.
struct BatchSlot {
  const int32_t* row_ptr;
  const int32_t* tile_row;
  const uint32_t* col;
  const uint16_t* head;
  const uint16_t* tail1;
  const uint32_t* tail2;
  const double* val;
  const double* b;
  double* x;
  double* r;
  double* p;
  double* q;
  double* w;
  double* hist;
  int32_t* seg_hist;
  int32_t n_rows;
  int32_t n_tiles;
  int32_t n_chunks;
  int32_t fmt;  // 1: GSE-SEM (stepped), 0: FP64 CSR
  int32_t max_row;  // non-zeros of the longest row
  ColSplit split;   // column / slot fields of the column words
  int16_t sem[GSE_MAX_EXP];
  // the matrix's own SpMV plan (filled by the caller)
  int32_t nnz;
  int32_t tile_nnz;
  int32_t rv_lanes;
  // filled by BatchEngine::add: ring = 1 when the system's product runs on
  // the single-system row-tile ring (large systems of short rows); parts =
  // partial slots reserved for its product; n_prod = partials the product
  // writes (n_tiles, or the ring's grid)
  int32_t ring;
  int32_t parts;
  int32_t n_prod;
};

// Rows from which a system of short rows (at most 8 non-zeros, the default
// 1024-non-zero plan) takes its batched product from the row-tile ring
// kernel -- one grouped launch per ring instance and iteration for all such
// systems -- instead of the batched tile kernel.
constexpr int32_t kRingRows = 1 << 16;

// The row-tile ring's operand for a batched system.
SpmvOperand ring_operand(const BatchSlot& B);

// Work items: a tile or a row chunk of one slot, and where its partial sum
// goes; a slot entry for the per-system finishers with its partial ranges.
struct WorkItem {
  int32_t slot;
  int32_t idx;
  int32_t part;
  int32_t pad;
};
struct SlotItem {
  int32_t slot;
  int32_t part;   // first tile partial
  int32_t vpart;  // first chunk partial
  int32_t pad;
};

// Per-slot action of a host round between iteration epochs.
enum Act : int32_t {
  kActNone = 0,
  kActInit = 1,      // ||b||, r = b - A_s x0, rho, p = r, history[0]
  kActReplace = 2,   // r = b - A_s x, rho (keep p)
  kActReplaceP = 3,  // r = b - A_s x, rho, p = r
  kActCheck = 4,     // w = b - A_3 x, ||w||^2 in scratch[0]
  kActZeroX = 5,     // x = 0 (b = 0)
  kActResetP = 6,    // p = r (after a replacement that moved ||r|| by more than 2x)
};

// One work list on the device: counts {tiles, chunks, slots} and entries.
struct ListView {
  const int32_t* counts;
  const WorkItem* tiles;
  const WorkItem* chunks;
  const SlotItem* slots;
};

// What the batched kernels see.
struct BatchView {
  ListView list;
  const BatchSlot* slot;
  SolverState* S;
  const int32_t* act;
  double* part;   // tile partials
  double* part2;  // chunk partials
};

// Host parameters and bookkeeping of one slot.
struct SlotHost {
  int phase = 0;
  int origin = 0;
  bool reset_p = false;
  int nsw = 0;
  int s_final = 3;
  bool stepped = false;
  double tol = 0.0;
  int max_iter = 0;
  int switch_mode = 1;
  double rho_before = 0.0;  // r.r when the switch was decided (switch_mode 2)
  int final_status = 0;
  std::chrono::steady_clock::time_point t0;
  gse_report rep{};
};

// Device header at the start of an engine region (read by gse_batch_history).
struct RegionHeader {
  int64_t magic;
  int32_t n_slots;
  int32_t pad;
  int64_t slots_off;
  int64_t states_off;
};

// One system handed to batch_cg: its operator part of the slot descriptor
// (vectors and history are placed by batch_cg), eta for the controller.
struct BatchSystemDesc {
  BatchSlot slot;
  const double* eta;
  int32_t n_rows;
  int32_t n_tiles;
};

// The engine: device tables carved from one caller region, host mirrors,
// the captured iteration epoch.  Not thread-safe; one stream.
class BatchEngine {
 public:
  static size_t region_bytes(int cap_slots, int64_t cap_tiles, int64_t cap_chunks);
  gse_status init(void* region, size_t bytes, int cap_slots, int64_t cap_tiles, int64_t cap_chunks,
                  hipStream_t st, bool graphs);
  ~BatchEngine();

  // Add a system (operator, vectors and history already placed in device
  // memory); returns the slot id or a negative status.
  int add(const BatchSlot& d, const gse_params* p, const double* eta);
  // One host round: pending actions, or one epoch of iterations.  Slots
  // that finish are appended to `done`.
  gse_status step(std::vector<int>* done);
  int live() const { return n_live_; }
  bool idle() const { return n_live_ == 0; }
  const gse_report& report(int slot) const { return meta_[slot].rep; }
  void release(int slot);
  const BatchSlot* device_slots() const { return slots_; }
  const SolverState* device_states() const { return S_; }
  int capacity() const { return cap_slots_; }

 private:
  gse_status actions(std::vector<int>* done);
  gse_status epoch();
  gse_status upload_list(int which, const std::vector<int>& ids);
  gse_status finish(int slot, int status, std::vector<int>* done);
  void resume(int slot);
  // The recursive residual met the tolerance outside an iteration: check it
  // with all segments on an exact operator, else switch up (trigger TOL).
  void tol_met(int slot);
  BatchView view(int which) const;
  hipError_t launch_epoch_kernels(int iters);
  hipError_t sync_states_in();
  hipError_t sync_states_out();

  int cap_slots_ = 0;
  int64_t cap_tiles_ = 0, cap_chunks_ = 0;
  hipStream_t st_ = nullptr;
  bool graphs_ = true;
  hipGraphExec_t graph_ = nullptr;
  // device tables
  int32_t* counts_[2] = {nullptr, nullptr};
  WorkItem* tiles_[2] = {nullptr, nullptr};
  WorkItem* chunks_[2] = {nullptr, nullptr};
  SlotItem* slot_items_[2] = {nullptr, nullptr};
  BatchSlot* slots_ = nullptr;
  SolverState* S_ = nullptr;
  int32_t* act_ = nullptr;
  double* part_ = nullptr;
  double* part2_ = nullptr;
  // host mirrors
  std::vector<BatchSlot> hslot_;
  std::vector<SolverState> hS_;
  std::vector<int32_t> hact_;
  std::vector<SlotHost> meta_;
  std::vector<char> used_;
  std::vector<WorkItem> wt_[2], wc_[2];
  std::vector<SlotItem> ws_[2];
  std::vector<int> ids_;
  std::vector<int32_t> seg_buf_;
  std::vector<int32_t> prod_off_;   // first product partial of each slot in list 0
  std::vector<int> ring_ids_;       // running systems whose product runs on the ring
  // this epoch's grouped ring products: one launch per instance, over the
  // descriptors [first, first + n) of groups_ and `total` workgroups
  struct RingLaunch {
    RowClass c;
    int first, n, total;
  };
  std::vector<RingLaunch> ring_launches_;
  std::vector<RowGroup> hgroups_;
  RowGroup* groups_ = nullptr;      // device descriptors, one per slot at most
  int32_t hcounts_[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  RegionHeader hhdr_{};
  bool run_dirty_ = true;
  int n_live_ = 0;
  int grid_spmv_ = 0, grid_vec_ = 0, grid_slot_ = 0;
};

size_t batch_workspace_bytes(int32_t n_sys, const BatchSystemDesc* d, int32_t max_iter);
gse_status batch_cg(int32_t n_sys, const BatchSystemDesc* d, const gse_params* p, gse_report* rep,
                    void* ws, size_t ws_bytes, hipStream_t st);
gse_status batch_history(const void* ws, int32_t index, int32_t cap, double* hist, int32_t* seg,
                         hipStream_t st);

}  // namespace gse
