// solver_state.h -- device state record of one solve and the stepped
// controller, shared by the single-system and the batched solvers.
#pragma once

#include <math.h>

#include "gse_internal.h"

namespace gse {

enum Stop : int { kRun = 0, kConv = 1, kSwitch = 2, kBreak = 3, kCap = 4 };

// Device-resident solver state.
struct SolverState {
  double rho;        // r.r
  double pq;         // p.q (CG) or scratch dot
  double alpha, beta;
  double nb;         // ||b||
  double nb2;        // b.b
  double relres;     // current recursive residual / ||b||
  double tol;
  double eta[3];
  double floor_c;
  double rsd_limit, reldec_limit;
  double scratch[4];
  int it;            // completed iterations
  int s;             // segment count in use (0: FP64 CSR)
  int stop;          // Stop
  int trig;          // trigger of a switch
  int k3_armed;      // batched CG: the x/p update of the last completed iteration is pending
  int go;            // CG: this iteration's r step ran (read by the x step)
  int it_next;       // CG: the iteration the r step started
  int max_iter;
  int stepped;
  int fixed;
  int l, t, m, ndec_limit, ndec_rule;
  int pad0;
  long long hist_off;  // byte offsets of the residual / segment histories
  long long seg_off;   // in the workspace (read by gse_solve_history)
  int hist_cap;
  int pad1;
  double rho_p[2];   // CG: r.r after `it` iterations lives in rho_p[it & 1]
};

// ------------------------------------------------------------ controller --
// Conditions 1-3 at j = l + q*m once t residuals exist (Section III-D).
// RSD (Eq. 3): population standard deviation over resid[j-t..j-1] divided
// by their mean; nDec (Eqs. 4-5): decreases resid[i] > resid[i+1] for
// i = j-t..j-1; relDec (Eq. 6): (resid[j-t] - resid[j-1]) / resid[j-t].
// Called by every thread of one workgroup of NT threads; returns the
// trigger (1..3) or 0.
template <int NT = kWG>
__device__ inline int grid_conditions(const SolverState* S, const double* hist, int j, double* red) {
  const int t = S->t;
  double sum = 0.0;
  for (int i = threadIdx.x; i < t; i += NT) sum += hist[j - t + i];
  const double avg = block_sum<NT>(sum, red) / (double)t;
  double var = 0.0, dec = 0.0;
  for (int i = threadIdx.x; i < t; i += NT) {
    const double d = hist[j - t + i] - avg;
    var += d * d;
    dec += (hist[j - t + i] > hist[j - t + i + 1]) ? 1.0 : 0.0;
  }
  var = block_sum<NT>(var, red) / (double)t;
  const int ndec = (int)block_sum<NT>(dec, red);
  const double rsd = sqrt(var) / avg;
  const double reldec = (hist[j - t] - hist[j - 1]) / hist[j - t];
  bool below;
  if (S->ndec_rule == 1) below = 2 * ndec < t;
  else below = ndec < S->ndec_limit;
  if (rsd > S->rsd_limit && below) return GSE_TRIG_C1;
  if (!below && reldec < S->reldec_limit) return GSE_TRIG_C2;
  if (ndec == 0) return GSE_TRIG_C3;
  return GSE_TRIG_NONE;
}

// Whether the controller evaluates Conditions 1-3 after iteration j (it
// then reads the residual history of the last t iterations).
__device__ inline bool on_check_grid(const SolverState* S, int j, double relres, int s) {
  return S->stepped && s < 3 && relres > S->tol && j >= S->l && j >= S->t && S->m > 0 &&
         ((j - S->l) % S->m) == 0;
}

// After iteration j recorded relres (values broadcast through LDS by the
// caller): convergence, the floor and tolerance triggers, Conditions 1-3 on
// the check grid, the cap.  Every thread of the workgroup (NT threads)
// calls it.
template <int NT = kWG>
__device__ inline void controller(SolverState* S, const double* hist, double* red, int j, double relres,
                           int s) {
  const bool exact_op = S->fixed != 0 || s >= 3 || S->eta[s - 1] == 0.0;
  const bool on_grid = on_check_grid(S, j, relres, s);
  int cond = GSE_TRIG_NONE;
  if (on_grid) cond = grid_conditions<NT>(S, hist, j, red);  // uniform branch
  if (threadIdx.x == 0) {
    int stop = kRun, trig = GSE_TRIG_NONE;
    if (relres <= S->tol) {
      if (exact_op) stop = kConv;
      else { stop = kSwitch; trig = GSE_TRIG_TOL; }
    } else if (S->stepped && s < 3) {
      const double eta = S->eta[s - 1];
      if (S->floor_c > 0.0 && eta > 0.0 && relres <= S->floor_c * eta) {
        stop = kSwitch;
        trig = GSE_TRIG_FLOOR;
      } else if (cond != GSE_TRIG_NONE) {
        stop = kSwitch;
        trig = cond;
      }
    }
    if (stop == kRun && j >= S->max_iter) stop = kCap;
    S->stop = stop;
    S->trig = trig;
  }
}

// CG direction after a residual replacement at a switch: restart p = r
// (mode 0), keep p (mode 1), or keep it only while the replacement leaves
// the residual norm within a factor of two (mode 2; rho = r.r before and
// after).  A kept direction serves when the operators differ by little at
// the residual's scale; after a large jump (the tolerance escalation, a warm
// start) it can stall CG.
__host__ __device__ inline bool restart_direction(int mode, double rho_old, double rho_new) {
  return mode == 0 || (mode == 2 && (rho_new > 4.0 * rho_old || 4.0 * rho_new < rho_old));
}

// ------------------------------------------------------------- streams --
// A non-blocking stream of this thread on the current device: solves run on
// it (it can be captured into a HIP graph, the legacy null stream cannot)
// after waiting for the caller's stream.
struct SolveStream {
  hipStream_t caller;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  hipError_t err = hipSuccess;
  explicit SolveStream(hipStream_t c) : caller(c) {
    thread_local hipStream_t cache[16] = {};
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return;
    if (dev < 0 || dev >= 16) {
      err = hipErrorInvalidDevice;
      return;
    }
    if (!cache[dev]) {
      err = hipStreamCreateWithFlags(&cache[dev], hipStreamNonBlocking);
      if (err != hipSuccess) return;
    }
    s = cache[dev];
    err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(ev, caller);
    if (err == hipSuccess) err = hipStreamWaitEvent(s, ev, 0);
  }
  ~SolveStream() {
    if (ev) {
      if (s && hipEventRecord(ev, s) == hipSuccess) (void)hipStreamWaitEvent(caller, ev, 0);
      (void)hipEventDestroy(ev);
    }
  }
};

template <typename F>
hipError_t capture(hipStream_t st, hipGraphExec_t* out, F&& body) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t eb = body();
  e = hipStreamEndCapture(st, &graph);
  if (eb != hipSuccess) e = eb;
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

}  // namespace gse
