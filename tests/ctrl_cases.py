"""Solver cases in which the stepped controller makes each of its decisions
(Conditions 1-3 of Section III-D on a short check grid, the tolerance
escalation, a warm start that already meets the tolerance on an inexact
operator, fixed segment counts), shared by the GPU parity tests and the CPU
test that checks the oracle takes every decision with a margin (so that the
rounding differences between the two sides cannot flip one).

Each case: a matrix builder, the method, the restart length, the controller
parameters (oracle names, also the gse_params field names) and the x0 rule.
"""
from __future__ import annotations

import numpy as np

import oracle as O
from workloads import convdiff2d, diffusion2d, diffusion3d, rhs_from_solution

# A short check grid: l = 20, t = m = 10 (Section III-D's schedule, scaled
# down so that the Conditions are evaluated within a few dozen iterations).
SHORT = dict(l=20, t=10, m=10)

CASES = {
    # CG above 4096 rows: the multi-launch path.  rsd_limit 0.15 and
    # ndec_limit 10 make Condition 1 fire at j = 60; the t/2 rule instead
    # reads nDec = 9 as "not below" and Condition 2 fires at the same j.
    "cg_multi_c1": dict(A=lambda: diffusion3d(24, 3), method="cg", seed=3,
                        ctrl=dict(SHORT, ndec_limit=10, rsd_limit=0.15, floor_c=0.0)),
    "cg_multi_rule_t_half": dict(A=lambda: diffusion3d(24, 3), method="cg", seed=3,
                                 ctrl=dict(SHORT, ndec_limit=10, rsd_limit=0.15, ndec_rule=1,
                                           floor_c=0.0)),
    # one-workgroup CG (at most 4096 rows) with the t/2 rule
    "cg_small_rule_t_half": dict(A=lambda: diffusion2d(40, 5), method="cg", seed=5,
                                 ctrl=dict(SHORT, ndec_limit=10, rsd_limit=0.15, ndec_rule=1,
                                           floor_c=0.0)),
    # the paper's check grid with no floor trigger: each switch is the
    # tolerance escalation (the A_s residual meets 1e-10 on an inexact A_s)
    "cg_multi_tol_chain": dict(A=lambda: diffusion3d(24, 5), method="cg", seed=5,
                               ctrl=dict(floor_c=0.0)),
    # GMRES(10): Condition 2 on the check grid (at a cycle end)
    "gmres_c2": dict(A=lambda: convdiff2d(48, 2), method="gmres", seed=3, restart=10,
                     ctrl=dict(SHORT, ndec_limit=6, reldec_limit=0.5, floor_c=0.0)),
    "gmres_c2_4096": dict(A=lambda: convdiff2d(64, 4), method="gmres", seed=3, restart=10,
                          ctrl=dict(SHORT, ndec_limit=6, reldec_limit=0.5, floor_c=0.0)),
    "gmres_tol_chain": dict(A=lambda: convdiff2d(48, 2), method="gmres", seed=3, restart=30,
                            ctrl=dict(floor_c=0.0)),
    # warm starts at the solution of the head-only system: the tolerance is
    # met at iteration 0 on an inexact operator, which escalates
    "cg_multi_warm": dict(A=lambda: diffusion3d(24, 3), method="cg", seed=3, ctrl={},
                          x0="head_solution"),
    "cg_small_warm": dict(A=lambda: diffusion2d(40, 5), method="cg", seed=5, ctrl={},
                          x0="head_solution"),
    "gmres_warm": dict(A=lambda: convdiff2d(48, 2), method="gmres", seed=3, restart=30,
                       ctrl={}, x0="head_solution"),
    # a fixed count of two segments (no escalation; converged only if the
    # all-segment residual meets the tolerance)
    "cg_fixed2": dict(A=lambda: diffusion3d(12, 4), method="cg", seed=4, ctrl={}, fixed=2),
    "gmres_fixed2": dict(A=lambda: convdiff2d(32, 5), method="gmres", seed=5, restart=30, ctrl={},
                         fixed=2),
}

# Batched / served systems of uneven sizes (1000 .. 8000 rows) on the short
# grid: Conditions 2 and the tolerance escalation fire among them.
BATCH_CTRL = dict(SHORT, ndec_limit=6, floor_c=0.0)
BATCH_SYSTEMS = [("d3d10", lambda: diffusion3d(10, 1), 7), ("d3d14", lambda: diffusion3d(14, 2), 7),
                 ("d2d70", lambda: diffusion2d(70, 5), 7), ("d3d20", lambda: diffusion3d(20, 6), 7)]


def max_iter_of(case) -> int:
    return 15000 if case["method"] == "gmres" else 5000


def oracle_params(case, switch_mode: int = 0):
    preset = "paper_gmres" if case["method"] == "gmres" else "paper_cg"
    return O.make_params(tol=1e-10, max_iter=max_iter_of(case), restart=case.get("restart", 30),
                         fixed_segments=case.get("fixed", 0), preset=preset,
                         switch_mode=switch_mode,
                         orth=2 if case["method"] == "gmres" and case.get("restart", 30) <= 32
                         else 1, **case["ctrl"])


def head_solution(A, enc, b):
    """Solution of A_1 x = b (the head-only operator), by a direct solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    A1 = sp.csr_matrix((O.decode(enc, 1), A.indices, A.indptr), shape=(A.n_rows, A.n_cols))
    return spl.spsolve(A1.tocsc(), b)


def build(case):
    """(A, b, enc, x0) of a case."""
    A = case["A"]()
    _, b = rhs_from_solution(A, case["seed"])
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    x0 = head_solution(A, enc, b) if case.get("x0") == "head_solution" else None
    return A, b, enc, x0


def run_oracle(case, A, b, enc, x0, switch_mode: int = 0):
    fn = O.gmres if case["method"] == "gmres" else O.cg
    return fn(A.indptr, b, oracle_params(case, switch_mode), A.indices, A.data, enc, x0=x0)


def decision_margin(hist, prm, upto: int) -> float:
    """Smallest relative distance of a decision input from its threshold at
    the iterations up to `upto`: the window metrics at every check (RSD vs
    rsd_limit, relDec vs reldec_limit, every nDec comparison of neighbouring
    residuals), and the residual against tol and floor_c * eta thresholds is
    checked by the caller."""
    worst = np.inf
    l, t, m = prm.l, prm.t, prm.m
    for j in range(max(l, t), upto + 1):
        if m <= 0 or (j - l) % m:
            continue
        rsd, _, rd = O.window_metrics(hist, j, t)
        worst = min(worst, abs(rsd - prm.rsd_limit) / prm.rsd_limit,
                    abs(rd - prm.reldec_limit) / prm.reldec_limit)
        w = hist[j - t:j + 1]
        gaps = np.abs(np.diff(w)) / np.maximum(w[:-1], 1e-300)
        worst = min(worst, float(gaps.min()))
    return worst


def tol_margin(hist, tol: float) -> float:
    """Smallest relative distance of a recorded residual from the tolerance."""
    h = np.asarray(hist, dtype=np.float64)
    h = h[np.isfinite(h) & (h > 0)]
    return float(np.min(np.abs(h - tol) / tol)) if h.size else np.inf


def replay_cg_decisions(hist, seg, iters: int, eta, prm, fixed: int = 0):
    """The stepped controller's decisions (Section III-D with the floor and
    tolerance additions, as the oracle's CG takes them) replayed on a
    recorded CG residual history: after iteration j (and at j = 0 for the
    starting residual), with s the segment count that produced hist[j],
      relres <= tol on an inexact operator     -> tolerance escalation (5);
      else, stepped, s < 3 and j >= 1:
        relres <= floor_c * eta_s              -> floor trigger (4);
        Conditions 1-3 on the check grid       -> 1, 2 or 3.
    Returns [(j, trigger), ...].  The recorded segment history must step up
    exactly after each replayed switch (checked here), so a switch the
    recorder made without cause, or a missed one, both show."""
    out = []
    s = int(seg[0])
    tol = prm.tol
    for j in range(iters + 1):
        r = float(hist[j])
        exact = fixed != 0 or s >= 3 or eta[s - 1] == 0.0
        trig = 0
        if r <= tol:
            if not exact:
                trig = 5
        elif j >= 1 and fixed == 0 and s < 3:
            e = eta[s - 1]
            if prm.floor_c > 0.0 and e > 0.0 and r <= prm.floor_c * e:
                trig = 4
            else:
                trig = O.precision_trigger(hist, j, prm)
        if trig:
            out.append((j, trig))
            s += 1
        if j < iters:
            assert int(seg[j + 1]) == s, ("segment history disagrees with the decisions", j, s,
                                          int(seg[j + 1]))
    return out
