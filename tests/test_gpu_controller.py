"""GPU parity of the stepped controller's decisions against the oracle, on
every path that runs it: multi-launch CG (above 4096 rows), the
one-workgroup CG loop, GMRES, the batched CG engine and the server.

The cases (tests/ctrl_cases.py) make Conditions 1-3 fire on a short check
grid, escalate on the tolerance, start warm at a point that already meets
the tolerance on the inexact head-only operator, and run with two fixed
segments.  Parity is held at three levels:
  * decisions: the oracle's controller replayed on the GPU's recorded
    residual history reproduces every switch the GPU made (iteration and
    trigger) and no other -- same inputs, same decisions;
  * trajectories: where both residual histories still agree (switches in
    the first 40 iterations, and every GMRES case, whose estimates stay
    within rounding of the oracle's), the GPU switches at the oracle's
    iterations for the oracle's reasons;
  * results: same status, solution within 1e-6 of the oracle's, iteration
    count within 10 %.
CG on these variable-coefficient operators amplifies summation-order
rounding: two runs that differ only in the order of their dot products
drift apart by 1e-2 in relres within ~50 iterations (measured; a 1e-16
perturbation of b moves the oracle's own switch by one or two iterations),
so later CG switch points are checked by the replay, not by equality.
"""
import time

import numpy as np
import pytest

import oracle as O
from ctrl_cases import (BATCH_CTRL, BATCH_SYSTEMS, CASES, build, head_solution, max_iter_of,
                        oracle_params, replay_cg_decisions, run_oracle)
from workloads import rhs_from_solution

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def gpu_params(case, launch_mode=0):
    method = G.GMRES if case["method"] == "gmres" else G.CG
    p = G.gse_default_params(method)
    p.max_iter = max_iter_of(case)
    p.restart = case.get("restart", 30)
    p.fixed_segments = case.get("fixed", 0)
    p.switch_mode = 0
    p.launch_mode = launch_mode
    for k, v in case["ctrl"].items():
        setattr(p, k, v)
    return method, p


def gpu_solve(case, A, b, x0, launch_mode=0):
    method, p = gpu_params(case, launch_mode)
    rp = torch.from_numpy(A.indptr).to(DEV)
    ci = torch.from_numpy(A.indices).to(DEV)
    va = torch.from_numpy(A.data).to(DEV)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV) if x0 is None else \
        torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
    fn = G.gse_gmres if method == G.GMRES else G.gse_cg
    rep = fn(M.A, torch.from_numpy(b).to(DEV), x, p, ws)
    torch.cuda.synchronize()
    hist, seg = G.gse_solve_history(ws, rep.iters + 1)
    return rep, x.cpu().numpy(), hist, seg, list(M.eta)


def true_relres(A, x, b):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


EARLY = 40  # switch points up to here: histories still agree to ~1e-9


def switches(rep):
    return [(int(j), int(t)) for j, t in zip(rep.switch_iter, rep.switch_trigger) if j >= 0]


def assert_decisions(rep, hist, seg, eta, prm, fixed, what):
    """The oracle's controller on the GPU's own history makes the GPU's switches."""
    replayed = replay_cg_decisions(hist, seg, rep.iters, eta, prm, fixed)
    assert replayed[:2] == switches(rep), (what, replayed, switches(rep))


def assert_results(rep, x, ref, A, b, what, exact_trajectory):
    info = (what, rep.as_dict(), ref.switch_iter, ref.switch_trigger, ref.iters)
    assert rep.status == ref.status, info
    mine, theirs = switches(rep), [(int(j), int(t)) for j, t in
                                   zip(ref.switch_iter, ref.switch_trigger) if j >= 0]
    if exact_trajectory:
        assert mine == theirs, info
    else:  # the switches inside the window where both histories agree
        assert [m for m in mine if m[0] <= EARLY] == [t for t in theirs if t[0] <= EARLY], info
        assert len(mine) == len(theirs), info
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10), info
    if ref.status == O.OK:
        assert rep.relres_true <= 1e-10 and true_relres(A, x, b) <= 1e-10, info
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x), info


@pytest.mark.parametrize("name", list(CASES))
def test_single_system_decisions_match_oracle(name):
    case = CASES[name]
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0)
    rep, x, hist, seg, eta = gpu_solve(case, A, b, x0)
    if case["method"] == "cg":
        assert_decisions(rep, hist, seg, eta, oracle_params(case), case.get("fixed", 0), name)
    assert_results(rep, x, ref, A, b, name, exact_trajectory=case["method"] == "gmres")


@pytest.mark.parametrize("name", ["cg_multi_warm", "cg_small_warm", "cg_multi_tol_chain"])
def test_adaptive_direction_matches_oracle(name):
    """switch_mode 2 (the default): after the warm start's or the tolerance
    escalation's large replacement the direction restarts, at floor
    switches it is kept -- on the GPU as in the oracle."""
    case = dict(CASES[name])
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0, switch_mode=2)
    method, p = gpu_params(case)
    p.switch_mode = 2
    rp = torch.from_numpy(A.indptr).to(DEV)
    ci = torch.from_numpy(A.indices).to(DEV)
    va = torch.from_numpy(A.data).to(DEV)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV) if x0 is None else \
        torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
    rep = G.gse_cg(M.A, torch.from_numpy(b).to(DEV), x, p, ws)
    torch.cuda.synchronize()
    hist, seg = G.gse_solve_history(ws, rep.iters + 1)
    assert_decisions(rep, hist, seg, list(M.eta), oracle_params(case), 0, name)
    assert_results(rep, x.cpu().numpy(), ref, A, b, name, exact_trajectory=False)


@pytest.mark.parametrize("name", ["cg_multi_c1", "cg_multi_warm", "gmres_c2"])
def test_direct_launches_take_the_same_decisions(name):
    case = CASES[name]
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0)
    rep, x, hist, seg, eta = gpu_solve(case, A, b, x0, launch_mode=1)
    if case["method"] == "cg":
        assert_decisions(rep, hist, seg, eta, oracle_params(case), 0, name)
    assert_results(rep, x, ref, A, b, name, exact_trajectory=case["method"] == "gmres")


def _batch_systems(warm=False):
    out = []
    for name, mk, seed in BATCH_SYSTEMS:
        A = mk()
        _, b = rhs_from_solution(A, seed)
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        x0 = head_solution(A, enc, b) if warm else None
        out.append((name, A, b, enc, x0))
    return out


def _batch_params(ctrl):
    ctrl = dict(ctrl)
    mode = ctrl.pop("switch_mode", 0)
    return O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", switch_mode=mode, orth=1,
                         **ctrl)


def _batch_oracle(A, b, enc, x0, ctrl):
    return O.cg(A.indptr, b, _batch_params(ctrl), A.indices, A.data, enc, x0=x0)


@pytest.mark.parametrize("mode", [0, 2], ids=["restart", "adaptive"])
@pytest.mark.parametrize("warm", [False, True], ids=["short_grid", "warm_start"])
def test_batch_decisions_match_oracle(warm, mode):
    ctrl = {} if warm else BATCH_CTRL
    systems = _batch_systems(warm)
    p = G.gse_default_params(G.CG)
    p.max_iter = 5000
    p.switch_mode = mode
    for k, v in ctrl.items():
        setattr(p, k, v)
    keep, triples = [], []
    for name, A, b, enc, x0 in systems:
        rp = torch.from_numpy(A.indptr).to(DEV)
        ci = torch.from_numpy(A.indices).to(DEV)
        va = torch.from_numpy(A.data).to(DEV)
        M = G.GseMatrix(rp, ci, va, A.n_cols)
        bd = torch.from_numpy(b).to(DEV)
        xd = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV) if x0 is None else \
            torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
        keep.append((M, bd, xd))
        triples.append((M.A, bd, xd))
    ws = torch.empty(G.gse_batch_workspace(triples, p), dtype=torch.uint8, device=DEV)
    reps = G.gse_batch_cg(triples, p, ws)
    torch.cuda.synchronize()
    for i, ((name, A, b, enc, x0), rep, (M, _, xd)) in enumerate(zip(systems, reps, keep)):
        hist, seg = G.gse_batch_history(ws, i, rep.iters + 1)
        assert_decisions(rep, hist, seg, list(M.eta), _batch_params(ctrl), 0, name)
        ref = _batch_oracle(A, b, enc, x0, dict(ctrl, switch_mode=mode))
        assert_results(rep, xd.cpu().numpy(), ref, A, b, name, exact_trajectory=False)


def test_served_requests_match_oracle():
    """Every request of a mixed stream, served with the short check grid,
    returns the oracle's status and solution, switches as often, and where
    the histories still agree, at the oracle's iterations for its reasons
    (the served iterates are the batch engine's, whose decisions the test
    above replays: a request gives the same bits alone and in the mix)."""
    p = G.gse_default_params(G.CG)
    p.max_iter = 5000
    p.switch_mode = 0
    for k, v in BATCH_CTRL.items():
        setattr(p, k, v)
    systems = _batch_systems()
    arena = torch.empty(256 << 20, dtype=torch.uint8, device=DEV)
    server = G.gse_solver_create(arena, 8)
    try:
        reqs, tickets = [], []
        for i, (name, A, b, enc, x0) in enumerate(systems):
            rq = G.Request(A, b, G.FMT_GSE, params=p)
            reqs.append(rq)
            tickets.append(G.gse_solver_submit(server, rq.rq))
            if i % 2:
                time.sleep(0.01)  # later arrivals join a running batch
        done = {}
        t0 = time.time()
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = G.gse_solver_poll(server, t)
                    if r is not None:
                        done[t] = r
            assert time.time() - t0 < 120.0, "server did not finish"
            time.sleep(0.002)
    finally:
        G.gse_solver_destroy(server)
    for (name, A, b, enc, x0), rq, t in zip(systems, reqs, tickets):
        ref = _batch_oracle(A, b, enc, None, BATCH_CTRL)
        assert_results(done[t], rq.x, ref, A, b, name, exact_trajectory=False)
