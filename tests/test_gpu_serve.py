"""GPU tests of the solver server (gse_solver_*): requests submitted over
time complete with the same bits as the batched solver gives each system
alone, and agree with the CPU oracle's CG on each request (status, solution
within 1e-6, iteration count within 10 %, as for the batched solver);
admission keeps the arena within its size; bad requests are refused on the
host."""
import time

import numpy as np
import pytest

import oracle as O
from workloads import diffusion2d, diffusion3d, poisson2d, rhs_from_solution

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def wait_all(server, tickets, timeout=120.0):
    reps = {}
    t0 = time.time()
    while len(reps) < len(tickets):
        for t in tickets:
            if t not in reps:
                r = G.gse_solver_poll(server, t)
                if r is not None:
                    reps[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return [reps[t] for t in tickets]


def batch_alone(A, b, fmt):
    """The same system through gse_batch_cg, alone."""
    rp = torch.from_numpy(A.indptr).to(DEV)
    ci = torch.from_numpy(A.indices).to(DEV)
    va = torch.from_numpy(A.data).to(DEV)
    holder = G.GseMatrix(rp, ci, va, A.n_cols) if fmt == G.FMT_GSE else \
        G.CsrMatrix(rp, ci, va, A.n_cols)
    rec = holder.A if fmt == G.FMT_GSE else holder.M
    bd = torch.from_numpy(b).to(DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    p = G.gse_default_params(G.CG)
    ws = torch.empty(G.gse_batch_workspace([(rec, bd, x)], p), dtype=torch.uint8, device=DEV)
    rep, = G.gse_batch_cg([(rec, bd, x)], p, ws)
    torch.cuda.synchronize()
    return rep, x.cpu().numpy()


def systems():
    out = []
    for k, (A, fmt) in enumerate([(diffusion3d(12, 11), G.FMT_GSE), (diffusion2d(40, 12), G.FMT_GSE),
                                  (poisson2d(20), G.FMT_GSE), (diffusion3d(10, 13), G.FMT_CSR64),
                                  (diffusion2d(64, 14), G.FMT_GSE), (diffusion3d(7, 15), G.FMT_GSE)]):
        _, b = rhs_from_solution(A, 20 + k)
        out.append((A, b, fmt))
    return out


def test_server_results_equal_batch_alone():
    arena = torch.empty(256 << 20, dtype=torch.uint8, device=DEV)
    server = G.gse_solver_create(arena, 8)
    try:
        reqs, tickets = [], []
        for i, (A, b, fmt) in enumerate(systems()):
            rq = G.Request(A, b, fmt)
            reqs.append(rq)
            tickets.append(G.gse_solver_submit(server, rq.rq))
            if i % 2:
                time.sleep(0.01)  # arrivals while others run
        reps = wait_all(server, tickets)
        st = G.gse_solver_stats(server)
        assert st.completed == len(reqs) and st.running == 0 and st.queued == 0
        assert st.arena_used == 0 and st.arena_peak <= st.arena_bytes
    finally:
        G.gse_solver_destroy(server)
    for (A, b, fmt), rq, rep in zip(systems(), reqs, reps):
        assert rep.status == G.OK, rep.as_dict()
        assert np.linalg.norm(b - A.to_scipy() @ rq.x) <= 1e-10 * np.linalg.norm(b)
        ref, xref = batch_alone(A, b, fmt)
        assert rep.iters == ref.iters and list(rep.iters_per_seg) == list(ref.iters_per_seg)
        assert np.array_equal(rq.x, xref)
        # and the CPU oracle's CG on the same request
        orc = oracle_cg(A, b, fmt)
        assert orc.status == O.OK
        assert np.linalg.norm(rq.x - orc.x) <= 1e-6 * np.linalg.norm(orc.x), A.name
        assert abs(rep.iters - orc.iters) <= max(3, orc.iters // 10), (A.name, rep.iters, orc.iters)
        if fmt == G.FMT_GSE:
            assert sum(rep.iters_per_seg) == rep.iters


def oracle_cg(A, b, fmt):
    """The oracle's CG with the server's defaults (stepped on the request's
    own table, or FP64 CSR)."""
    if fmt == G.FMT_GSE:
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg")
        return O.cg(A.indptr, b, prm, A.indices, A.data, enc)
    prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", fixed_segments=-1)
    return O.cg(A.indptr, b, prm, A.indices, A.data)


def test_server_admission_respects_the_arena():
    sysl = systems()
    A, b, fmt = sysl[4]
    one = G.Request(A, b, fmt)
    res, tr = G.gse_solver_footprint(one.rq)
    # room for the batch tables and two running requests, not three
    arena_bytes = 2 * res + tr + (256 << 10)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=DEV)
    server = G.gse_solver_create(arena, 4)
    try:
        reqs = [G.Request(A, b, fmt) for _ in range(6)]
        tickets = [G.gse_solver_submit(server, r.rq) for r in reqs]
        peak_running = 0
        t0 = time.time()
        done = {}
        while len(done) < len(tickets):
            s = G.gse_solver_stats(server)
            peak_running = max(peak_running, s.running)
            assert s.arena_used <= s.arena_bytes
            for t in tickets:
                if t not in done:
                    r = G.gse_solver_poll(server, t)
                    if r is not None:
                        done[t] = r
            assert time.time() - t0 < 120
            time.sleep(0.001)
        s = G.gse_solver_stats(server)
        assert s.arena_peak <= s.arena_bytes
        assert s.admitted == 6 and s.completed == 6
        assert peak_running <= 2  # the arena, not the 4 slots, bounds admission
    finally:
        G.gse_solver_destroy(server)
    xs = [r.x for r in reqs]
    for t, x in zip(tickets, xs):
        assert done[t].status == G.OK
        assert np.array_equal(x, xs[0])  # same system, same bits, whatever ran beside it


def test_server_rejects_bad_requests():
    arena = torch.empty(64 << 20, dtype=torch.uint8, device=DEV)
    server = G.gse_solver_create(arena, 2)
    try:
        A = poisson2d(8)
        b = np.ones(A.n_rows)
        bad = G.Request(A, b)
        bad.row_ptr[3] = bad.row_ptr[2] - 1  # decreasing row pointer
        with pytest.raises(G.GseError) as ei:
            G.gse_solver_submit(server, bad.rq)
        assert ei.value.status == G.ERR_ARG
        badc = G.Request(A, b)
        badc.col[5] = A.n_rows  # column out of range
        with pytest.raises(G.GseError) as ei:
            G.gse_solver_submit(server, badc.rq)
        assert ei.value.status == G.ERR_ARG
        big = diffusion3d(80, 0)
        big_rq = G.Request(big, np.ones(big.n_rows))  # kept alive while the server reads it
        with pytest.raises(G.GseError) as ei:
            G.gse_solver_submit(server, big_rq.rq)
        assert ei.value.status == G.ERR_NOMEM
        with pytest.raises(G.GseError) as ei:
            G.gse_solver_poll(server, 12345)
        assert ei.value.status == G.ERR_TICKET
        ok = G.Request(A, b)
        t = G.gse_solver_submit(server, ok.rq)
        rep, = wait_all(server, [t])
        assert rep.status == G.OK
    finally:
        G.gse_solver_destroy(server)
