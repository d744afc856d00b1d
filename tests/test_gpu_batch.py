"""GPU parity of the batched stepped CG (gse_batch_cg) against the oracle,
and the batch invariants: a system gives the same bits alone as in a mix,
and replayed epochs give the same bits as direct launches.

As for the single-system solver, several iterates are correct: every system
must reach a true relative residual <= 1e-10 (recomputed here in FP64 on
the host), its solution must agree with the oracle's within 1e-6, and its
iteration count within 10 % (stepped controller per system on both sides).
"""
import numpy as np
import pytest

import oracle as O
from workloads import CSR, diffusion2d, diffusion3d, poisson2d, rhs_from_solution

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


class Sys:
    """One system on the device: its operator (GSE or FP64 CSR), b and x."""

    def __init__(self, A: CSR, seed: int, kind: str = "gse", b=None, x0=None):
        self.A = A
        self.x0 = x0
        self.kind = kind
        if b is None:
            _, b = rhs_from_solution(A, seed)
        self.b_host = b
        rp = torch.from_numpy(A.indptr).to(DEV)
        ci = torch.from_numpy(A.indices).to(DEV)
        va = torch.from_numpy(A.data).to(DEV)
        if kind == "gse":
            self.holder = G.GseMatrix(rp, ci, va, A.n_cols)
            self.rec = self.holder.A
        else:
            self.holder = G.CsrMatrix(rp, ci, va, A.n_cols)
            self.rec = self.holder.M
        self.b = torch.from_numpy(b).to(DEV)
        self.x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)

    def reset(self):
        if self.x0 is None:
            self.x.zero_()
        else:
            self.x.copy_(torch.from_numpy(self.x0))
        return (self.rec, self.b, self.x)


def batch_solve(systems, launch_mode=0, max_iter=5000):
    p = G.gse_default_params(G.CG)
    p.max_iter = max_iter
    p.launch_mode = launch_mode
    triples = [s.reset() for s in systems]
    ws = torch.empty(G.gse_batch_workspace(triples, p), dtype=torch.uint8, device=DEV)
    reps = G.gse_batch_cg(triples, p, ws)
    torch.cuda.synchronize()
    out = []
    for i, (s, r) in enumerate(zip(systems, reps)):
        hist, seg = G.gse_batch_history(ws, i, r.iters + 1)
        out.append((r, s.x.cpu().numpy(), hist, seg))
    return out


def oracle_solve(s: Sys):
    A = s.A
    if s.kind == "gse":
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", switch_mode=2, orth=1)
        return O.cg(A.indptr, s.b_host, prm, A.indices, A.data, enc)
    prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", fixed_segments=-1, orth=1)
    return O.cg(A.indptr, s.b_host, prm, A.indices, A.data)


def true_relres(A: CSR, x, b):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


def spd_dense(n, seed):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return CSR.from_scipy(sp.csr_matrix(M @ M.T + n * np.eye(n)))


def mix():
    return [Sys(diffusion3d(10, 1), 1), Sys(diffusion3d(14, 2), 2), Sys(poisson2d(30), 3),
            Sys(diffusion3d(9, 4), 4, kind="csr"), Sys(spd_dense(12, 5), 5),
            Sys(diffusion3d(20, 6), 6)]


def test_batch_matches_oracle():
    systems = mix()
    res = batch_solve(systems)
    for s, (r, x, hist, seg) in zip(systems, res):
        ref = oracle_solve(s)
        assert r.status == G.OK and ref.status == O.OK, (s.A.name, r.as_dict())
        assert r.relres_true <= 1e-10 and true_relres(s.A, x, s.b_host) <= 1e-10
        assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(r.iters - ref.iters) <= max(3, ref.iters // 10), (s.A.name, r.iters, ref.iters)
        assert hist[0] == pytest.approx(ref.hist[0], rel=1e-12)
        # the segment history steps by one and agrees with the report
        d = np.diff(seg[1:])
        assert np.all((d == 0) | (d == 1))
        if s.kind == "gse":
            assert [int((seg[1:] == k).sum()) for k in (1, 2, 3)] == list(r.iters_per_seg)


def test_batch_system_alone_equals_in_mix():
    systems = mix()
    in_mix = batch_solve(systems)
    for i in (0, 2, 3, 5):
        (r1, x1, h1, s1), = batch_solve([systems[i]])
        r0, x0, h0, s0 = in_mix[i]
        assert r1.status == r0.status == G.OK
        assert r1.iters == r0.iters and list(r1.iters_per_seg) == list(r0.iters_per_seg)
        assert list(r1.switch_iter) == list(r0.switch_iter)
        assert np.array_equal(x1, x0)
        assert np.array_equal(h1, h0) and np.array_equal(s1, s0)
    # and in another order, next to other systems
    reordered = [systems[5], systems[3], systems[0]]
    again = batch_solve(reordered)
    for k, i in enumerate((5, 3, 0)):
        assert np.array_equal(again[k][1], in_mix[i][1])


def test_batch_graph_replay_equals_direct_launches():
    systems = mix()[:3]
    direct = batch_solve(systems, launch_mode=1)
    for _ in range(2):
        junk = torch.randn(1 << 20, device=DEV).sum()  # unrelated eager work
        graph = batch_solve(systems, launch_mode=0)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for (rd, xd, hd, _), (rg, xg, hg, _) in zip(direct, graph):
            assert rd.iters == rg.iters and np.array_equal(xd, xg) and np.array_equal(hd, hg)


def test_batch_edge_cases():
    import scipy.sparse as sp
    zero_b = Sys(poisson2d(8), 0, b=np.zeros(64), x0=np.ones(64))
    one = Sys(CSR.from_scipy(sp.csr_matrix(np.array([[4.0]]))), 0, b=np.array([2.0]))
    indef = Sys(CSR.from_scipy(sp.csr_matrix(np.diag([1.0, -1.0, 2.0]))), 0, kind="csr",
                b=np.ones(3))
    normal = Sys(diffusion3d(8, 7), 7)
    res = batch_solve([zero_b, one, indef, normal])
    (rz, xz, _, _), (r1, x1, _, _), (ri, _, _, _), (rn, xn, _, _) = res
    assert rz.status == G.OK and np.all(xz == 0)
    assert r1.status == G.OK and x1[0] == pytest.approx(0.5, rel=1e-15)
    assert ri.status == G.ERR_BREAKDOWN
    assert rn.status == G.OK and true_relres(normal.A, xn, normal.b_host) <= 1e-10
    # a breakdown beside it leaves the other system's iterates untouched
    (ra, xa, _, _), = batch_solve([normal])
    assert ra.iters == rn.iters and np.array_equal(xa, xn)


def test_batch_argument_errors():
    s = Sys(poisson2d(8), 0)
    p = G.gse_default_params(G.CG)
    ws = torch.empty(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(G.GseError) as ei:
        G.gse_batch_cg([s.reset()], p, ws)
    assert ei.value.status == G.ERR_NOMEM
    with pytest.raises(G.GseError) as ei:
        G.gse_batch_workspace([], p)
    assert ei.value.status == G.ERR_ARG


def test_large_systems_run_their_product_on_the_ring():
    """Systems of at least 2^16 rows of short rows take their product from
    the single-system row-tile ring (grouped launches) while the others stay
    on the batched tile kernel: both against the oracle, each alone equal to
    the mix bit for bit, stepped GSE and FP64 CSR."""
    systems = [Sys(diffusion3d(64, 7), 7), Sys(diffusion3d(65, 8), 8, kind="csr"),
               Sys(diffusion3d(12, 9), 9), Sys(poisson2d(30), 10)]
    assert systems[0].A.n_rows >= 1 << 18 and systems[1].A.n_rows >= 1 << 18
    res = batch_solve(systems)
    for s, (r, x, hist, seg) in zip(systems, res):
        ref = oracle_solve(s)
        assert r.status == G.OK and ref.status == O.OK, (s.A.name, r.as_dict())
        assert r.relres_true <= 1e-10 and true_relres(s.A, x, s.b_host) <= 1e-10
        assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(r.iters - ref.iters) <= max(3, ref.iters // 10), (s.A.name, r.iters, ref.iters)
    for i in (0, 1, 3):
        (r1, x1, h1, s1), = batch_solve([systems[i]])
        r, x, hist, seg = res[i]
        assert r1.iters == r.iters and list(r1.iters_per_seg) == list(r.iters_per_seg)
        assert np.array_equal(x1, x) and np.array_equal(h1, hist)


def test_medium_systems_share_grouped_ring_launches():
    """Systems just above 2^16 rows in three ring instances -- two 3-D
    stencils (rows of 7) and a 2-D one (rows of 5) stepped in GSE-SEM, so
    each instance holds one or more systems as they step through the
    segment counts, and a 3-D FP64 CSR one -- beside a small system on the
    batched tile kernel: every result against the oracle's CG, and each
    system alone equal to the mix bit for bit (its grid and partials are
    those of its own plain launch whatever the group holds)."""
    systems = [Sys(diffusion3d(41, 11), 11), Sys(diffusion3d(42, 12), 12),
               Sys(diffusion2d(262, 13, decades=1.0), 13), Sys(diffusion3d(41, 14), 14, kind="csr"),
               Sys(diffusion3d(10, 1), 1)]
    assert all(s.A.n_rows >= 1 << 16 for s in systems[:4]) and systems[4].A.n_rows < 1 << 16
    res = batch_solve(systems)
    for s, (r, x, hist, seg) in zip(systems, res):
        ref = oracle_solve(s)
        assert r.status == G.OK and ref.status == O.OK, (s.A.name, r.as_dict())
        assert r.relres_true <= 1e-10 and true_relres(s.A, x, s.b_host) <= 1e-10
        assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(r.iters - ref.iters) <= max(3, ref.iters // 10), (s.A.name, r.iters, ref.iters)
    for i in range(5):
        (r1, x1, h1, s1), = batch_solve([systems[i]])
        r, x, hist, seg = res[i]
        assert r1.iters == r.iters and list(r1.iters_per_seg) == list(r.iters_per_seg)
        assert np.array_equal(x1, x) and np.array_equal(h1, hist)
