"""Pins of the oracle's switch points: the floor trigger, the tolerance
escalation and the residual replacement at a switch (the additions to the
stepped scheme of Section III-D that reach a 1e-10 tolerance).

The system is hand-built so that every quantity has a closed form:
A = diag(a, 3) with a = 1 + 2^-20, b = (1, 1), and a reused one-slot table
holding the shared exponent 1025 (biased exponent 1024 + 1, Section III-B.2).
3 = 1.5 * 2^1 has that exponent (minDiff 1); a has exponent 1023 (minDiff 2),
so its head keeps 13 significant bits and reads as exactly 1 with one
segment, and as a with two.  Hence A_1 = diag(1, 3), A_2 = A_3 = A,
eta_1 = ||A - A_1||_inf / ||A||_inf = 2^-20 / 3 and eta_2 = eta_3 = 0.

CG on A_1 from x0 = 0 (derived by hand): r0 = p0 = (1, 1), q = (1, 3),
alpha = 2/4, x1 = (1/2, 1/2), r1 = (1/2, -1/2), relres_1 = 1/2.  Then
beta = 1/4, p1 = (3/4, -1/4), q = (3/4, -3/4), alpha = (1/2)/(3/4) = 2/3 and
r2 = r1 - alpha q = 0: A_1 has two distinct eigenvalues.

GMRES on A_1 from x0 = 0: the first step minimises ||b - alpha A_1 b|| at
alpha = (b.A_1 b)/(A_1 b.A_1 b) = 4/10, leaving (3/5, -1/5), relres_1 =
sqrt(2/5)/sqrt(2) = sqrt(1/5).
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import CSR

A_VAL = 1.0 + 2.0**-20
SEM_ONE_SLOT = [1025]


def diag_system(copies=1):
    """`copies` diagonal blocks diag(a, 3); CG and GMRES on it behave as on
    one block (every dot is `copies` times the block's)."""
    d = np.tile([A_VAL, 3.0], copies)
    return CSR.from_scipy(sp.csr_matrix(sp.diags(d))), np.ones(2 * copies)


def encoded(A):
    return O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=1, sem_in=SEM_ONE_SLOT)


def test_hand_system_encoding():
    A, _ = diag_system()
    enc = encoded(A)
    assert list(O.decode(enc, 1)) == [1.0, 3.0]
    assert list(O.decode(enc, 2)) == [A_VAL, 3.0]
    assert list(O.decode(enc, 3)) == [A_VAL, 3.0]
    # eta_1 = 2^-20 / 3 (the FP64 quotient of the two row sums' maximum)
    assert enc.eta[0] == 2.0**-20 / 3.0 and enc.eta[1] == 0.0 and enc.eta[2] == 0.0


def _replacement_step(x1):
    """relres after one CG step on A from x1 with p = r = b - A x1 (exact
    rationals): alpha = r.r / r.Ar, r' = r - alpha A r."""
    a = Fr(A_VAL)
    r = [Fr(1) - a * Fr(x1[0]), Fr(1) - 3 * Fr(x1[1])]
    Ar = [a * r[0], 3 * r[1]]
    alpha = (r[0] ** 2 + r[1] ** 2) / (r[0] * Ar[0] + r[1] * Ar[1])
    r2 = [r[0] - alpha * Ar[0], r[1] - alpha * Ar[1]]
    return math.sqrt(float(r2[0] ** 2 + r2[1] ** 2)) / math.sqrt(2.0), r


@pytest.mark.parametrize("copies", [1, 3])
def test_floor_trigger_fires_at_the_closed_form_iteration(copies):
    """floor_c * eta_1 = 2^21 * 2^-20 / 3 = 2/3 >= relres_1 = 1/2 > tol: the
    floor trigger fires after iteration 1, and not before (relres_0 = 1).
    The switch replaces the residual with b - A_2 x1 = (1/2 - 2^-21, -1/2);
    the next iteration's residual follows from it in closed form (with the
    head-only residual (1/2, -1/2) instead it would be 0)."""
    A, b = diag_system(copies)
    enc = encoded(A)
    p = O.make_params(tol=1e-10, max_iter=50, floor_c=2.0**21, switch_mode=0)
    r = O.cg(A.indptr, b, p, A.indices, A.data, enc)
    assert r.status == O.OK
    assert r.switch_iter == (1, -1) and O.TRIG_NAMES[r.switch_trigger[0]] == "floor"
    assert r.iters_per_seg == (1, 2, 0) and r.iters == 3
    assert r.hist[0] == 1.0 and abs(r.hist[1] - 0.5) <= 2e-16
    want, r_repl = _replacement_step([0.5, 0.5])
    assert r_repl == [Fr(1, 2) - Fr(1, 2**21), Fr(-1, 2)]
    assert abs(r.hist[2] - want) <= 1e-15 * want
    assert r.hist[3] <= 1e-10
    assert np.allclose(r.x, np.tile([1.0 / A_VAL, 1.0 / 3.0], copies), rtol=1e-14, atol=0)


def test_floor_threshold_is_inclusive_below_and_silent_above():
    """floor_c = 2^20 puts floor_c * eta_1 = 1/3 below relres_1 = 1/2: no
    floor switch after iteration 1; iteration 2 then reaches r2 = 0 on A_1,
    the tolerance is met with an inexact operator and the solver escalates
    (trigger TOL at iteration 2) instead of stopping."""
    A, b = diag_system()
    enc = encoded(A)
    p = O.make_params(tol=1e-10, max_iter=50, floor_c=2.0**20, switch_mode=0)
    r = O.cg(A.indptr, b, p, A.indices, A.data, enc)
    assert r.status == O.OK
    assert r.switch_iter == (2, -1) and O.TRIG_NAMES[r.switch_trigger[0]] == "tol"
    assert r.hist[2] <= 1e-16
    # after the switch: r = b - A x2 with x2 = (1, 1/3), i.e. (-2^-20, ~0),
    # an eigenvector of A: one more iteration (at s = 2) solves the system
    assert r.iters_per_seg == (2, 1, 0)
    assert r.relres_true <= 1e-15


def test_floor_off_reaches_the_same_escalation():
    A, b = diag_system()
    enc = encoded(A)
    r = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=50, floor_c=0.0, switch_mode=0),
             A.indices, A.data, enc)
    assert r.switch_iter == (2, -1) and O.TRIG_NAMES[r.switch_trigger[0]] == "tol"


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_warm_start_solving_the_head_only_system_escalates(solver):
    """x0 = (1, 1/3) solves A_1 x = b to rounding, so the residual with one
    segment meets the tolerance before any iteration, but A_1 is inexact:
    the solver switches at iteration 0 (TOL) and converges with two
    segments, whose residual at x0 is (1 - a, 0) = (-2^-20, 0)."""
    A, b = diag_system()
    enc = encoded(A)
    x0 = np.array([1.0, 1.0 / 3.0])
    fn = O.cg if solver == "cg" else O.gmres
    p = O.make_params(tol=1e-10, max_iter=50, floor_c=10.0, switch_mode=0,
                      preset="paper_cg" if solver == "cg" else "paper_gmres")
    r = fn(A.indptr, b, p, A.indices, A.data, enc, x0=x0)
    assert r.status == O.OK
    assert r.switch_iter[0] == 0 and O.TRIG_NAMES[r.switch_trigger[0]] == "tol"
    assert r.iters_per_seg[0] == 0 and r.iters >= 1
    assert np.allclose(r.x, [1.0 / A_VAL, 1.0 / 3.0], rtol=1e-14, atol=0)


def test_gmres_floor_trigger_closed_form():
    """GMRES: relres_1 = sqrt(1/5) ~ 0.447 <= 2/3 fires the floor trigger
    after step 1; the cycle ends with x1 = (2/5)(1, 1) and the next cycle
    starts from b - A_2 x1 = (1 - 2a/5, -1/5).  Its first step's residual is
    the one-dimensional least-squares minimum, in closed form."""
    A, b = diag_system()
    enc = encoded(A)
    p = O.make_params(tol=1e-10, max_iter=60, floor_c=2.0**21, preset="paper_gmres")
    r = O.gmres(A.indptr, b, p, A.indices, A.data, enc)
    assert r.status == O.OK
    assert r.switch_iter == (1, -1) and O.TRIG_NAMES[r.switch_trigger[0]] == "floor"
    assert abs(r.hist[1] - math.sqrt(0.2)) <= 2e-16
    a = Fr(A_VAL)
    x1 = Fr(2, 5)
    rr = [1 - a * x1, 1 - 3 * x1]
    Ar = [a * rr[0], 3 * rr[1]]
    rr2 = rr[0] ** 2 + rr[1] ** 2
    rAr = rr[0] * Ar[0] + rr[1] * Ar[1]
    Ar2 = Ar[0] ** 2 + Ar[1] ** 2
    want = math.sqrt(float(rr2 - rAr * rAr / Ar2)) / math.sqrt(2.0)
    assert abs(r.hist[2] - want) <= 1e-14 * want
    assert r.iters_per_seg[0] == 1 and r.iters_per_seg[2] == 0
