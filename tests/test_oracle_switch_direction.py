"""Pins of the CG direction after a switch (reading R7): restart p = r
(switch_mode 0), keep p (1), or keep it only while the residual replacement
r = b - A_{s+1} x leaves ||r|| within a factor of two (2, the default).

The replacement changes r by about ||(A_{s+1} - A_s) x||; at a floor switch
(relres ~ 10 eta_s) that is ~10 % of ||r||, and a kept direction stays
nearly conjugate; after a tolerance escalation or a warm start the
recursive residual of the old operator is far below the new operator's
true one (a factor 1e5 .. 1e10 here), and a kept direction stalls CG into a
breakdown.  Checked on the oracle: mode 2 takes mode 0's path where the
replacement jumps and mode 1's where it does not."""
import numpy as np
import pytest

import oracle as O
from ctrl_cases import CASES, build
from workloads import diffusion3d, rhs_from_solution


def solve(case_or_matrix, mode):
    if isinstance(case_or_matrix, str):
        c = CASES[case_or_matrix]
        A, b, enc, x0 = build(c)
        ctrl = c["ctrl"]
    else:
        A, seed = case_or_matrix
        _, b = rhs_from_solution(A, seed)
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        x0, ctrl = None, {}
    prm = O.make_params(tol=1e-10, max_iter=20000, switch_mode=mode, orth=1, **ctrl)
    return O.cg(A.indptr, b, prm, A.indices, A.data, enc, x0=x0)


@pytest.mark.parametrize("name", ["cg_multi_tol_chain", "cg_multi_warm"])
def test_kept_direction_stalls_after_a_jump_and_mode_2_restarts(name):
    r0, r1, r2 = (solve(name, m) for m in (0, 1, 2))
    assert r1.status == O.ERR_BREAKDOWN and r1.iters > 10 * r0.iters
    assert r0.status == r2.status == O.OK
    assert r2.switch_iter[0] == r0.switch_iter[0]
    assert r2.iters <= r0.iters


@pytest.mark.parametrize("seed", [0, 1])
def test_mode_2_keeps_the_direction_at_floor_switches(seed):
    """Floor switches move ||r|| by ~0.5 %: mode 2 is mode 1 bit for bit."""
    A = diffusion3d(24, seed)
    r1, r2 = solve((A, seed), 1), solve((A, seed), 2)
    assert r2.status == r1.status == O.OK
    assert r2.iters == r1.iters and np.array_equal(r2.x, r1.x)
    assert all(t == 4 for t in r2.switch_trigger)


def test_default_is_mode_2():
    assert O.make_params().switch_mode == 2
