"""The controller cases of the GPU parity tests, on the oracle alone: each
takes the decision it is there for, and takes it with a margin -- no window
metric within 1e-4 (relative) of its threshold at a check, no two
neighbouring residuals in a window within 1e-6 of each other, no recorded
residual within 1e-6 of the tolerance -- so that the few-ulp differences of
the GPU's reduction order cannot flip a decision and exact equality of the
switch points is a fair test."""
import numpy as np
import pytest

import oracle as O
from ctrl_cases import (BATCH_CTRL, BATCH_SYSTEMS, CASES, build, decision_margin, run_oracle,
                        tol_margin)
from workloads import rhs_from_solution

EXPECT = {
    "cg_multi_c1": (O.OK, (1, 2)),
    "cg_multi_rule_t_half": (O.OK, (2, 2)),
    "cg_small_rule_t_half": (O.OK, None),
    "cg_multi_tol_chain": (O.OK, (5, 5)),
    "gmres_c2": (O.OK, (2, 2)),
    "gmres_c2_4096": (O.OK, (2, 2)),
    "gmres_tol_chain": (O.OK, (5, 5)),
    "cg_multi_warm": (O.OK, None),
    "cg_small_warm": (O.OK, None),
    "gmres_warm": (O.OK, None),
    "cg_fixed2": (None, (0, 0)),
    "gmres_fixed2": (None, (0, 0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_case_decides_with_margin(name):
    case = CASES[name]
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0)
    status, trig = EXPECT[name]
    if status is not None:
        assert ref.status == status, (name, ref.status)
    if trig is not None:
        assert tuple(ref.switch_trigger) == trig, (name, ref.switch_trigger)
    if case.get("x0") == "head_solution":
        assert ref.switch_iter[0] == 0 and ref.switch_trigger[0] == 5
    if case["ctrl"].get("l") is not None:
        prm = case["ctrl"]
        assert all(t in (1, 2, 3, 5) for t in ref.switch_trigger)
        p = O.make_params(**{k: v for k, v in prm.items()})
        upto = max(ref.switch_iter) if max(ref.switch_iter) > 0 else ref.iters
        assert decision_margin(ref.hist, p, upto) > 1e-4
    assert tol_margin(ref.hist, 1e-10) > 1e-6
    if ref.status == O.OK:
        assert ref.relres_true <= 1e-10
    else:  # fixed two segments: the all-segment residual stays clearly above 1e-10
        assert ref.relres_true > 1.5e-10


def test_t_half_rule_changes_the_decision():
    """Same system and grid: nDec_limit reads nDec = 9 as below the limit
    (Condition 1), t/2 = 5 as not below (Condition 2)."""
    a = run_oracle(CASES["cg_multi_c1"], *build(CASES["cg_multi_c1"]))
    b = run_oracle(CASES["cg_multi_rule_t_half"], *build(CASES["cg_multi_rule_t_half"]))
    assert a.switch_iter[0] == b.switch_iter[0] == 60
    assert a.switch_trigger[0] == 1 and b.switch_trigger[0] == 2


def test_batch_systems_decide_with_margin():
    trig = set()
    for name, mk, seed in BATCH_SYSTEMS:
        A = mk()
        _, b = rhs_from_solution(A, seed)
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", switch_mode=0, orth=1,
                            **BATCH_CTRL)
        ref = O.cg(A.indptr, b, prm, A.indices, A.data, enc)
        assert ref.status == O.OK, name
        assert decision_margin(ref.hist, prm, max(ref.switch_iter)) > 1e-4, name
        assert tol_margin(ref.hist, 1e-10) > 1e-6, name
        trig |= set(ref.switch_trigger)
    assert 2 in trig and 5 in trig  # Condition 2 and the tolerance escalation


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c["method"] == "cg"])
def test_decision_replay_reproduces_the_oracle(name):
    """Replaying the controller on the oracle's own CG history gives the
    oracle's switch points and triggers: the replay is a faithful statement
    of the decisions the GPU tests hold the GPU's histories to."""
    from ctrl_cases import oracle_params, replay_cg_decisions
    case = CASES[name]
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0)
    got = replay_cg_decisions(ref.hist, ref.seg_hist, ref.iters, enc.eta, oracle_params(case),
                              case.get("fixed", 0))
    want = [(j, t) for j, t in zip(ref.switch_iter, ref.switch_trigger) if j >= 0]
    assert got[:2] == want


def test_decision_replay_catches_a_planted_mistake():
    """A history whose segment record steps up one iteration late (as a
    controller reading a stale residual would record) is rejected."""
    from ctrl_cases import oracle_params, replay_cg_decisions
    case = CASES["cg_multi_rule_t_half"]
    A, b, enc, x0 = build(case)
    ref = run_oracle(case, A, b, enc, x0)
    seg = ref.seg_hist.copy()
    j = ref.switch_iter[0]
    seg[j + 1] = seg[j]  # the switch recorded one iteration late
    with pytest.raises(AssertionError):
        replay_cg_decisions(ref.hist, seg, ref.iters, enc.eta, oracle_params(case))
