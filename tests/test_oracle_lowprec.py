"""Pins of the oracle's FP16 / BF16 comparators (Section IV-C: the 16-bit
formats against which the paper compares the head-only GSE-SEM operator;
every value stored in FP16 or BF16, widened to FP64, FP64 accumulation).

Checks independent of the oracle's arithmetic:
  * binary16 rounding against numpy's float16 conversion (IEEE round to
    nearest even, overflow to infinity), on random values over the whole
    range, its subnormals, exact ties and the overflow boundary;
  * bfloat16 rounding against exact rational arithmetic of the definition
    (the nearest multiple of the value's quantum 2^(e-7), ties to even), and
    against torch's bfloat16 conversion on values that are already FP32
    (where converting through FP32 cannot round twice);
  * widening is exact: the widened value is the rounded rational;
  * the 16-bit SpMV equals the dense product with the rounded values.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def rng_values(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    v = np.exp2(rng.uniform(lo, hi, n)) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return v


def fp16_cases():
    v = [rng_values(1, 40000, -30, 17)]
    # exact midpoints between neighbours (ties), normal and subnormal, and the overflow edge
    k = np.arange(1, 2000, dtype=np.float64)
    v.append((1024 + k + 0.5) * 2.0 ** -10)        # ties in [1, 2)
    v.append((k + 0.5) * 2.0 ** -24)                # ties among subnormals
    v.append(np.array([65504.0, 65519.99, 65520.0, 65536.0, 1e300, 2.0 ** -25,
                       np.nextafter(2.0 ** -25, 1.0), 0.0, -0.0, 6.1e-5]))
    return np.concatenate(v)


def test_fp16_rounding_equals_ieee_binary16():
    v = fp16_cases()
    with np.errstate(over="ignore"):
        want = v.astype(np.float16).view(np.uint16)
    got, over = O.lp_convert(v, O.LP_FP16)
    assert np.array_equal(got, want)
    with np.errstate(over="ignore"):
        assert over == int(np.sum(np.isinf(v.astype(np.float16)) & np.isfinite(v)))
    assert over >= 3  # 65520, 65536 and 1e300 overflow


def bf16_exact(v: float) -> float:
    """Round-to-nearest-even onto bfloat16 (8 exponent, 7 fraction bits)."""
    if v == 0.0:
        return v
    a = abs(Fraction(v))
    e = math.floor(math.log2(a))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = Fraction(2) ** (max(e, -126) - 7)
    n = a / q
    fl = math.floor(n)
    d = n - fl
    r = fl + 1 if (d > Fraction(1, 2) or (d == Fraction(1, 2) and fl % 2 == 1)) else fl
    mag = r * q
    if mag > (2 - Fraction(1, 128)) * Fraction(2) ** 127:
        return math.copysign(math.inf, v)
    return math.copysign(float(mag), v)


def test_bf16_rounding_equals_the_rational_definition():
    v = np.concatenate([rng_values(2, 6000, -140, 130),
                        (np.arange(128, 256) + 0.5) * 2.0 ** -7,   # ties in [1, 2)
                        (np.arange(1, 200) + 0.5) * 2.0 ** -133,   # ties among subnormals
                        np.array([3.4e38, 3.4028235e38, 3.39e38, 1e300, -0.0])])
    for x in v:
        h, over = O.lp_round(float(x), O.LP_BF16)
        want = bf16_exact(float(x))
        assert O.lp_widen(h, O.LP_BF16) == want, (x, want)
        assert over == (math.isinf(want) and math.isfinite(x))


def test_bf16_rounding_equals_torch_on_fp32_values():
    torch = pytest.importorskip("torch")
    v = rng_values(3, 50000, -120, 120).astype(np.float32).astype(np.float64)
    want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy()
    got, _ = O.lp_convert(v, O.LP_BF16)
    assert np.array_equal(got, want.view(np.uint16))


@pytest.mark.parametrize("fmt", [O.LP_FP16, O.LP_BF16])
def test_lp_spmv_equals_dense_product_of_rounded_values(fmt):
    import scipy.sparse as sp
    rng = np.random.default_rng(fmt)
    n = 300
    M = sp.random(n, n, density=0.03, random_state=4, format="csr")
    M.data = rng.uniform(-4, 4, M.nnz)
    plane, over = O.lp_convert(M.data, fmt)
    assert over == 0
    wide = np.array([O.lp_widen(h, fmt) for h in plane])
    x = rng.uniform(-1, 1, n)
    y = O.lp_spmv(M.indptr, M.indices, plane, fmt, x)
    ref = sp.csr_matrix((wide, M.indices, M.indptr), shape=(n, n)) @ x
    assert np.allclose(y, ref, rtol=1e-14, atol=1e-14)
    if fmt == O.LP_FP16:
        assert np.array_equal(wide, M.data.astype(np.float16).astype(np.float64))


def test_lp_cg_converges_on_its_own_operator_and_floors_on_the_true_one():
    """CG on the FP16 operator of a diffusion system: the solver meets the
    tolerance on A_h (the operator it knows), while the true residual with
    the FP64 matrix stays near the rounding perturbation ||A - A_h||."""
    from workloads import diffusion3d, rhs_from_solution
    A = diffusion3d(10, 3, decades=2.0)
    _, b = rhs_from_solution(A, 3)
    plane, over = O.lp_convert(A.data, O.LP_FP16)
    assert over == 0
    prm = O.make_params(tol=1e-10, max_iter=5000, fixed_segments=O.S_LP, orth=1)
    r = O.cg(A.indptr, b, prm, A.indices, A.data, lp=(plane, O.LP_FP16))
    assert r.status == O.OK and r.relres_true <= 1e-10  # its own operator's residual
    true = np.linalg.norm(b - A.to_scipy() @ r.x) / np.linalg.norm(b)
    assert 1e-6 < true < 1e-1
