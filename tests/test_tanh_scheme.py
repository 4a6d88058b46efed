"""The branch-free tanh used by the HIP kernels (|x| < 0.4: Maclaurin series of
tanh(x)/x through x^12; otherwise 1 - 2/(exp(2|x|) + 1)), evaluated step by
step in float32, stays within 4 ulp of the float64 tanh everywhere."""
from fractions import Fraction as F

import numpy as np

# tanh(x)/x = sum_k c_k x^(2k); c_k = 2^(2k+2) (2^(2k+2) - 1) B_(2k+2) / (2k+2)!
COEF = [F(1), F(-1, 3), F(2, 15), F(-17, 315), F(62, 2835), F(-1382, 155925), F(21844, 6081075)]
NEXT = F(-929569, 638512875)


def bernoulli(n):
    A = [F(0)] * (n + 1)
    for m in range(n + 1):
        A[m] = F(1, m + 1)
        for j in range(m, 0, -1):
            A[j - 1] = j * (A[j - 1] - A[j])
    return A[0]


def test_series_coefficients_follow_bernoulli_numbers():
    from math import factorial
    for k, c in enumerate(COEF + [NEXT]):
        n = 2 * k + 2
        expect = F(2 ** n * (2 ** n - 1)) * bernoulli(n) / factorial(n)
        assert c == expect, k


def tanh_scheme_f32(x):
    x = np.asarray(x, np.float32)
    a = np.abs(x)
    u = (x * x).astype(np.float32)
    p = np.float32(float(COEF[6]))
    for k in range(5, -1, -1):
        p = (p * u + np.float32(float(COEF[k]))).astype(np.float32)
    small = (x * p).astype(np.float32)
    with np.errstate(over="ignore"):
        e = np.exp2((a * np.float32(2.8853900817779268)).astype(np.float32)).astype(np.float32)
    r = (np.float32(1) / (e + np.float32(1))).astype(np.float32)
    big = np.copysign((np.float32(1) - np.float32(2) * r).astype(np.float32), x)
    return np.where(a < np.float32(0.4), small, big)


def test_truncation_below_float32_rounding():
    assert abs(float(NEXT)) * 0.4 ** 14 < 1e-8


def test_scheme_within_4_ulp():
    xs = np.concatenate([np.linspace(-20, 20, 400_001), np.linspace(-0.5, 0.5, 400_001),
                         np.logspace(-30, 1.5, 40_001), -np.logspace(-30, 1.5, 40_001)]).astype(np.float32)
    ref = np.tanh(xs.astype(np.float64))
    got = tanh_scheme_f32(xs).astype(np.float64)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) < 4.0
    ext = tanh_scheme_f32(np.array([0.0, 60.0, -60.0, np.inf, -np.inf], np.float32))
    assert list(ext) == [0.0, 1.0, -1.0, 1.0, -1.0]
