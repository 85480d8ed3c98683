"""The polynomial fits of the tangent-form step (csrc/tan_fit.hpp): for every variant,
|1 + x R(x) - tan(sqrt x)/sqrt x| <= 2^-57 on [0, X_v] with the coefficients as written, checked
in 40-digit arithmetic on a grid finer than the generator's (T(0) = 1 exactly by construction); the
cos^2 degree table meets its own bound."""
import math
import os
import re

import mpmath as mp

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1704_08919_amd", "csrc",
                   "tan_fit.hpp")


def _tables():
    src = open(HDR).read()
    deg = [int(v) for v in re.search(r"kFitDegree\[kNumFit\] = \{([^}]*)\}", src).group(1).split(",")]
    xmax = [float(v) for v in re.search(r"kFitXmax\[kNumFit\] = \{([^}]*)\}", src).group(1).split(",")]
    cos2 = [int(v) for v in re.search(r"kFitCos2Degree\[kNumFit\] = \{([^}]*)\}", src).group(1).split(",")]
    body = re.search(r"kFitCoef\[kNumFit\]\[kFitMaxTerms\] = \{(.*?)\n\};", src, re.S).group(1)
    coef = [[float(v) for v in row.split(",")] for row in re.findall(r"\{([^{}]*)\}", body)]
    return deg, xmax, cos2, coef


def _T(x):
    if x == 0:
        return mp.mpf(1)
    r = mp.sqrt(x)
    return mp.tan(r) / r


def test_fits_meet_their_bound():
    mp.mp.dps = 40
    deg, xmax, _, coef = _tables()
    assert len(deg) == len(xmax) == len(coef) == 8
    assert all(a < b for a, b in zip(xmax, xmax[1:]))
    tol = mp.mpf(2) ** -57
    for n, X, c in zip(deg, xmax, coef):
        c = [mp.mpf(v) for v in c[:n]]  # R has degree n - 1
        assert abs(c[0] - mp.mpf(1) / 3) < 1e-13  # R(0) = 1/3 up to the fit's own error
        worst = mp.mpf(0)
        for i in range(6001):
            x = mp.mpf(X) * i / 6000
            r = mp.mpf(0)
            for cj in reversed(c):
                r = r * x + cj
            worst = max(worst, abs(1 + x * r - _T(x)))
        assert worst <= tol, (n, X, float(worst / tol))


def test_cos2_degrees_cover_the_ranges():
    _, xmax, cos2, _ = _tables()
    for X, M in zip(xmax, cos2):
        first_omitted = 2.0 ** (2 * M + 1) * X ** (M + 1) / math.factorial(2 * M + 2)
        assert first_omitted < 2.0 ** -59
