"""The branch-free FP64 sin/cos of the FP64 kernels (sincos_halfturn in dbie_internal.h), checked on
the CPU: its constants are read from the source, every step is emulated in double precision with
single-rounded FMAs (exact rational arithmetic, then one rounding), and the results are compared
with 40-digit mpmath over random and adversarial arguments (near multiples of pi/2, zeros,
tiny values, the edges of the reduction interval and of the argument bound)."""
import os
import random
import re
import struct
from fractions import Fraction

import mpmath as mp
import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1306_1122_amd", "csrc", "dbie_internal.h")


def _body():
    src = open(SRC).read()
    m = re.search(r"uint64_t sincos_halfturn\(double t, double\* s, double\* c\) \{(.*?)\n\}", src, re.S)
    assert m, "sincos_halfturn not found"
    return m.group(1), src


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _constants():
    body, src = _body()
    num = r"(-?[0-9.]+(?:e-?[0-9]+)?)"
    k1pi = float(re.search(r"double kb = __builtin_fma\(t, " + num + r", kRoundMagic\)", body).group(1))
    assert re.search(r"double k = kb - kRoundMagic;", body)
    assert re.search(r"return __builtin_bit_cast\(uint64_t, kb\) << 63;", body)
    pi_parts = [float(x) for x in re.findall(r"__builtin_fma\(-k, " + num + r", ", body)]
    p = re.findall(r"double p = __builtin_fma\(z, " + num + r", " + num + r"\)", body)[0]
    ps = [float(x) for x in re.findall(r"p = __builtin_fma\(z, p, " + num + r"\)", body)]
    q = re.findall(r"double q = __builtin_fma\(z, " + num + r", " + num + r"\)", body)[0]
    qs = [float(x) for x in re.findall(r"q = __builtin_fma\(z, q, " + num + r"\)", body)]
    bound = float(re.search(r"kSincosBound = " + num + ";", src).group(1))
    magic = float(re.search(r"kRoundMagic = " + num + ";", src).group(1))
    # highest degree first, as the Horner steps of the source
    return k1pi, pi_parts, [float(p[0]), float(p[1])] + ps, [float(q[0]), float(q[1])] + qs, bound, magic


K1PI, PI_PARTS, PC, QC, BOUND, MAGIC = _constants()


def sincos_halfturn(t):
    """(sin t, cos t) from the device steps: sin r, cos r and the parity of k, t = k pi + r."""
    kb = _fma(t, K1PI, MAGIC)           # t/pi rounded to an integer (ties to even) by the addition
    k = kb - MAGIC                      # exact
    odd = struct.unpack("<Q", struct.pack("<d", kb))[0] & 1   # the sign mask is this bit moved to bit 63
    assert k == int(k) and odd == int(k) & 1
    r = _fma(-k, PI_PARTS[0], t)
    r = _fma(-k, PI_PARTS[1], r)
    z = r * r
    p = _fma(z, PC[0], PC[1])
    for cf in PC[2:]:
        p = _fma(z, p, cf)
    sr = _fma(r * z, p, r)
    q = _fma(z, QC[0], QC[1])
    for cf in QC[2:]:
        q = _fma(z, q, cf)
    cr = _fma(z * z, q, _fma(z, -0.5, 1.0))
    return (-sr, -cr) if odd else (sr, cr)


def test_constants_parsed():
    assert len(PI_PARTS) == 2 and len(PC) == 8 and len(QC) == 7
    assert BOUND == 2.0 ** 19
    # 1.5 2^52: spacing 1 in its binade, which |t/pi| < 2^51 never leaves
    assert MAGIC == 1.5 * 2.0 ** 52 and BOUND * K1PI < 2.0 ** 51
    mp.mp.dps = 40
    assert abs(mp.mpf(PI_PARTS[0]) + mp.mpf(PI_PARTS[1]) - mp.pi) < 1e-32


@pytest.mark.parametrize("seed", [1, 2])
def test_within_one_ulp_of_40_digit_values(seed):
    mp.mp.dps = 40
    rng = random.Random(seed)
    ts = [rng.uniform(-BOUND, BOUND) for _ in range(700)] + [rng.uniform(-8.0, 8.0) for _ in range(500)]
    ts += [float(mp.pi * k / 2) + d for k in range(-300000, 300001, 29989) for d in (0.0, 3e-13, -2e-9)]
    ts += [float(mp.pi * (k + mp.mpf(1) / 2)) + d for k in range(-150000, 150001, 14999) for d in (0.0, 1e-10)]
    ts += [0.0, -0.0, 1e-300, -5e-324, 1.5707963267948966, -1.5707963267948968, 3.141592653589793,
           BOUND * 0.999999, -BOUND * 0.999999]
    worst = 0.0
    for t in ts:
        s, c = sincos_halfturn(t)
        es, ec = abs(s - float(mp.sin(t))), abs(c - float(mp.cos(t)))
        worst = max(worst, es, ec)
        assert es <= 2.3e-16 and ec <= 2.3e-16, (t, es, ec)
    print("largest absolute error %.2e" % worst)


# ------------------------------------------------------------------------------------------------
# sincos_table16: the table-driven form of the FP64 bulk kernel
# ------------------------------------------------------------------------------------------------
def _table16():
    src = open(SRC).read()
    tab = re.search(r"kSinCos16\[64\] = \{(.*?)\};", src, re.S).group(1)
    vals = [float(x) for x in re.findall(r"-?[0-9.]+(?:e-?[0-9]+)?", tab)]
    body = re.search(r"void sincos_table16\(double t, const double2\* __restrict__ tab, double\* s, double\* c\) "
                     r"\{(.*?)\n\}", src, re.S).group(1)
    num = r"(-?[0-9.]+(?:e-?[0-9]+)?)"
    k16 = float(re.search(r"double kb = __builtin_fma\(t, " + num + r", kRoundMagic\)", body).group(1))
    parts = [float(x) for x in re.findall(r"__builtin_fma\(-k, " + num + r", ", body)]
    p = re.findall(r"double p = __builtin_fma\(z, " + num + r", " + num + r"\)", body)[0]
    ps = [float(x) for x in re.findall(r"p = __builtin_fma\(z, p, " + num + r"\)", body)]
    q = re.findall(r"double q = __builtin_fma\(z, " + num + r", " + num + r"\)", body)[0]
    qs = [float(x) for x in re.findall(r"q = __builtin_fma\(z, q, " + num + r"\)", body)]
    assert re.search(r"tab\[\(uint32_t\)__builtin_bit_cast\(uint64_t, kb\) & 31u\]", body)
    assert re.search(r"\*s = __builtin_fma\(e\.y, sr, e\.x \* cr\);", body)
    assert re.search(r"\*c = __builtin_fma\(-e\.x, sr, e\.y \* cr\);", body)
    return vals, k16, parts, [float(p[0]), float(p[1])] + ps, [float(q[0]), float(q[1])] + qs


TAB16, K16, PARTS16, PS16, QS16 = _table16()


def _fit_script():
    """csrc/sincos_fit.py, the provenance of the constants (loaded as a module; it needs mpmath)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("sincos_fit", os.path.join(os.path.dirname(SRC), "sincos_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def sincos_table16(t):
    """(sin t, cos t) from the device steps of sincos_table16."""
    kb = _fma(t, K16, MAGIC)
    k = kb - MAGIC
    j = struct.unpack("<Q", struct.pack("<d", kb))[0] & 31
    assert k == int(k) and j == int(k) % 32
    r = _fma(-k, PARTS16[0], t)
    r = _fma(-k, PARTS16[1], r)
    z = r * r
    p = _fma(z, PS16[0], PS16[1])
    for cf in PS16[2:]:
        p = _fma(z, p, cf)
    sr = _fma(r * z, p, r)
    q = _fma(z, QS16[0], QS16[1])
    for cf in QS16[2:]:
        q = _fma(z, q, cf)
    cr = _fma(z * z, q, _fma(z, -0.5, 1.0))
    S, C = TAB16[2 * j], TAB16[2 * j + 1]
    return _fma(C, sr, S * cr), _fma(-S, sr, C * cr)


def test_table16_constants():
    """The table holds (sin, cos)(j pi/16) correctly rounded; the reduction constants split pi/16 to
    ~1e-33 and 16/pi is rounded to nearest; the cosine coefficients are +-1/n! rounded, and the sine
    coefficients are those the committed fit script computes."""
    import math
    from fractions import Fraction
    mp.mp.dps = 40
    assert len(TAB16) == 64
    for j in range(32):
        assert TAB16[2 * j] == float(mp.sinpi(mp.mpf(j) / 16)) and TAB16[2 * j + 1] == float(mp.cospi(mp.mpf(j) / 16))
    assert abs(mp.mpf(PARTS16[0]) + mp.mpf(PARTS16[1]) - mp.pi / 16) < 1e-33
    assert K16 == float(16 / mp.pi)
    assert PS16 == list(reversed(_fit_script().table16_sin()))
    assert QS16 == [float(Fraction((-1) ** (n // 2), math.factorial(n))) for n in (8, 6, 4)]


@pytest.mark.parametrize("seed", [1, 2])
def test_table16_within_one_and_a_half_ulp_of_40_digit_values(seed):
    mp.mp.dps = 40
    rng = random.Random(seed)
    ts = [rng.uniform(-BOUND, BOUND) for _ in range(700)] + [rng.uniform(-8.0, 8.0) for _ in range(500)]
    # near the reduction points k pi/32 (both sides of a rounding of k) and near zeros of sin, cos
    ts += [float(mp.pi * (2 * k + 1) / 32) + d for k in range(-600000, 600001, 59999) for d in (0.0, 1e-12, -1e-12)]
    ts += [float(mp.pi * k / 2) + d for k in range(-300000, 300001, 29989) for d in (0.0, 3e-13, -2e-9)]
    ts += [0.0, -0.0, 1e-300, -5e-324, 0.09817477042468103, -0.09817477042468103, BOUND * 0.999999,
           -BOUND * 0.999999]
    worst = 0.0
    for t in ts:
        s, c = sincos_table16(t)
        es, ec = abs(s - float(mp.sin(t))), abs(c - float(mp.cos(t)))
        worst = max(worst, es, ec)
        assert es <= 3.4e-16 and ec <= 3.4e-16, (t, es, ec)
    print("largest absolute error %.2e" % worst)
