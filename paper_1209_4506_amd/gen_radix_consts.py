"""Write csrc/radix_consts.hpp: cos(2 pi t / R) and sin(2 pi t / R) for the
butterfly radices, as decimal literals correct to 32 significant digits.

The values are computed in 60-digit decimal arithmetic: pi from Machin's
formula, 16 atan(1/5) - 4 atan(1/239), and cos / sin of 2 pi t / R from their
Taylor series.  The compiler rounds each literal to double (the nearest
double, since 32 digits pin it) and the kernels then to their working
precision.  Usage: python -m paper_1209_4506_amd.gen_radix_consts
"""
from decimal import Decimal, getcontext
import os

RADICES = (2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16)
getcontext().prec = 60


def _atan_inv(n):
    """atan(1 / n) by its alternating series."""
    x = Decimal(1) / n
    x2 = x * x
    term, total, k = x, x, 1
    while True:
        term *= -x2
        k += 2
        t = term / k
        if abs(t) < Decimal(10) ** -58:
            return total
        total += t


def _pi():
    return 16 * _atan_inv(5) - 4 * _atan_inv(239)


def _cos_sin(a):
    """cos a and sin a by their Taylor series (|a| < 2 pi)."""
    c, s = Decimal(0), Decimal(0)
    term, k = Decimal(1), 0  # a^k / k!
    while abs(term) > Decimal(10) ** -58 or k < 4:
        if k % 4 == 0:
            c += term
        elif k % 4 == 1:
            s += term
        elif k % 4 == 2:
            c -= term
        else:
            s -= term
        k += 1
        term = term * a / k
    return c, s


def _lit(v):
    if abs(v) < Decimal(10) ** -40:  # exact zeros (the series leaves ~1e-59)
        return "0.0"
    return format(v, ".31e")


def render():
    pi = _pi()
    rows = {}
    for R in RADICES:
        vals = []
        for t in range(R):
            vals.append(_cos_sin(2 * pi * t / R))
        rows[R] = vals
    out = ["// cos(2 pi t / R) and sin(2 pi t / R), 0 <= t < R, for the butterfly radices,",
           "// as decimal literals correct to 32 significant digits (written by",
           "// gen_radix_consts.py from 60-digit decimal arithmetic; the compiler rounds",
           "// them to double, then the kernels to their working precision).",
           "#pragma once", "namespace hartree {"]
    for fn, idx in (("unit_cos", 0), ("unit_sin", 1)):
        out.append("__host__ __device__ constexpr double %s(int R, int t)" % fn)
        out.append("{")
        out.append("    t = ((t % R) + R) % R;")
        for R in RADICES:
            vals = [_lit(rows[R][t][idx]) for t in range(R)]
            expr = vals[-1]
            for t in range(R - 2, -1, -1):
                expr = "t == %d ? %s : %s" % (t, vals[t], expr)
            out.append("    if (R == %d) return %s;" % (R, expr))
        out.append("    return 0.0;")
        out.append("}")
    out.append("}  // namespace hartree")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "radix_consts.hpp")
    with open(path, "w") as fh:
        fh.write(render())
    print("wrote", path)
