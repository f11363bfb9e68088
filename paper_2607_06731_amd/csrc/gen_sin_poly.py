#!/usr/bin/env python3
"""Generate the fp32 coefficients of the device sine kernel.

sin(r) ~= r + r^3 * (c0 + c1 u + c2 u^2 + c3 u^3),  u = r^2  (odd degree 9),
on |r| <= pi/2 + 0.01, minimising the maximum *relative* error (Lawson's
iteratively reweighted least squares, which converges to the minimax
solution), then rounding the coefficients to fp32 and re-fitting the
remaining ones after each rounding.  The device uses it for sin after a
Cody-Waite reduction by pi (Cody & Waite, "Software Manual for the
Elementary Functions", 1980) and for cos after a reduction by pi around
(k + 1/2) pi.  Also prints the three-part fp32 split of pi and 1/pi.  Run: python gen_sin_poly.py  (prints the C constants and the
achieved error).
"""
from decimal import Decimal, getcontext

import numpy as np

# pi to 60 significant digits (enough for the three-part fp32 split below)
PI_DIGITS = "3.14159265358979323846264338327950288419716939937510582097494"

DEG = 4              # number of coefficients c0..c3 (odd degree 9)
HALF_PI = np.pi / 2 + 0.01   # margin: k = rint(x / pi) is computed in fp32


def fit(fixed, n_pts=4000, iters=60):
    """Minimax fit of the free coefficients; `fixed` maps index -> value."""
    x = np.cos(np.linspace(0, np.pi / 2, n_pts)) * HALF_PI      # Chebyshev-like
    x = x[x > 1e-4]
    u = x * x
    target = (np.sin(x) - x) / x ** 3                          # = Q(u)
    # relative error of sin = x^3 (Q - target) / sin(x)
    wt = x ** 3 / np.sin(x)
    free = [i for i in range(DEG) if i not in fixed]
    A = np.stack([u ** i for i in free], axis=1)
    b = target - sum(v * u ** i for i, v in fixed.items())
    lw = np.ones_like(x)
    for _ in range(iters):
        W = lw * wt
        coef, *_ = np.linalg.lstsq(A * W[:, None], b * W, rcond=None)
        err = np.abs((A @ coef - b) * wt)
        lw = lw * (err + 1e-30)
        lw /= lw.sum()
    out = dict(fixed)
    out.update(zip(free, coef))
    return [out[i] for i in range(DEG)]


def main():
    fixed = {}
    for i in range(DEG):
        c = fit(fixed)
        fixed[i] = float(np.float32(c[i]))
    c = [fixed[i] for i in range(DEG)]
    # error of the fp32-rounded coefficients evaluated in fp64
    x = np.linspace(1e-6, HALF_PI, 200001)
    u = x * x
    q = sum(ci * u ** i for i, ci in enumerate(c))
    rel = np.abs((x + x ** 3 * q - np.sin(x)) / np.sin(x))
    for i, ci in enumerate(c):
        print("constexpr float kSinC%d = %.9e;  // 0x%08x" % (
            i, ci, np.float32(ci).view(np.uint32)))
    print("// max relative error of the polynomial (fp64 evaluation): %.3e" % rel.max())
    # Cody-Waite split of pi into three fp32 parts (each the fp32 rounding of
    # what the previous parts leave), and 1/pi
    getcontext().prec = 60
    rest = Decimal(PI_DIGITS)
    for name in ("kPiA", "kPiB", "kPiC"):
        part = np.float32(float(rest))
        rest -= Decimal(float(part))
        print("constexpr float %s = %.9e;  // 0x%08x" % (name, part, part.view(np.uint32)))
    inv = np.float32(float(1 / Decimal(PI_DIGITS)))
    print("constexpr float kInvPi = %.9e;  // 0x%08x" % (inv, inv.view(np.uint32)))


if __name__ == "__main__":
    main()
