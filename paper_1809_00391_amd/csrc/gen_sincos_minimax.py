"""Coefficients of the sine, cosine and logarithm polynomials in mbt_fastmath.h.

On |x| <= pi/4, with z = x^2:
    sin x = x + x z P(z),   P of degree 5  (terms x^3 .. x^13)
    cos x = 1 - z/2 + z^2 Q(z),  Q of degree 5  (terms x^4 .. x^14)
P and Q minimise the largest error of sin and cos themselves, i.e. the
weighted errors z (g_s - P) and z^2 (g_c - Q) with
    g_s(z) = (sin(sqrt z) / sqrt z - 1) / z,   g_c(z) = (cos(sqrt z) - 1 + z/2) / z^2,
and for the logarithm's atanh series on |s| <= 3 - 2 sqrt(2),
    atanh s = s + s z L(z),  L of degree 6  (terms s^3 .. s^15),
minimising the relative error of atanh, i.e. z (g_l - L) with
    g_l(z) = (atanh(sqrt z) / sqrt z - 1) / z,
found by the Remez exchange algorithm in 60-digit arithmetic (mpmath).
Run: python gen_sincos_minimax.py  (prints the coefficients and the
achieved maximum errors).
"""
import mpmath as mp

mp.mp.dps = 60
ZMAX = (mp.pi / 4) ** 2
DEG = 5


def g_sin(z):
    if z == 0:
        return mp.mpf(-1) / 6
    r = mp.sqrt(z)
    return (mp.sin(r) / r - 1) / z


def g_cos(z):
    if z == 0:
        return mp.mpf(1) / 24
    return (mp.cos(mp.sqrt(z)) - 1 + z / 2) / (z * z)


def g_log(z):
    if z == 0:
        return mp.mpf(1) / 3
    r = mp.sqrt(z)
    return (mp.atanh(r) / r - 1) / z


def remez(g, weight, deg=DEG, lo=mp.mpf(0), hi=ZMAX, iters=30):
    n = deg + 2
    # Chebyshev extrema as the first reference
    pts = [lo + (hi - lo) * (1 - mp.cos(mp.pi * i / (n - 1))) / 2 for i in range(n)]
    for _ in range(iters):
        # solve sum_k c_k z_i^k + (-1)^i E / w(z_i) = g(z_i)
        A = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, z in enumerate(pts):
            for k in range(deg + 1):
                A[i, k] = z ** k
            A[i, deg + 1] = (-1) ** i / weight(z) if weight(z) != 0 else (-1) ** i * mp.mpf(10) ** 30
            b[i] = g(z)
        sol = mp.lu_solve(A, b)
        c = [sol[k] for k in range(deg + 1)]
        err = lambda z: weight(z) * (g(z) - sum(c[k] * z ** k for k in range(deg + 1)))
        # new reference: extrema of the weighted error between sign changes
        grid = [lo + (hi - lo) * i / 4000 for i in range(4001)]
        vals = [err(z) for z in grid]
        ext = []
        seg_best = 0
        for i in range(1, len(grid)):
            if vals[i] * vals[seg_best] < 0:
                ext.append(seg_best)
                seg_best = i
            elif abs(vals[i]) > abs(vals[seg_best]):
                seg_best = i
        ext.append(seg_best)
        if len(ext) < n:
            break
        # keep n alternating extrema of largest size
        while len(ext) > n:
            if abs(vals[ext[0]]) < abs(vals[ext[-1]]):
                ext.pop(0)
            else:
                ext.pop()
        pts = [grid[i] for i in ext]
    return c, max(abs(v) for v in vals)


def main():
    cs, es = remez(g_sin, lambda z: z)
    cc, ec = remez(g_cos, lambda z: z * z)
    print("sin: x + x z P(z), P coefficients (z^0 .. z^5):")
    for k, v in enumerate(cs):
        print(f"  S{k} = {mp.nstr(v, 25)}  -> {float(v)!r}")
    print(f"  max |error of sin| ~ {mp.nstr(es, 5)}")
    print("cos: 1 - z/2 + z^2 Q(z), Q coefficients (z^0 .. z^5):")
    for k, v in enumerate(cc):
        print(f"  C{k} = {mp.nstr(v, 25)}  -> {float(v)!r}")
    print(f"  max |error of cos| ~ {mp.nstr(ec, 5)}")
    smax = 3 - 2 * mp.sqrt(2)
    cl, el = remez(g_log, lambda z: z, deg=6, hi=smax * smax)
    print("atanh: s + s z L(z), L coefficients (z^0 .. z^6):")
    for k, v in enumerate(cl):
        print(f"  L{k} = {mp.nstr(v, 25)}  -> {float(v)!r}")
    print(f"  max relative error of atanh ~ {mp.nstr(el, 5)}")


if __name__ == "__main__":
    main()
