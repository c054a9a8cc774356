"""Coefficients of the double-precision exp/expm1 kernel polynomial in
emrkc_device.h: after the reduction x = k ln2 + r, |r| <= ln2/2,
e^r - 1 = r + r^2 p(r) with p(r) ~ (e^r - 1 - r) / r^2, and p is the
degree-9 minimax polynomial of that function on [-ln2/2, ln2/2] (absolute
error), found by the Remez exchange algorithm (E. Ya. Remez, 1934) in
50-digit decimal arithmetic.  Prints the coefficients rounded to double and
the fitted error.  Run: python3 gen_exp_minimax.py"""
from decimal import Decimal, getcontext

getcontext().prec = 50
DEG = 9
A = Decimal(2).ln() / 2


def f(r):
    """(e^r - 1 - r) / r^2 = sum_{j>=0} r^j / (j+2)!, by its series."""
    s, term, j = Decimal(0), Decimal(1) / 2, 0
    while abs(term) > Decimal(10) ** -48:
        s += term
        j += 1
        term = term * r / (j + 2)
    return s


def poly(c, r):
    acc = Decimal(0)
    for cj in reversed(c):
        acc = acc * r + cj
    return acc


def solve(M, b):
    """Gaussian elimination with partial pivoting, in Decimal."""
    n = len(b)
    M = [row[:] + [b[i]] for i, row in enumerate(M)]
    for col in range(n):
        piv = max(range(col, n), key=lambda i: abs(M[i][col]))
        M[col], M[piv] = M[piv], M[col]
        for i in range(col + 1, n):
            fac = M[i][col] / M[col][col]
            for j in range(col, n + 1):
                M[i][j] -= fac * M[col][j]
    x = [Decimal(0)] * n
    for i in reversed(range(n)):
        x[i] = (M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))) / M[i][i]
    return x


def remez(iterations=12, grid=4000):
    import math
    n = DEG + 2  # reference points: DEG + 1 coefficients and the level E
    pts = [A * Decimal(math.cos(math.pi * (n - 1 - i) / (n - 1))) for i in range(n)]
    xs = [-A + 2 * A * Decimal(i) / grid for i in range(grid + 1)]
    fx = [f(x) for x in xs]
    for _ in range(iterations):
        # p(x_i) + (-1)^i E = f(x_i)
        M = [[x ** j for j in range(DEG + 1)] + [Decimal((-1) ** i)] for i, x in enumerate(pts)]
        sol = solve(M, [f(x) for x in pts])
        c, E = sol[:-1], sol[-1]
        err = [poly(c, x) - v for x, v in zip(xs, fx)]
        # new reference: the extremum of each run of one sign
        new, start = [], 0
        for i in range(1, len(err) + 1):
            if i == len(err) or (err[i] > 0) != (err[start] > 0):
                k = max(range(start, i), key=lambda t: abs(err[t]))
                new.append(xs[k])
                start = i
        if len(new) >= n:
            # keep n alternating extrema with the largest errors
            while len(new) > n:
                ends = [abs(poly(c, new[0]) - f(new[0])), abs(poly(c, new[-1]) - f(new[-1]))]
                new = new[1:] if ends[0] < ends[1] else new[:-1]
            pts = new
    maxerr = max(abs(e) for e in err)
    return c, abs(E), maxerr


if __name__ == "__main__":
    c, level, maxerr = remez()
    print("// degree-%d minimax of (e^r - 1 - r)/r^2 on [-ln2/2, ln2/2]: level %.3e, max error %.3e"
          % (DEG, float(level), float(maxerr)))
    for j, cj in enumerate(c):
        print("  c%d = %r  (1/(j+2)! = %r)" % (j, float(cj), float(1 / Decimal(__import__("math").factorial(j + 2)))))
