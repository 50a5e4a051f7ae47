"""Generate the constant tables of the HIP path (cgks_tables.inc).

Exact rational arithmetic (fractions) for the Hermite stencils of Sec. 3.2
(Eq. 3.6-3.10, 3.18: every polynomial satisfies cell-average conditions and
cell-averaged-derivative conditions on unit cells), 40-digit mpmath for the
Gauss-Legendre points and everything evaluated at them.  Each face-value row
is checked against the coefficients printed in the paper (Eq. 3.8, 3.10,
3.18, with the one term the printed 7th-order point value omits restored).

Data slots of every stencil: [Q_{-2}, Q_{-1}, Q_0, Q_{+1}, Q_{+2},
h Qx_{-2}, h Qx_{-1}, h Qx_{+1}, h Qx_{+2}] (Q cell averages, Qx cell-averaged
derivatives, h the cell size); polynomials are in xi = (x - x_i)/h.

Run:  python gen_tables.py  (writes cgks_tables.inc next to this file)
"""
import os
from fractions import Fraction as Fr

import mpmath as mp

mp.mp.dps = 40

STENCILS = {
    # name: (average offsets, gradient offsets)
    "S0": ([-1, 0], [-1]),
    "S1": ([0, 1], [1]),
    "S2": ([-1, 0, 1], []),
    "R5": ([-1, 0, 1], [-1, 1]),
    "R7": ([-2, -1, 0, 1, 2], [-1, 1]),
    "R9": ([-2, -1, 0, 1, 2], [-2, -1, 1, 2]),
}
SLOT_Q = {-2: 0, -1: 1, 0: 2, 1: 3, 2: 4}
SLOT_H = {-2: 5, -1: 6, 1: 7, 2: 8}

# Face value / first / second derivative at xi = +1/2 as printed (rows over the 9 slots).
PRINTED = {
    "S0": ([0, Fr(-7, 6), Fr(13, 6), 0, 0, 0, Fr(-2, 3), 0, 0], [0, -3, 3, 0, 0, 0, -2, 0, 0],
           [0, -2, 2, 0, 0, 0, -2, 0, 0]),
    "S1": ([0, 0, Fr(1, 6), Fr(5, 6), 0, 0, 0, Fr(-1, 3), 0], [0, 0, -1, 1, 0, 0, 0, 0, 0],
           [0, 0, 2, -2, 0, 0, 0, 2, 0]),
    "S2": ([0, Fr(-1, 6), Fr(5, 6), Fr(1, 3), 0, 0, 0, 0, 0], [0, 0, -1, 1, 0, 0, 0, 0, 0],
           [0, 1, -2, 1, 0, 0, 0, 0, 0]),
    "R5": ([0, Fr(-23, 120), Fr(19, 30), Fr(67, 120), 0, 0, Fr(-3, 40), Fr(-7, 40), 0],
           [0, Fr(3, 8), -2, Fr(13, 8), 0, 0, Fr(1, 8), Fr(-3, 8), 0],
           [0, Fr(7, 4), -2, Fr(1, 4), 0, 0, Fr(3, 4), Fr(3, 4), 0]),
    "R7": ([Fr(-13, 1260), Fr(-223, 1260), Fr(717, 1260), Fr(757, 1260), Fr(22, 1260), 0, Fr(-120, 1260),
            Fr(-300, 1260), 0],
           [Fr(2, 108), Fr(53, 108), Fr(-243, 108), Fr(187, 108), Fr(1, 108), 0, Fr(24, 108), Fr(-48, 108), 0],
           [Fr(3, 24), Fr(38, 24), Fr(-30, 24), Fr(-6, 24), Fr(-5, 24), 0, 1, Fr(36, 24), 0]),
    "R9": ([Fr(-601, 15120), Fr(-2076, 15120), Fr(7524, 15120), Fr(9124, 15120), Fr(1149, 15120), Fr(-150, 15120),
            Fr(-1800, 15120), Fr(-4920, 15120), Fr(-270, 15120)],
           [Fr(275, 2592), Fr(1424, 2592), Fr(-6480, 2592), Fr(4720, 2592), Fr(61, 2592), Fr(66, 2592),
            Fr(984, 2592), Fr(-1320, 2592), Fr(-6, 2592)],
           [Fr(1291, 2592), Fr(2624, 2592), Fr(-432, 2592), Fr(-832, 2592), Fr(-2651, 2592), Fr(330, 2592),
            Fr(3288, 2592), Fr(7080, 2592), Fr(642, 2592)]),
}


def solve_exact(A, B):
    """Solve A X = B over the rationals (Gauss-Jordan); B has several columns."""
    n = len(A)
    M = [list(A[r]) + list(B[r]) for r in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def coefficient_map(name):
    """C[k][s]: coefficient of xi^k of the stencil polynomial per unit datum in slot s."""
    avg, grad = STENCILS[name]
    n = len(avg) + len(grad)
    A, B = [], []
    for o in avg:
        A.append([(Fr(2 * o + 1, 2) ** (k + 1) - Fr(2 * o - 1, 2) ** (k + 1)) / (k + 1) for k in range(n)])
        row = [Fr(0)] * 9
        row[SLOT_Q[o]] = Fr(1)
        B.append(row)
    for o in grad:
        A.append([Fr(0) if k == 0 else Fr(2 * o + 1, 2) ** k - Fr(2 * o - 1, 2) ** k for k in range(n)])
        row = [Fr(0)] * 9
        row[SLOT_H[o]] = Fr(1)
        B.append(row)
    return solve_exact(A, B)  # n x 9


def eval_row(C, xi, d):
    """Weights over the slots of the d-th xi-derivative at xi (xi exact or mpf)."""
    out = []
    for s in range(9):
        acc = 0
        for k in range(d, len(C)):
            f = 1
            for t in range(d):
                f *= (k - t)
            acc += f * C[k][s] * (xi ** (k - d))
        out.append(acc)
    return out


def gauss(m):
    xs, ws = mp.gauss_quadrature(m, "legendre") if hasattr(mp, "gauss_quadrature") else (None, None)
    if xs is None:
        # Newton on P_m (mpmath.legendre) from Chebyshev starts, on [-1, 1]
        xs, ws = [], []
        for i in range(1, m + 1):
            x = mp.cos(mp.pi * (i - mp.mpf(1) / 4) / (m + mp.mpf(1) / 2))
            for _ in range(100):
                p = mp.legendre(m, x)
                dp = m * (x * p - mp.legendre(m - 1, x)) / (x * x - 1)
                x = x - p / dp
            dp = m * (x * mp.legendre(m, x) - mp.legendre(m - 1, x)) / (x * x - 1)
            xs.append(x)
            ws.append(2 / ((1 - x * x) * dp * dp))
    pts = sorted(zip(xs, ws))
    return [p / 2 for p, _ in pts], [w / 2 for _, w in pts]


def tangential_weights(m):
    """First/second xi-derivative at Gauss point l of the middle row of the
    least-squares polynomial of degree min(2m+1, 8) through the m Gauss points
    of rows -1, 0, +1 (3m points; the interpolant for m = 2)."""
    xg, _ = gauss(m)
    X = [mp.mpf(r - 1) + xg[q] for r in range(3) for q in range(m)]
    n = len(X)
    q = min(2 * m + 2, 9)              # coefficients: degree + 1
    V = mp.matrix([[x ** k for k in range(q)] for x in X])
    P = (V.T * V) ** -1 * V.T          # q x n: coefficients per datum
    d1 = [[mp.mpf(0)] * n for _ in range(m)]
    d2 = [[mp.mpf(0)] * n for _ in range(m)]
    for l in range(m):
        x0 = xg[l]
        for a in range(n):
            d1[l][a] = mp.fsum(k * P[k, a] * x0 ** (k - 1) for k in range(1, q))
            d2[l][a] = mp.fsum(k * (k - 1) * P[k, a] * x0 ** (k - 2) for k in range(2, q))
    return d1, d2


def dbl(x):
    if isinstance(x, Fr):
        return float(x)  # correctly rounded
    return float(mp.mpf(x))


def fmt(v):
    return repr(dbl(v))


def main():
    lines = ["// Generated by gen_tables.py -- do not edit.", "// Slots: Q[-2..2], hQx[-2], hQx[-1], hQx[+1], hQx[+2].",
             "// constexpr tables are indexed with compile-time indices only (folded into the",
             "// instructions); the tangential weights are indexed per thread (device memory)."]
    maps = {k: coefficient_map(k) for k in STENCILS}
    # check the face rows against the printed coefficients
    for k, rows in PRINTED.items():
        for d in range(3):
            got = eval_row(maps[k], Fr(1, 2), d)
            want = [Fr(x) for x in rows[d]]
            assert got == want, (k, d, got, want)
    # polynomial coefficient maps for the AO(5,3) members
    for k, deg in (("S0", 3), ("S1", 3), ("S2", 3), ("R5", 5)):
        C = maps[k]
        lines.append(f"constexpr double kC_{k}[{deg}][9] = {{")
        for r in range(deg):
            lines.append("  {" + ", ".join(fmt(C[r][s]) for s in range(9)) + "},")
        lines.append("};")
    # linear-stencil evaluation weights at the faces: [side 0: xi=+1/2, 1: xi=-1/2][d][9]
    for k in ("R5", "R7", "R9"):
        C = maps[k]
        lines.append(f"constexpr double kF_{k}[2][3][9] = {{")
        for side, xi in ((0, Fr(1, 2)), (1, Fr(-1, 2))):
            lines.append("  {")
            for d in range(3):
                lines.append("    {" + ", ".join(fmt(w) for w in eval_row(C, xi, d)) + "},")
            lines.append("  },")
        lines.append("};")
    # Gauss points, weights, and linear-stencil values at the Gauss points
    lines.append("// Gauss-Legendre points on [-1/2, 1/2] and weights (sum 1) for m = 2, 3, 4")
    lines.append("constexpr double kGx[5][4] = {")
    gx = {}
    for m in range(5):
        if m < 2:
            lines.append("  {0, 0, 0, 0},")
            continue
        x, w = gauss(m)
        gx[m] = (x, w)
        lines.append("  {" + ", ".join(fmt(v) for v in x + [0] * (4 - m)) + "},")
    lines.append("};")
    lines.append("constexpr double kGw[5][4] = {")
    for m in range(5):
        if m < 2:
            lines.append("  {0, 0, 0, 0},")
            continue
        lines.append("  {" + ", ".join(fmt(v) for v in gx[m][1] + [0] * (4 - m)) + "},")
    lines.append("};")
    for k in ("R5", "R7", "R9"):
        C = [[mp.mpf(c.numerator) / c.denominator for c in row] for row in maps[k]]
        lines.append(f"constexpr double kN_{k}[5][4][9] = {{  // [m][l][slot]: value at node l")
        for m in range(5):
            lines.append("  {")
            for l in range(4):
                if m < 2 or l >= m:
                    lines.append("    {" + ", ".join(["0"] * 9) + "},")
                else:
                    lines.append("    {" + ", ".join(fmt(w) for w in eval_row(C, gx[m][0][l], 0)) + "},")
            lines.append("  },")
        lines.append("};")
    lines.append("// Tangential derivative weights [m][l][r*m+q] (Sec. 3.3 Step 3, least squares of degree min(2m+1, 8)), units of xi")
    for name, idx, ty in (("kT1", 0, "double"), ("kT2", 1, "double"), ("kT1f", 0, "float"), ("kT2f", 1, "float")):
        if ty == "float":
            lines.append(f"// {name}: the same weights rounded to float (the FP32-flux variant)")
        lines.append(f"__constant__ {ty} {name}[5][4][12] = {{")
        for m in range(5):
            lines.append("  {")
            if m < 2:
                for _ in range(4):
                    lines.append("    {" + ", ".join(["0"] * 12) + "},")
            else:
                W = tangential_weights(m)[idx]
                for l in range(4):
                    row = W[l] if l < m else []
                    row = [fmt(v) for v in row] + ["0"] * (12 - len(row))
                    lines.append("    {" + ", ".join(row) + "},")
            lines.append("  },")
        lines.append("};")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cgks_tables.inc")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
