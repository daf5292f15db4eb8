"""Exact-arithmetic random walker on tiny grids — TEST INFRASTRUCTURE ONLY.

The combinatorial Dirichlet problem ``L_U x = -B^T m`` (random walker, the
paper's Sec. III-A operator) solved by Gaussian elimination over the
rationals.  Edge weights are the float64 values of exp(-beta (g_i - g_j)^2)
taken exactly as fractions, so the only rounding in the result is the final
conversion to float.  Used to write and check the fixtures in tests/golden.
"""
from __future__ import annotations

import math
from fractions import Fraction


def _neighbours(shape, v):
    nz, ny, nx = shape
    z, rem = divmod(v, ny * nx)
    y, x = divmod(rem, nx)
    for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
        zz, yy, xx = z + dz, y + dy, x + dx
        if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
            yield (zz * ny + yy) * nx + xx


def solve_exact(shape, g_flat, labels_flat, beta, label):
    """Exact x^label on every voxel (list of Fractions), seeds exact."""
    n = len(g_flat)
    U = [v for v in range(n) if labels_flat[v] == 0]
    pos = {v: k for k, v in enumerate(U)}
    m = len(U)
    A = [[Fraction(0)] * (m + 1) for _ in range(m)]
    for row, i in enumerate(U):
        for j in _neighbours(shape, i):
            d = g_flat[i] - g_flat[j]
            w = Fraction(math.exp(-beta * d * d))
            A[row][row] += w
            if labels_flat[j] == 0:
                A[row][pos[j]] -= w
            elif labels_flat[j] == label:
                A[row][m] += w
    # Gauss-Jordan elimination with exact pivots
    for c in range(m):
        piv = next(r for r in range(c, m) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        inv = 1 / A[c][c]
        A[c] = [a * inv for a in A[c]]
        for r in range(m):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    x = [Fraction(int(labels_flat[v] == label)) for v in range(n)]
    for k, i in enumerate(U):
        x[i] = A[k][m]
    return x
