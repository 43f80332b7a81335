"""Brute-force vertex enumeration for tiny standard-form LPs (test helper).

Every basis B (m linearly independent columns) gives the basic solution
x_B = A_B^{-1} b (primal vertex if x_B >= 0) and the dual basic solution
y = A_B^{-T} c_B (dual vertex if A^T y <= c).  The LP optimum is the minimum
of c^T x over primal vertices; by strong duality it equals the maximum of
b^T y over dual vertices.
"""
import itertools

import numpy as np


def enumerate_vertices(A, b, c, tol=1e-9):
    m, n = A.shape
    pv, dv = [], []
    for B in itertools.combinations(range(n), m):
        AB = A[:, B]
        if abs(np.linalg.det(AB)) < 1e-12:
            continue
        xB = np.linalg.solve(AB, b)
        if np.all(xB >= -tol):
            x = np.zeros(n)
            x[list(B)] = xB
            pv.append(x)
        y = np.linalg.solve(AB.T, c[list(B)])
        if np.all(A.T @ y <= c + tol):
            dv.append(y)
    return pv, dv


def lp_optimum(A, b, c):
    pv, dv = enumerate_vertices(A, b, c)
    p = min(float(c @ x) for x in pv)
    d = max(float(b @ y) for y in dv)
    return p, d, pv, dv
