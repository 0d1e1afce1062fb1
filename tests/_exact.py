"""Exact polynomial integration over triangles, independent of any quadrature rule.

A monomial (x - x0)^p (y - y0)^q is pulled back to the reference triangle through the affine map
x = a + s (b - a) + t (c - a), expanded in (s, t), and integrated term by term with
int_ref s^i t^j ds dt = i! j! / (i + j + 2)!.
"""
from math import factorial

import numpy as np
from scipy.signal import convolve2d


def _lin(c0, cs, ct):
    P = np.zeros((2, 2))
    P[0, 0], P[1, 0], P[0, 1] = c0, cs, ct
    return P


def _pow(P, n):
    R = np.ones((1, 1))
    for _ in range(n):
        R = convolve2d(R, P)
    return R


_REF = {}


def _ref_avg(i, j):
    key = (i, j)
    if key not in _REF:
        _REF[key] = 2.0 * factorial(i) * factorial(j) / factorial(i + j + 2)
    return _REF[key]


def mono_avg(tri_xy, x0, p, q):
    """Average of (x - x0[0])^p (y - x0[1])^q over the triangle with vertices tri_xy[3, 2]."""
    a, b, c = np.asarray(tri_xy, dtype=np.float64)
    X = _lin(a[0] - x0[0], b[0] - a[0], c[0] - a[0])
    Y = _lin(a[1] - x0[1], b[1] - a[1], c[1] - a[1])
    C = convolve2d(_pow(X, p), _pow(Y, q))
    tot = 0.0
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            if C[i, j] != 0.0:
                tot += C[i, j] * _ref_avg(i, j)
    return tot


def poly_avg(tri_xy, coeffs):
    """Average over a triangle of sum c_pq x^p y^q, coeffs = {(p, q): c}."""
    return sum(c * mono_avg(tri_xy, (0.0, 0.0), p, q) for (p, q), c in coeffs.items())


def poly_eval(coeffs, x, y):
    return sum(c * x ** p * y ** q for (p, q), c in coeffs.items())


def poly_grad(coeffs, x, y):
    gx = sum(c * p * x ** (p - 1) * y ** q for (p, q), c in coeffs.items() if p > 0)
    gy = sum(c * q * x ** p * y ** (q - 1) for (p, q), c in coeffs.items() if q > 0)
    return gx, gy
