"""Exact rational integration of polynomials over simplices (test helper).

A polynomial in (x, y, z) is a dict {(a, b, c): Fraction}.  Over a simplex
with vertices V_0..V_d, substituting x = sum_i lam_i V_i turns it into a
polynomial in the barycentric coordinates, which is integrated with the
Dirichlet formula

    int_S prod_i lam_i^{k_i} dS = d! |S| prod_i k_i! / (sum_i k_i + d)!.

Used to pin the oracle against closed forms; shares nothing with it.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction as Fr


def poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return out


def poly_pow(p, n, nvar):
    out = {(0,) * nvar: Fr(1)}
    for _ in range(n):
        out = poly_mul(out, p)
    return out


def monomial(a, b, c):
    return {(a, b, c): Fr(1)}


def eval_poly(p, X):
    import numpy as np
    X = np.asarray(X, dtype=float)
    out = np.zeros(X.shape[:-1])
    for (a, b, c), coef in p.items():
        out = out + float(coef) * X[..., 0] ** a * X[..., 1] ** b * X[..., 2] ** c
    return out


def integrate(p, verts, measure):
    """Integral of polynomial p over the simplex with the given vertices.

    measure: the simplex volume (or area) in the chosen measure.
    """
    d = len(verts) - 1
    nl = d + 1
    # each coordinate as a linear polynomial in lam
    coords = []
    for axis in range(3):
        lin = {}
        for i, v in enumerate(verts):
            e = tuple(1 if j == i else 0 for j in range(nl))
            lin[e] = lin.get(e, 0) + Fr(v[axis])
        coords.append(lin)
    total = Fr(0)
    for (a, b, c), coef in p.items():
        term = poly_mul(poly_mul(poly_pow(coords[0], a, nl), poly_pow(coords[1], b, nl)),
                        poly_pow(coords[2], c, nl))
        for e, ce in term.items():
            num = math.factorial(d) * math.prod(math.factorial(k) for k in e)
            den = math.factorial(sum(e) + d)
            total += coef * ce * Fr(num, den)
    return total * Fr(measure)


REF_TET = [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
REF_VOL = Fr(4, 3)


def monomials(deg):
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a) for c in range(deg + 1 - a - b)]


def exps_upto(deg):
    return list(itertools.chain.from_iterable(monomials(deg) for _ in [0]))
