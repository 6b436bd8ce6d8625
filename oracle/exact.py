"""Exact rational arithmetic for tiny cases -- TEST INFRASTRUCTURE ONLY.

These routines pin the FP64 oracle to something other than itself: with
``fractions.Fraction`` every operation is exact, so a dense mat-vec, Gaussian
elimination and conjugate gradients give the mathematically exact result
(CG then terminates with r = 0 in at most n steps, a property of the method
in exact arithmetic).
"""
from __future__ import annotations

from fractions import Fraction


def frac_vec(v):
    return [Fraction(float(t)) for t in v]


def frac_mat(D):
    return [[Fraction(float(t)) for t in row] for row in D]


def matvec(A, x):
    """Exact y = A x for dense Fraction lists."""
    return [sum((a * b for a, b in zip(row, x)), Fraction(0)) for row in A]


def solve(A, b):
    """Exact Gaussian elimination with row pivoting on the first nonzero."""
    n = len(A)
    M = [list(r) + [bb] for r, bb in zip(A, b)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [u - f * v for u, v in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def cg(A, b, dinv=None, max_iters=None):
    """Exact (preconditioned) CG from x0 = 0.  Returns (x, iterations, r).

    Stops as soon as the residual is exactly zero.
    """
    n = len(A)
    max_iters = n if max_iters is None else max_iters
    x = [Fraction(0)] * n
    r = list(b)
    z = [d * t for d, t in zip(dinv, r)] if dinv else list(r)
    p = list(z)
    rho = sum((u * v for u, v in zip(r, z)), Fraction(0))
    k = 0
    while any(t != 0 for t in r) and k < max_iters:
        q = matvec(A, p)
        eta = sum((u * v for u, v in zip(p, q)), Fraction(0))
        alpha = rho / eta
        x = [u + alpha * v for u, v in zip(x, p)]
        r = [u - alpha * v for u, v in zip(r, q)]
        k += 1
        if all(t == 0 for t in r):
            break
        z = [d * t for d, t in zip(dinv, r)] if dinv else list(r)
        rho_new = sum((u * v for u, v in zip(r, z)), Fraction(0))
        p = [u + (rho_new / rho) * v for u, v in zip(z, p)]
        rho = rho_new
    return x, k, r
