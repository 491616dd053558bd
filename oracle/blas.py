"""Level-1 operations on spin-colour fields, FP64 (test infrastructure only).

Sec. 4 of the paper analyses caxpy: c*psi + psi' with complex c on complex
spin-colour vectors.  The solvers also need xpay, inner products and norms.
"""
import numpy as np


def caxpy(c, x, y):
    """c*x + y."""
    return c * x + y


def xpay(x, a, y):
    """x + a*y."""
    return x + a * y


def cdot(x, y):
    """<x, y> = sum conj(x) y."""
    return complex(np.sum(np.conj(x) * y))


def norm2(x):
    return float(np.sum(x.real * x.real + x.imag * x.imag))
