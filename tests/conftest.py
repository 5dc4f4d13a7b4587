import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the GPU)")


def dense_P(g):
    """Transition matrix of Section 2 as a dense numpy array (duplicates add up)."""
    P = np.zeros((g.n, g.n))
    d = np.diff(g.row_ptr)
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            P[v, g.col[e]] += 1.0 / d[v]
    return P


def dense_ppr_matrix(g, alpha):
    """All PPR vectors as rows: Pi = alpha (I - (1-alpha) P)^-1 (Eq. 1 for every source),
    by numpy's LU solve."""
    P = dense_P(g)
    return alpha * np.linalg.solve(np.eye(g.n) - (1 - alpha) * P, np.eye(g.n))


def dense_ppr(g, s, alpha):
    """pi_s from Eq. 1 written as (I - (1-alpha) P^T) x = alpha e_s."""
    P = dense_P(g)
    e = np.zeros(g.n)
    e[s] = 1.0
    return np.linalg.solve(np.eye(g.n) - (1 - alpha) * P.T, alpha * e)
