"""Oracle: extreme eigenvalues of the reduced operator (conditioning).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper stops CG on the residual (section "Matrix-Free Conjugate Gradient with
Multiple Constraint Enforcement"); how far a given residual is from the solution
depends on the condition number of A = T^T K T.  Two quantities:

* ``condition_number(A)`` -- lambda_min, lambda_max and their ratio for the whole
  operator: the plain definition, by a dense symmetric eigensolver on small
  systems, and by ARPACK (largest eigenvalue directly, smallest by shift-invert
  about zero, which factors A) on large ones;
* ``lanczos_extremes(A, b, m)`` -- the extreme eigenvalues of the m x m Lanczos
  tridiagonal of A started from b (plain three-term recurrence in FP64, no
  reorthogonalisation): the Ritz values of the Krylov space that CG on A y = b
  explores.  CG's step lengths and direction factors (Algorithm 1's alpha and
  beta) define the same tridiagonal, so this is what a condition estimate from a
  CG solve converges to.  Eigenvectors that b barely touches show late: for a
  mirror-symmetric layout b is odd in y and only rounding gives it weight on the
  even eigenvectors (among them the one of lambda_min), which the recurrence then
  finds after more steps than the odd extremes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

DENSE_MAX = 4000


def condition_number(A):
    """(lambda_min, lambda_max, lambda_max / lambda_min) of the symmetric positive
    definite matrix A."""
    n = A.shape[0]
    if n <= DENSE_MAX:
        w = np.linalg.eigvalsh(A.toarray() if hasattr(A, "toarray") else np.asarray(A))
        lmin, lmax = float(w[0]), float(w[-1])
    else:
        lmax = float(spla.eigsh(A, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0])
        lmin = float(spla.eigsh(A.tocsc(), k=1, sigma=0.0, which="LM",
                                return_eigenvectors=False, tol=1e-10)[0])
    return lmin, lmax, lmax / lmin


def lanczos_tridiagonal(A, b, m):
    """Diagonal a[0..k) and off-diagonal c[0..k-1) of the Lanczos tridiagonal of A
    from q_1 = b / |b|: A q_j = c_(j-1) q_(j-1) + a_j q_j + c_j q_(j+1).  Stops early
    (k < m) if the next vector vanishes."""
    q_prev = np.zeros_like(b, dtype=np.float64)
    q = np.asarray(b, dtype=np.float64) / np.linalg.norm(b)
    a, c = [], []
    beta = 0.0
    for _ in range(m):
        v = A @ q - beta * q_prev
        alpha = float(q @ v)
        v -= alpha * q
        a.append(alpha)
        beta = float(np.linalg.norm(v))
        if len(a) == m or beta == 0.0:
            break
        c.append(beta)
        q_prev, q = q, v / beta
    return np.array(a), np.array(c)


def lanczos_extremes(A, b, m):
    """(smallest, largest) eigenvalue of the m-step Lanczos tridiagonal of A from b."""
    a, c = lanczos_tridiagonal(A, b, m)
    w = sla.eigvalsh_tridiagonal(a, c)
    return float(w[0]), float(w[-1])
