"""FP64 oracle of the Lanczos condition-number estimate (Sec. 6.4).

TEST INFRASTRUCTURE ONLY (see fill_oracle).

The paper sizes its solves by a Lanczos estimate of the condition number:
the Krylov space that CG builds carries a tridiagonal matrix whose extreme
eigenvalues (found with a QR method) approach those of the operator.  CG's
own coefficients give that matrix directly (the CG-Lanczos relation, Golub
and Van Loan, "Matrix Computations", Sec. 10.2): with step lengths alpha_j
and direction coefficients beta_j = rho_{j+1} / rho_j,

    T[j, j]     = 1 / alpha_j + beta_{j-1} / alpha_{j-1}   (second term absent for j = 0)
    T[j, j + 1] = sqrt(beta_j) / alpha_j.

For preconditioned CG the matrix belongs to the preconditioned operator
(here E A E, whose eigenvalues are those of M^-1 A with M^-1 = E E); for
plain CG to A.  Its eigenvalues (Ritz values) always lie inside the
operator's spectrum.
"""

from __future__ import annotations

import numpy as np

__all__ = ["lanczos_tridiagonal", "ritz_values", "condition_estimate"]


def lanczos_tridiagonal(alphas, betas) -> tuple[np.ndarray, np.ndarray]:
    """(diagonal, off-diagonal) of the k x k Lanczos matrix of k CG steps.

    alphas has k entries; betas at least k - 1 (extra entries are ignored).
    """
    a = np.asarray(alphas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    k = len(a)
    if k == 0:
        return np.zeros(0), np.zeros(0)
    if len(b) < k - 1:
        raise ValueError("need k - 1 direction coefficients for k step lengths")
    b = b[:k - 1]
    diag = 1.0 / a
    diag[1:] += b / a[:-1]
    off = np.sqrt(b) / a[:-1]
    return diag, off


def ritz_values(alphas, betas) -> np.ndarray:
    """Eigenvalues of the Lanczos matrix, ascending (LAPACK's symmetric QR)."""
    diag, off = lanczos_tridiagonal(alphas, betas)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    return np.linalg.eigvalsh(T)


def condition_estimate(alphas, betas) -> tuple[float, float, float]:
    """(lambda_min, lambda_max, kappa) from the extreme Ritz values."""
    ev = ritz_values(alphas, betas)
    return float(ev[0]), float(ev[-1]), float(ev[-1] / ev[0])
