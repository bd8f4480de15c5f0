"""First-order rounding bounds for comparing two independent FP64 evaluations of the
SEM geometry (test infrastructure: it sets no expected value, only how far two
correct evaluations may lie apart).

Both the library and the oracle form the Jacobian J = dx/dr by differentiating the
nodal coordinates with the GLL derivative matrix D (a dot product of N+1 terms per
entry), then |J|, J^{-1} and G = w |J| J^{-1} J^{-T}. With unit roundoff u:

* one J entry carries an absolute error of at most u (N+1) ||D||_inf max|x|
  (the accumulated products, plus the O(u ||D||) errors of D's own entries);
* relative to the smallest singular value of J this is u kappa with
  kappa = (N+1) ||D||_inf max|x| / sigma_min(J), and the 2-norm of the error matrix
  is at most 3 u kappa sigma_min(J);
* det J: d|J| / |J| = tr(J^{-1} dJ), at most 3 * 3 u kappa = 9 u kappa;
* G: the determinant plus two inverse factors (3 u kappa each): 15 u kappa relative
  to max|G|;
* two independent evaluations differ by at most twice that: 18 u kappa for the mass
  B = w |J| (and B lambda), 30 u kappa for G.

These are worst-case first-order bounds; rounding errors of opposite sign cancel, so
the differences observed are one to three orders of magnitude smaller.
"""
from __future__ import annotations

import numpy as np

from oracle.gll import derivative_matrix
from oracle.sem import grad_local

U = np.finfo(np.float64).eps / 2


def geometry_kappa(box) -> float:
    """kappa = (N+1) ||D||_inf max|x| / min sigma_min(J) over all nodes of an oracle SemBox."""
    N = box.N
    D = derivative_matrix(N)
    J = np.empty(box.X.shape[:4] + (3, 3))
    for d in range(3):
        ur, us, ut = grad_local(box.D, box.X[..., d])
        J[..., d, 0], J[..., d, 1], J[..., d, 2] = ur, us, ut
    smin = np.linalg.svd(J.reshape(-1, 3, 3), compute_uv=False)[:, -1].min()
    return (N + 1) * np.abs(D).sum(axis=1).max() * np.abs(box.X).max() / smin


def mass_bound(box) -> float:
    """Relative (max-norm) bound on the difference of two FP64 mass evaluations."""
    return 18.0 * U * geometry_kappa(box)


def factor_bound(box) -> float:
    """Bound on max|G_1 - G_2| / max|G| for two FP64 evaluations of the factors."""
    return 30.0 * U * geometry_kappa(box)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """x rounded to bfloat16 (through float32, round to nearest, ties to even), returned
    as float64: the storage rounding of the mixed cycle's geometric factors, applied to
    the oracle's factors to separate that rounding from the FP32 arithmetic."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
