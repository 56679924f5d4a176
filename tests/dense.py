"""Dense-matrix helpers for the tests (tiny sizes only).

These build matrices straight from their definitions so that the lazy
algorithms can be checked against explicit linear algebra.
"""
import numpy as np


def reflector_matrix(dim, refl):
    """Dense H_k(p) of eq. (Householder_e) from an exported reflector:
    diag(I_{k-1}, -s (I - tau u u'))."""
    H = np.eye(dim)
    if refl["ident"]:
        return H
    k = refl["k"]
    u = refl["u"]
    blk = -refl["s"] * (np.eye(u.size) - refl["tau"] * np.outer(u, u))
    H[k - 1:, k - 1:] = blk
    return H


def haar_dense(n, rng):
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of R's diagonal moved into Q (Mezzadri 2007)."""
    A = rng.standard_normal((n, n))
    Qm, Rm = np.linalg.qr(A)
    return Qm * np.sign(np.diag(Rm))[None, :]


def r_factor_positive(X):
    """R factor of the thin QR of X (columns x_1..x_t) with positive diagonal."""
    _, Rm = np.linalg.qr(X)
    sg = np.sign(np.diag(Rm))
    sg[sg == 0] = 1.0
    return Rm * sg[:, None]
