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


def ginibre_rec(orc, m, n, sigma, W):
    """Dense Q consistent with every answer the lazy Gaussian matrix gave
    (eq. (Gaussian_t)): sigma (sum_i u_i v_i' + L_1..L_l Z W Z R_r..R_1) for
    an arbitrary m x n matrix W."""
    from oracle import SIDE_L, SIDE_R
    t, r, l = orc.counts()
    S = np.zeros((m, n))
    for i in range(1, t + 1):
        u, v = orc.basis(i)
        S += np.outer(u, v)
    Lm = np.eye(m)
    for i in range(1, l + 1):
        Lm = Lm @ reflector_matrix(m, orc.reflector(SIDE_L, i))
    Rm = np.eye(n)
    for i in range(1, r + 1):
        Rm = reflector_matrix(n, orc.reflector(SIDE_R, i)) @ Rm
    Zl = np.diag(np.r_[np.zeros(l), np.ones(m - l)])
    Zr = np.diag(np.r_[np.zeros(r), np.ones(n - r)])
    return sigma * (S + Lm @ Zl @ W @ Zr @ Rm)
