"""FP64 CPU oracle for Householder Dice -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library never calls it, and it
imports nothing from the product package.

``hd_oracle.c`` holds Algorithms 1 and 2 of Lu, "Householder Dice" (Sec. 3.2,
Sec. 3.3) with reflectors applied one at a time; this module is the ctypes
wrapper plus the dynamics maps f_t of eq. (dynamics) used by the workloads.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

GINIBRE = 0
HAAR = 1
SIDE_R = 0
SIDE_L = 1


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp, i64, i32, u32, dbl = (ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int, ctypes.c_uint32,
                                  ctypes.c_double)
        L.hdo_new.restype = vp
        L.hdo_new.argtypes = [i32, i64, i64, i32, u32, u32, dbl]
        L.hdo_delete.argtypes = [vp]
        L.hdo_delete.restype = None
        L.hdo_query.argtypes = [vp, i32, vp, vp]
        L.hdo_query.restype = i32
        L.hdo_counts.argtypes = [vp, vp, vp, vp]
        L.hdo_counts.restype = None
        L.hdo_force_sign.argtypes = [vp, i32, i32, i32]
        L.hdo_force_sign.restype = i32
        L.hdo_reflector.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.hdo_reflector.restype = i32
        L.hdo_basis.argtypes = [vp, i32, vp, vp]
        L.hdo_basis.restype = i32
        L.hdo_philox4x32_10.argtypes = [vp, vp, vp]
        L.hdo_philox4x32_10.restype = None
        L.hdo_normals.argtypes = [u32, u32, u32, u32, i64, i64, vp]
        L.hdo_normals.restype = None
        L.hdo_apply_householder.argtypes = [vp, i64, vp, vp, i32]
        L.hdo_apply_householder.restype = i32
        # complex HD (hd_cplx_oracle.c)
        L.hdoc_normals.argtypes = [u32, u32, u32, u32, i64, i64, vp]
        L.hdoc_normals.restype = None
        L.hdoc_apply_householder.argtypes = [vp, i64, vp, i32, vp]
        L.hdoc_apply_householder.restype = i32
        L.hdoc_new.restype = vp
        L.hdoc_new.argtypes = [i32, i64, i64, i32, u32, u32, dbl]
        L.hdoc_delete.argtypes = [vp]
        L.hdoc_delete.restype = None
        L.hdoc_query.argtypes = [vp, i32, vp, vp]
        L.hdoc_query.restype = i32
        L.hdoc_counts.argtypes = [vp, vp, vp, vp]
        L.hdoc_counts.restype = None
        L.hdoc_reflector.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.hdoc_reflector.restype = i32
        L.hdoc_basis.argtypes = [vp, i32, vp, vp]
        L.hdoc_basis.restype = i32
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().hdo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed, trial, step, tag, i0, count):
    """Normals i0..i0+count-1 of the stream (seed, trial, step, tag)."""
    out = np.empty(int(count), dtype=np.float64)
    if count:
        lib().hdo_normals(seed, trial, step, tag, int(i0), int(count),
                          _ptr(out))
    return out


def apply_householder(v, z, forced_sign=0):
    """H(v) z with H of eq. (Householder); returns (result, is_identity)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty_like(z)
    ident = lib().hdo_apply_householder(_ptr(v), v.size, _ptr(z), _ptr(out),
                                        int(forced_sign))
    if ident < 0:
        raise MemoryError
    return out, bool(ident)


class HDOracle:
    """Lazy random matrix Q (Ginibre GE(m,n) scaled by sigma, or Haar O(n))
    answering y = Q x and y = Q' x by Algorithm 1 / Algorithm 2."""

    def __init__(self, ensemble, n, m=None, tmax=None, seed=0, trial=0,
                 sigma=1.0):
        m = n if m is None else m
        if tmax is None:
            tmax = min(m, n)
        self.ensemble, self.m, self.n, self.tmax = ensemble, m, n, tmax
        self.seed, self.trial, self.sigma = seed, trial, sigma
        self._h = lib().hdo_new(ensemble, m, n, tmax, seed, trial, sigma)
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().hdo_delete(h)
            self._h = None

    def query(self, x, transpose=False):
        din, dout = (self.m, self.n) if transpose else (self.n, self.m)
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.shape != (din,):
            raise ValueError("x has shape %s, expected (%d,)" % (x.shape, din))
        y = np.empty(dout, dtype=np.float64)
        rc = lib().hdo_query(self._h, int(bool(transpose)), _ptr(x), _ptr(y))
        if rc == -2:
            raise OverflowError("HD capacity exhausted")
        if rc != 0:
            raise MemoryError
        return y

    def mv(self, x):
        return self.query(x, False)

    def rmv(self, x):
        return self.query(x, True)

    def counts(self):
        t, r, l = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib().hdo_counts(self._h, ctypes.byref(t), ctypes.byref(r),
                         ctypes.byref(l))
        return t.value, r.value, l.value

    def force_sign(self, side, index1, s):
        if lib().hdo_force_sign(self._h, side, index1, int(s)) != 0:
            raise IndexError(index1)

    def reflector(self, side, index1):
        """Reflector `index1` (1-based) of side SIDE_R / SIDE_L as a dict with
        k, u (length dim-k+1), tau, s, nu, pivot, ident."""
        dim = self.n if side == SIDE_R else self.m
        u = np.zeros(dim - index1 + 1, dtype=np.float64)
        tau, nu, piv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        s, ident = ctypes.c_int(), ctypes.c_int()
        rc = lib().hdo_reflector(self._h, side, index1, _ptr(u),
                                 ctypes.byref(tau), ctypes.byref(s),
                                 ctypes.byref(nu), ctypes.byref(piv),
                                 ctypes.byref(ident))
        if rc != 0:
            raise IndexError(index1)
        return dict(k=index1, u=u, tau=tau.value, s=s.value, nu=nu.value,
                    pivot=piv.value, ident=bool(ident.value))

    def basis(self, step1):
        u = np.empty(self.m, dtype=np.float64)
        v = np.empty(self.n, dtype=np.float64)
        if lib().hdo_basis(self._h, step1, _ptr(u), _ptr(v)) != 0:
            raise IndexError(step1)
        return u, v


# ---------------------------------------------------------------------
# Complex HD (Sec. 3.4): complex Ginibre and the unitary group U(n).
# ---------------------------------------------------------------------

def cnormals(seed, trial, step, tag, i0, count):
    """Complex normals i0..i0+count-1: (N_2i + i N_2i+1) / sqrt(2) from the
    real stream (seed, trial, step, tag)."""
    out = np.empty(int(count), dtype=np.complex128)
    if count:
        lib().hdoc_normals(seed, trial, step, tag, int(i0), int(count),
                           _ptr(out))
    return out


def capply_householder(v, z, adjoint=False):
    """H(v) z (or H(v)^H z) with the unitary reflector of eq.
    (Householder_c); returns (result, is_identity)."""
    v = np.ascontiguousarray(v, dtype=np.complex128)
    z = np.ascontiguousarray(z, dtype=np.complex128)
    out = np.empty_like(z)
    ident = lib().hdoc_apply_householder(_ptr(v), v.size, _ptr(z),
                                         int(bool(adjoint)), _ptr(out))
    if ident < 0:
        raise MemoryError
    return out, bool(ident)


class CHDOracle:
    """Lazy complex random matrix Q (complex Ginibre, E|Q_ij|^2 = sigma^2, or
    Haar on U(n)) answering y = Q x and y = Q^H x."""

    def __init__(self, ensemble, n, m=None, tmax=None, seed=0, trial=0,
                 sigma=1.0):
        m = n if m is None else m
        if tmax is None:
            tmax = min(m, n)
        self.ensemble, self.m, self.n, self.tmax = ensemble, m, n, tmax
        self.seed, self.trial, self.sigma = seed, trial, sigma
        self._h = lib().hdoc_new(ensemble, m, n, tmax, seed, trial, sigma)
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().hdoc_delete(h)
            self._h = None

    def query(self, x, adjoint=False):
        din, dout = (self.m, self.n) if adjoint else (self.n, self.m)
        x = np.ascontiguousarray(x, dtype=np.complex128)
        if x.shape != (din,):
            raise ValueError("x has shape %s, expected (%d,)" % (x.shape, din))
        y = np.empty(dout, dtype=np.complex128)
        rc = lib().hdoc_query(self._h, int(bool(adjoint)), _ptr(x), _ptr(y))
        if rc == -2:
            raise OverflowError("HD capacity exhausted")
        if rc != 0:
            raise MemoryError
        return y

    def mv(self, x):
        return self.query(x, False)

    def rmv(self, x):
        return self.query(x, True)

    def counts(self):
        t, r, l = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lib().hdoc_counts(self._h, ctypes.byref(t), ctypes.byref(r),
                          ctypes.byref(l))
        return t.value, r.value, l.value

    def reflector(self, side, index1):
        """Reflector `index1` (1-based) of a side: dict with k, w (length
        dim - k + 1), r, theta, nu, pivot, ident."""
        dim = self.n if side == SIDE_R else self.m
        w = np.zeros(dim - index1 + 1, dtype=np.complex128)
        r, th, nu = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        piv = np.zeros(1, dtype=np.complex128)
        ident = ctypes.c_int()
        rc = lib().hdoc_reflector(self._h, side, index1, _ptr(w),
                                  ctypes.byref(r), ctypes.byref(th),
                                  ctypes.byref(nu), _ptr(piv),
                                  ctypes.byref(ident))
        if rc != 0:
            raise IndexError(index1)
        return dict(k=index1, w=w, r=r.value, theta=th.value, nu=nu.value,
                    pivot=complex(piv[0]), ident=bool(ident.value))

    def basis(self, step1):
        u = np.empty(self.m, dtype=np.complex128)
        v = np.empty(self.n, dtype=np.complex128)
        if lib().hdoc_basis(self._h, step1, _ptr(u), _ptr(v)) != 0:
            raise IndexError(step1)
        return u, v


def f_ctanh(y, x_t, a, b):
    """Complex map x_{t+1} = tanh(a |y|) e^{i arg y} + b x_t (0 where y = 0),
    the complex workload's stand-in for the real tanh map."""
    mag = np.abs(y)
    ph = np.where(mag > 0, y / np.where(mag > 0, mag, 1.0), 0.0)
    return np.tanh(a * mag) * ph + b * x_t


def run_ctrajectory(orc, x1, T, a, b, pattern="Q"):
    """Free-running complex trajectory: X (T+1 rows) and Y (T rows);
    pattern "Q" or "alt" (Q, Q^H, Q, ...; square Q only)."""
    X = [np.asarray(x1, dtype=np.complex128)]
    Y = []
    for t in range(T):
        adj = pattern == "alt" and t % 2 == 1
        y = orc.query(X[-1], adj)
        Y.append(y)
        X.append(f_ctanh(y, X[-1], a, b))
    return np.array(X), np.array(Y)


# ---------------------------------------------------------------------
# Dynamics maps f_t of eq. (dynamics) used by the workloads (FP64).
# ---------------------------------------------------------------------

def soft_threshold(v, theta):
    """Element-wise soft threshold eta_theta(v) = sign(v) max(|v|-theta, 0)
    (the operator in eq. (ista))."""
    return np.sign(v) * np.maximum(np.abs(v) - theta, 0.0)


def f_tanh_affine(y, x_t, x_prev, a, b):
    """x_{t+1} = tanh(a y) + b x_t."""
    return np.tanh(a * y) + b * x_t


def f_soft_hist(y, x_t, x_prev, a, b):
    """x_{t+1} = soft_threshold(y, a) + b x_{t-1}."""
    return soft_threshold(y, a) + b * x_prev


def f_normalize(y, x_t, x_prev, a, b):
    """x_{t+1} = y / ||y|| + b x_t."""
    return y / np.linalg.norm(y) + b * x_t


DYNAMICS = {"tanh": f_tanh_affine, "soft_hist": f_soft_hist,
            "normalize": f_normalize}


def run_trajectory(orc, x1, T, dyn, a, b, pattern="Q", x0=None,
                   state_dtype=None):
    """Free-running trajectory (Mode A): returns X (T+1 rows: x_1..x_{T+1})
    and Y (T rows).  pattern "Q" = every query uses Q, "alt" = Q, Q', Q, ...

    state_dtype=np.float32 rounds y_t and x_{t+1} to that type after each
    step (the queries stay FP64): the divergence of that run from the FP64
    one measures how much the dynamics themselves amplify storage rounding,
    independent of any implementation of the queries."""
    f = DYNAMICS[dyn]
    rnd = (lambda v: v) if state_dtype is None else \
        (lambda v: np.asarray(v, state_dtype).astype(np.float64))
    x_t = rnd(np.asarray(x1, dtype=np.float64))
    x_prev = np.zeros_like(x_t) if x0 is None else np.asarray(x0, np.float64)
    X, Y = [x_t.copy()], []
    for t in range(T):
        transpose = (pattern == "alt" and t % 2 == 1)
        y = rnd(orc.query(x_t, transpose))
        x_next = rnd(f(y, x_t, x_prev, a, b))
        X.append(x_next)
        Y.append(y)
        x_prev, x_t = x_t, x_next
    return np.array(X), np.array(Y)


def goe_query(orc, x):
    """y = G x for G = (Q + Q') / sqrt(2) ~ sigma GOE(n) (section "Other
    Random Matrix Ensembles"): the lazy square Gaussian Q answers
    y_hat = Q x, then y = (Q' x + y_hat) / sqrt(2)."""
    y_hat = orc.query(np.asarray(x, np.float64), False)
    return (orc.query(np.asarray(x, np.float64), True) + y_hat) / np.sqrt(2.0)


def usv_query(orc_u, orc_v, s, x, transpose=False):
    """Q = U S V with U ~ Haar(m), V ~ Haar(n) independent lazy matrices and
    S the m x n matrix with diagonal s (min(m, n) entries) and zeros
    elsewhere (section "Other Random Matrix Ensembles"):
    Q x = U (S (V x)) and Q' x = V' (S' (U' x))."""
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    m, n = orc_u.n, orc_v.n
    p = min(m, n)
    if transpose:
        u = orc_u.query(x, True)
        w = np.zeros(n)
        w[:p] = s[:p] * u[:p]
        return orc_v.query(w, True)
    v = orc_v.query(x, False)
    w = np.zeros(m)
    w[:p] = s[:p] * v[:p]
    return orc_u.query(w, False)


def spectral_power(orc, xi, x1, K, scale=1.0):
    """Spectral method of Sec. 2.2 on a lazy Haar Q of size m (the oracle
    `orc`), with A = [I_n 0] Q (eq. (A_ortho)), measurements
    y_i = tanh|a_i' xi| and D = (1/m) A diag(y) A' (eq. (D_mtx)).

    The measurements take one query: A' xi = Q' [xi; 0].  Each power step
    x_{k+1} = scale * m * D x_k takes two: u = Q' [x_k; 0], then
    v = Q (y * u), of which x_{k+1} keeps the first n entries (times scale).
    Returns (A' xi, X) with X = [x_1, ..., x_{K+1}]."""
    xi = np.asarray(xi, np.float64)
    n = xi.size
    m = orc.n
    pad = np.zeros(m - n)
    z = orc.query(np.concatenate([xi, pad]), True)
    y = np.tanh(np.abs(z))
    x = np.asarray(x1, np.float64)
    X = [x]
    for _ in range(K):
        u = orc.query(np.concatenate([x, pad]), True)
        v = orc.query(y * u, False)
        x = scale * v[:n]
        X.append(x)
    return z, np.array(X)


def replay(orc, xs, transposes):
    """Mode B: answer the given query vectors in order; returns the outputs."""
    return [orc.query(np.asarray(x, np.float64), bool(tr))
            for x, tr in zip(xs, transposes)]


# ---------------------------------------------------------------------
# Unrolled ISTA with learned per-layer step and threshold, and its
# gradient with the lazy matrix held fixed.
#
# Layer t (eq. (ista) with tau -> a_t and lambda tau -> theta_t):
#     u_t = Q'(y - Q x_t),  v_t = x_t + a_t u_t,  x_{t+1} = eta_{theta_t}(v_t).
# Every product with Q or Q' is a query on the same lazy matrix, so Q is one
# fixed (if partly unrevealed) matrix throughout; the backward pass below is
# plain reverse-mode calculus for that fixed Q, whose two matrix products per
# layer are further queries.
# ---------------------------------------------------------------------

def lista_forward(orc, x1, y, a, theta):
    """Layers t = 1..L (L = len(a)); returns X (L+1 rows, X[0] = x1),
    U (L rows, u_t) and V (L rows, v_t).  2L queries: Q x_t, then Q'(.)."""
    x = np.asarray(x1, np.float64)
    y = np.asarray(y, np.float64)
    X, U, V = [x], [], []
    for at, th in zip(a, theta):
        r = orc.query(x, False)
        u = orc.query(y - r, True)
        v = x + at * u
        x = soft_threshold(v, th)
        X.append(x)
        U.append(u)
        V.append(v)
    return np.array(X), np.array(U), np.array(V)


def lista_backward(orc, g, a, theta, U, V, need_x1=False):
    """Reverse pass for dL/dx_{L+1} = g.  With the threshold mask
    m_t = [|v_t| > theta_t]:
        dL/dtheta_t = -sum(g * sign(v_t) * m_t),
        gbar = g * m_t,  dL/da_t = sum(gbar * u_t),
        dL/dx_t = gbar - a_t Q'Q gbar   (two queries: Q gbar, then Q'(.)).
    The last product (t = 1) runs only when need_x1.  Returns
    (da, dtheta, dL/dx_1 or None)."""
    L = len(a)
    g = np.asarray(g, np.float64)
    da = np.zeros(L)
    dth = np.zeros(L)
    for t in range(L - 1, -1, -1):
        m = np.abs(V[t]) > theta[t]
        dth[t] = -np.sum(g * np.sign(V[t]) * m)
        gbar = g * m
        da[t] = np.sum(gbar * U[t])
        if t == 0 and not need_x1:
            return da, dth, None
        q = orc.query(gbar, False)
        w = orc.query(q, True)
        g = gbar - a[t] * w
    return da, dth, g
