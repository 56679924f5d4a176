"""Householder Dice on MI355X (gfx950).

``LazyMatrix`` wraps one handle of libhd.so: a Ginibre or Haar random matrix Q
that is never formed and answers ``y = Q x`` / ``y = Q' x`` on torch CUDA
tensors (Lu, "Householder Dice", Algorithms 1 and 2).  The binding only
marshals arguments; all work runs in the library's HIP kernels on the
tensor's current stream.
"""
import ctypes

from . import _lib
from ._lib import (HD_F32, HD_F64, HD_GINIBRE, HD_HAAR, HD_DYN_NORMALIZE,
                   HD_DYN_SOFT_HIST, HD_DYN_TANH, HD_PATTERN_ALT, HD_PATTERN_Q,
                   HDCapacityError, HDError)

GINIBRE = HD_GINIBRE
HAAR = HD_HAAR

_DYN = {"tanh": HD_DYN_TANH, "soft_hist": HD_DYN_SOFT_HIST,
        "normalize": HD_DYN_NORMALIZE}
_PATTERN = {"Q": HD_PATTERN_Q, "alt": HD_PATTERN_ALT}


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class LazyMatrix:
    """Lazy m x n random matrix on one GPU.

    ensemble: GINIBRE (entries N(0, sigma^2)) or HAAR (orthogonal, m = n).
    dtype: torch.float32 or torch.float64 (panel and vector storage).
    t_max: number of queries the handle can answer (<= min(m, n)).
    """

    def __init__(self, ensemble, n, m=None, t_max=None, seed=0, trial=0,
                 sigma=1.0, dtype=None, device="cuda:0", state=None):
        torch = _torch()
        m = n if m is None else m
        t_max = min(m, n) if t_max is None else t_max
        dtype = torch.float32 if dtype is None else dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be float32 or float64")
        self.ensemble, self.m, self.n, self.t_max = ensemble, m, n, t_max
        self.dtype = dtype
        self.device = torch.device(device)
        cfg = _lib.HDConfig(ensemble, HD_F64 if dtype == torch.float64
                            else HD_F32, m, n, t_max, seed, trial, sigma,
                            _stream_ptr(self.device))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if state is None:
                _lib.check(_lib.load().hd_init(ctypes.byref(cfg),
                                               ctypes.byref(h)), "hd_init")
            else:
                import numpy as np
                buf = np.ascontiguousarray(state, dtype=np.uint8)
                _lib.check(_lib.load().hd_import(
                    ctypes.byref(cfg), buf.ctypes.data_as(ctypes.c_void_p),
                    buf.nbytes, ctypes.byref(h)), "hd_import")
        self._h = h

    def goe_mv(self, x):
        """y = (Q x + Q' x)/sqrt(2) (``hd_goe_step``): G x for the GOE matrix
        G = (Q + Q')/sqrt(2) of a square Gaussian handle, two queries.  See
        ``LazyGOE``."""
        torch = _torch()
        x = self._vec(x, self.n)
        y = torch.empty(self.n, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _lib.check(_lib.load().hd_goe_step(self._h,
                                           ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr())),
                   "hd_goe_step")
        return y

    def export_state(self):
        """The handle's state as a numpy uint8 array (``hd_export``); pass it
        as ``state=`` with the same ensemble, sizes, t_max, sigma and dtype
        to continue the same realisation in a new handle."""
        import numpy as np
        L = _lib.load()
        self._sync_stream()
        size = ctypes.c_size_t(0)
        _lib.check(L.hd_export(self._h, None, ctypes.byref(size)), "hd_export")
        buf = np.empty(size.value, dtype=np.uint8)
        _lib.check(L.hd_export(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(size)), "hd_export")
        return buf

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().hd_free(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _lib.check(_lib.load().hd_set_stream(self._h,
                                             _stream_ptr(self.device)),
                   "hd_set_stream")

    def _vec(self, x, size):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or x.device != self.device:
            raise TypeError("expected a tensor on %s" % self.device)
        if x.dtype != self.dtype or x.shape != (size,):
            raise ValueError("expected shape (%d,) and dtype %s" %
                             (size, self.dtype))
        return x.contiguous()

    def mv(self, x, out=None):
        """y = Q x (one query with M_t = Q)."""
        return self._query(x, out, False)

    def rmv(self, x, out=None):
        """y = Q' x (one query with M_t = Q')."""
        return self._query(x, out, True)

    def _query(self, x, out, transpose):
        torch = _torch()
        din, dout = (self.m, self.n) if transpose else (self.n, self.m)
        x = self._vec(x, din)
        y = torch.empty(dout, dtype=self.dtype, device=self.device) \
            if out is None else out
        self._vec(y, dout)
        self._sync_stream()
        f = _lib.load().hd_apply_T if transpose else _lib.load().hd_step
        _lib.check(f(self._h, ctypes.c_void_p(x.data_ptr()),
                     ctypes.c_void_p(y.data_ptr())),
                   "hd_apply_T" if transpose else "hd_step")
        return y

    def run(self, x1, T, dyn, a, b, pattern="Q", x0=None, record=True):
        """T steps of x_{t+1} = f_t(M_t x_t, ...) with a built-in f_t.
        Returns (X, Y) with X[t-1] = x_t (T+1 rows) and Y[t-1] = y_t when
        record is True, else (x_{T+1}, None)."""
        torch = _torch()
        x1 = self._vec(x1, self.n)
        if x0 is not None:
            x0 = self._vec(x0, self.n)
        d = _lib.HDDynamics(_DYN[dyn], _PATTERN[pattern], a, b)
        self._sync_stream()
        L = _lib.load()
        vp = ctypes.c_void_p
        if record:
            X = torch.empty((T + 1, self.n), dtype=self.dtype,
                            device=self.device)
            Y = torch.empty((T, self.m), dtype=self.dtype, device=self.device)
            rc = L.hd_run(self._h, ctypes.byref(d), T, vp(x1.data_ptr()),
                          vp(x0.data_ptr()) if x0 is not None else None,
                          None, vp(X.data_ptr()), vp(Y.data_ptr()))
            _lib.check(rc, "hd_run")
            return X, Y
        xo = torch.empty(self.n, dtype=self.dtype, device=self.device)
        rc = L.hd_run(self._h, ctypes.byref(d), T, vp(x1.data_ptr()),
                      vp(x0.data_ptr()) if x0 is not None else None,
                      vp(xo.data_ptr()), None, None)
        _lib.check(rc, "hd_run")
        return xo, None

    def spectral_power(self, xi, x1, K, scale=1.0):
        """Spectral method of Sec. 2.2 on this Haar handle of size m
        (``hd_spectral_power``): A = [I_n 0] Q with n = len(xi) < m,
        measurements y = tanh|A' xi|, and K power steps
        x_{k+1} = scale * A diag(y) A' x_k.  Returns (A' xi, X) with
        X[k] = x_{k+1}, (K+1) x n."""
        torch = _torch()
        n = int(xi.numel())
        xi = self._vec(xi, n)
        x1 = self._vec(x1, n)
        z = torch.empty(self.m, dtype=self.dtype, device=self.device)
        X = torch.empty((K + 1, n), dtype=self.dtype, device=self.device)
        self._sync_stream()
        _lib.check(_lib.load().hd_spectral_power(
            self._h, n, ctypes.c_void_p(xi.data_ptr()),
            ctypes.c_void_p(x1.data_ptr()), int(K), float(scale),
            ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(X.data_ptr())),
            "hd_spectral_power")
        return z, X

    def lista_forward(self, a, theta, x1, y):
        """Unrolled ISTA layers (see ``hd_lista_forward``): returns
        X ((L+1) x n, X[0] = x1), U and V (L x n)."""
        torch = _torch()
        L = len(a)
        af = (ctypes.c_float * L)(*[float(v) for v in a])
        tf = (ctypes.c_float * L)(*[float(v) for v in theta])
        X = torch.empty((L + 1, self.n), dtype=self.dtype, device=self.device)
        X[0] = self._vec(x1, self.n)
        U = torch.empty((L, self.n), dtype=self.dtype, device=self.device)
        V = torch.empty((L, self.n), dtype=self.dtype, device=self.device)
        y = self._vec(y, self.m)
        self._sync_stream()
        _lib.check(_lib.load().hd_lista_forward(
            self._h, L, af, tf, ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(U.data_ptr()),
            ctypes.c_void_p(V.data_ptr())), "hd_lista_forward")
        return X, U, V

    def lista_backward(self, a, theta, U, V, g, need_x1=False):
        """Reverse pass: (dL/da, dL/dtheta as FP64 tensors, dL/dx_1 or
        None) for g = dL/dx_{L+1}."""
        torch = _torch()
        L = len(a)
        af = (ctypes.c_float * L)(*[float(v) for v in a])
        tf = (ctypes.c_float * L)(*[float(v) for v in theta])
        ga = torch.empty(L, dtype=torch.float64, device=self.device)
        gt = torch.empty(L, dtype=torch.float64, device=self.device)
        gx = (torch.empty(self.n, dtype=self.dtype, device=self.device)
              if need_x1 else None)
        g = self._vec(g, self.n)
        self._sync_stream()
        _lib.check(_lib.load().hd_lista_backward(
            self._h, L, af, tf, ctypes.c_void_p(U.data_ptr()),
            ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(ga.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
            ctypes.c_void_p(gx.data_ptr()) if gx is not None else None),
            "hd_lista_backward")
        return ga, gt, gx

    def reset(self, seed, trial=0):
        """Restart with a fresh matrix keyed (seed, trial), same buffers."""
        _lib.check(_lib.load().hd_reset(self._h, seed, trial), "hd_reset")

    def status(self):
        rc = _lib.load().hd_status(self._h)
        return rc

    def counts(self):
        t, r, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().hd_counts(self._h, ctypes.byref(t),
                                         ctypes.byref(r), ctypes.byref(l)),
                   "hd_counts")
        return t.value, r.value, l.value

    def pivots(self, side, count=None):
        """(nu, pivot, sign) of the first `count` reflectors of a side
        (0 = R, 1 = L), as numpy arrays."""
        import numpy as np
        if count is None:
            t, r, l = self.counts()
            count = r if side == 0 else l
        nu = np.zeros(count)
        piv = np.zeros(count)
        sg = np.zeros(count, dtype=np.int32)
        _lib.check(_lib.load().hd_pivots(
            self._h, side, count, nu.ctypes.data_as(ctypes.c_void_p),
            piv.ctypes.data_as(ctypes.c_void_p),
            sg.ctypes.data_as(ctypes.c_void_p)), "hd_pivots")
        return nu, piv, sg

    def profile(self, enable=True):
        _lib.check(_lib.load().hd_profile(self._h, 1 if enable else 0),
                   "hd_profile")

    def profile_read(self, kind):
        ms, cnt, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _lib.check(_lib.load().hd_profile_read(self._h, kind,
                                               ctypes.byref(ms),
                                               ctypes.byref(cnt),
                                               ctypes.byref(by)),
                   "hd_profile_read")
        return ms.value, cnt.value, by.value


class HaarBatch:
    """Independent Haar trials run together (all Q-queries, one built-in f_t).

    trials: list of (n, T, seed, trial) tuples.  run() starts every trial
    from a fresh Q and returns, per trial in the given order, x_{T+1}, or the
    recorded (X, Y) trajectories when record is True.
    """

    def __init__(self, trials, dtype=None, device="cuda:0"):
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be float32 or float64")
        self.trials = [tuple(int(v) for v in t) for t in trials]
        self.dtype = dtype
        self.device = torch.device(device)
        arr = (_lib.HDBatchTrial * len(self.trials))(
            *[_lib.HDBatchTrial(n, T, s, k) for n, T, s, k in self.trials])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().hd_batch_init(
                HD_F64 if dtype == torch.float64 else HD_F32, arr,
                len(self.trials), _stream_ptr(self.device), ctypes.byref(h)),
                "hd_batch_init")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().hd_batch_free(h)
            self._h = None

    def _ptrs(self, tensors):
        return (ctypes.c_void_p * len(tensors))(
            *[t.data_ptr() for t in tensors])

    def run(self, x1, dyn, a, b, record=False):
        """x1: list of device tensors (n_i entries each)."""
        torch = _torch()
        if len(x1) != len(self.trials):
            raise ValueError("one x1 per trial")
        x1 = [t.to(self.device, self.dtype).contiguous() for t in x1]
        for t, (n, _, _, _) in zip(x1, self.trials):
            if t.numel() != n:
                raise ValueError("x1 length does not match the trial's n")
        L = _lib.load()
        _lib.check(L.hd_batch_set_stream(self._h, _stream_ptr(self.device)),
                   "hd_batch_set_stream")
        d = _lib.HDDynamics(_DYN[dyn], HD_PATTERN_Q, a, b)
        if record:
            X = [torch.empty((T + 1, n), dtype=self.dtype, device=self.device)
                 for n, T, _, _ in self.trials]
            Y = [torch.empty((T, n), dtype=self.dtype, device=self.device)
                 for n, T, _, _ in self.trials]
            _lib.check(L.hd_batch_run(self._h, ctypes.byref(d),
                                      self._ptrs(x1), None, self._ptrs(X),
                                      self._ptrs(Y)), "hd_batch_run")
            return X, Y
        out = [torch.empty(n, dtype=self.dtype, device=self.device)
               for n, _, _, _ in self.trials]
        _lib.check(L.hd_batch_run(self._h, ctypes.byref(d), self._ptrs(x1),
                                  self._ptrs(out), None, None),
                   "hd_batch_run")
        self._keep = (x1, out)
        return out

    def status(self):
        return _lib.load().hd_batch_status(self._h)

    def set_graph(self, enable=True):
        """Replay runs from a recorded HIP graph (``hd_batch_set_graph``);
        the current torch stream must not be the default stream."""
        _lib.check(_lib.load().hd_batch_set_stream(
            self._h, _stream_ptr(self.device)), "hd_batch_set_stream")
        _lib.check(_lib.load().hd_batch_set_graph(self._h,
                                                  1 if enable else 0),
                   "hd_batch_set_graph")

    def set_shape(self, chunks):
        """Chunks of 256 rows per workgroup of the batched kernels (1, 2, 4;
        ``hd_batch_set_shape``)."""
        _lib.check(_lib.load().hd_batch_set_shape(self._h, int(chunks)),
                   "hd_batch_set_shape")

    def shape(self):
        return _lib.load().hd_batch_shape(self._h)

    def autotune(self, x1, dyn, a, b, reps=2):
        """Time whole runs at 1, 2 and 4 chunks per workgroup and install
        the fastest (``hd_batch_autotune``).  Returns (chosen, {chunks: ms})."""
        if len(x1) != len(self.trials):
            raise ValueError("one x1 per trial")
        x1 = [t.to(self.device, self.dtype).contiguous() for t in x1]
        L = _lib.load()
        _lib.check(L.hd_batch_set_stream(self._h, _stream_ptr(self.device)),
                   "hd_batch_set_stream")
        d = _lib.HDDynamics(_DYN[dyn], HD_PATTERN_Q, a, b)
        ms = (ctypes.c_double * 3)()
        ch = ctypes.c_int32()
        _lib.check(L.hd_batch_autotune(self._h, ctypes.byref(d),
                                       self._ptrs(x1), int(reps), ms,
                                       ctypes.byref(ch)), "hd_batch_autotune")
        return ch.value, {1: ms[0], 2: ms[1], 4: ms[2]}


class IstaBatch:
    """Independent unrolled-ISTA trials on Gaussian matrices of one shape
    (``hd_ista_*``): trial i has an m x n Q with N(0, sigma^2) entries keyed
    (seed, trial0 + i), observes y = Q x* + w and runs L layers
    x_{t+1} = soft(x_t + a_t Q'(y - Q x_t), theta_t) from x_1 (zeros by
    default), all trials in lockstep.  With grad=True, ``grad`` runs the
    reverse pass of the last ``run`` for every trial."""

    def __init__(self, m, n, L, count, seed=0, trial0=0, sigma=1.0,
                 dtype=None, device="cuda:0", grad=False):
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        self.m, self.n, self.L, self.count = m, n, L, count
        self.dtype = dtype
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().hd_ista_init(
                _storage(dtype), m, n, L, count, seed, trial0, sigma,
                _lib.HD_ISTA_GRAD if grad else 0, _stream_ptr(self.device),
                ctypes.byref(h)), "hd_ista_init")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().hd_ista_free(h)
            self._h = None

    def run(self, a, theta, xstar, noise, x1=None):
        """a, theta: L floats; xstar: (count, n), noise: (count, m) device
        tensors; x1: None (zeros) or (count, n).  Returns X, (count, L+1, n)
        with X[:, t] = x_{t+1}."""
        torch = _torch()
        L = self.L
        if len(a) != L or len(theta) != L:
            raise ValueError("one (a, theta) pair per layer")
        xstar = xstar.to(self.device, self.dtype).contiguous()
        noise = noise.to(self.device, self.dtype).contiguous()
        if xstar.shape != (self.count, self.n) or \
                noise.shape != (self.count, self.m):
            raise ValueError("xstar must be (count, n), noise (count, m)")
        X = torch.zeros((self.count, L + 1, self.n), dtype=self.dtype,
                        device=self.device)
        if x1 is not None:
            X[:, 0] = x1
        af = (ctypes.c_float * L)(*[float(v) for v in a])
        tf = (ctypes.c_float * L)(*[float(v) for v in theta])
        Lb = _lib.load()
        _lib.check(Lb.hd_ista_set_stream(self._h, _stream_ptr(self.device)),
                   "hd_ista_set_stream")
        _lib.check(Lb.hd_ista_run(self._h, af, tf,
                                  ctypes.c_void_p(xstar.data_ptr()),
                                  ctypes.c_void_p(noise.data_ptr()),
                                  ctypes.c_void_p(X.data_ptr())),
                   "hd_ista_run")
        self._keep = (xstar, noise)
        return X

    def grad(self, a, theta, g):
        """Reverse pass of the last run (same a, theta): g = dL/dx_{L+1},
        (count, n).  Returns (dL/da, dL/dtheta) as (count, L) FP64 tensors
        (per trial) and dL/dx_2 per trial, (count, n)."""
        torch = _torch()
        L = self.L
        G = g.to(self.device, self.dtype).contiguous().clone()
        if G.shape != (self.count, self.n):
            raise ValueError("g must be (count, n)")
        ga = torch.empty((self.count, L), dtype=torch.float64,
                         device=self.device)
        gt = torch.empty_like(ga)
        af = (ctypes.c_float * L)(*[float(v) for v in a])
        tf = (ctypes.c_float * L)(*[float(v) for v in theta])
        Lb = _lib.load()
        _lib.check(Lb.hd_ista_set_stream(self._h, _stream_ptr(self.device)),
                   "hd_ista_set_stream")
        _lib.check(Lb.hd_ista_grad(self._h, af, tf,
                                   ctypes.c_void_p(G.data_ptr()),
                                   ctypes.c_void_p(ga.data_ptr()),
                                   ctypes.c_void_p(gt.data_ptr())),
                   "hd_ista_grad")
        return ga, gt, G

    def status(self):
        return _lib.load().hd_ista_status(self._h)


def _ista_batch_function():
    torch = _torch()

    class ISTABatch(torch.autograd.Function):
        """x_{L+1} of every trial of an IstaBatch (made with grad=True),
        differentiable in the shared per-layer a and theta (1-D tensors of
        length L): the gradient sums the trials' fixed-Q gradients."""

        @staticmethod
        def forward(ctx, a, theta, B, xstar, noise):
            ah = a.detach().float().cpu().tolist()
            th = theta.detach().float().cpu().tolist()
            X = B.run(ah, th, xstar, noise)
            ctx.B, ctx.ah, ctx.th = B, ah, th
            ctx.like = (a, theta)
            return X[:, -1].clone()

        @staticmethod
        def backward(ctx, gx):
            ga, gt, _ = ctx.B.grad(ctx.ah, ctx.th, gx)
            a, theta = ctx.like
            return (ga.sum(0).to(a.device, a.dtype),
                    gt.sum(0).to(theta.device, theta.dtype), None, None, None)

    return ISTABatch


_ISTA_BATCH = None


def ista_batch(a, theta, B, xstar, noise):
    """x_{L+1} of every trial of ``B`` (an IstaBatch with grad=True) as a
    differentiable function of the shared layer parameters a, theta."""
    global _ISTA_BATCH
    if _ISTA_BATCH is None:
        _ISTA_BATCH = _ista_batch_function()
    return _ISTA_BATCH.apply(a, theta, B, xstar, noise)


def _lista_function():
    torch = _torch()

    class LISTA(torch.autograd.Function):
        """x_{L+1} of unrolled ISTA layers on a lazy matrix, differentiable in
        the per-layer step a and threshold theta (1-D tensors of length L).
        The forward pass and the reverse pass are queries on the same handle
        (2L and 2(L-1) of them), so the gradient is that of one fixed Q."""

        @staticmethod
        def forward(ctx, a, theta, A, x1, y):
            ah = a.detach().float().cpu().tolist()
            th = theta.detach().float().cpu().tolist()
            X, U, V = A.lista_forward(ah, th, x1, y)
            ctx.A, ctx.ah, ctx.th, ctx.U, ctx.V = A, ah, th, U, V
            ctx.like = (a, theta)
            return X[-1].clone()

        @staticmethod
        def backward(ctx, gx):
            ga, gt, _ = ctx.A.lista_backward(ctx.ah, ctx.th, ctx.U, ctx.V,
                                             gx.contiguous())
            a, theta = ctx.like
            return (ga.to(device=a.device, dtype=a.dtype),
                    gt.to(device=theta.device, dtype=theta.dtype), None, None,
                    None)

    return LISTA


def lista(a, theta, A, x1, y):
    """Differentiable unrolled ISTA on the lazy matrix A (see LISTA)."""
    global _LISTA
    if _LISTA is None:
        _LISTA = _lista_function()
    return _LISTA.apply(a, theta, A, x1, y)


_LISTA = None


def _storage(dtype):
    torch = _torch()
    if dtype not in (torch.float32, torch.float64):
        raise TypeError("dtype must be float32 or float64")
    return HD_F64 if dtype == torch.float64 else HD_F32


def autotune(ensemble, lengths, dtype=None, k=8, device="cuda:0"):
    """Pick the panel kernels' launch shape per panel length on the device.

    For every length it times a whole trajectory of ``k`` queries of the
    ensemble (GINIBRE or HAAR) under each shape (workgroups of 1, 2 or 4
    chunks of 256 rows) and installs the fastest one process-wide for
    handles of that ensemble and storage type created afterwards.
    Returns {length: (chosen chunks, {chunks: microseconds})}.
    """
    torch = _torch()
    dtype = torch.float32 if dtype is None else dtype
    st = _storage(dtype)
    lengths = [int(v) for v in lengths]
    arr = (ctypes.c_int64 * len(lengths))(*lengths)
    rep = (ctypes.c_double * (3 * len(lengths)))()
    device = torch.device(device)
    with torch.cuda.device(device):
        _lib.check(_lib.load().hd_autotune(ensemble, st, arr, len(lengths),
                                           int(k), _stream_ptr(device), rep),
                   "hd_autotune")
    out = {}
    for i, n in enumerate(lengths):
        out[n] = (shape_rule(ensemble, n, dtype),
                  {c: rep[3 * i + j] for j, c in enumerate((1, 2, 4))})
    return out


def shape_rule(ensemble, n, dtype=None):
    """Chunks per workgroup a handle's panel of length n would use now."""
    torch = _torch()
    dtype = torch.float32 if dtype is None else dtype
    cpt = ctypes.c_int32()
    _lib.check(_lib.load().hd_shape_rule(ensemble, _storage(dtype), int(n),
                                         ctypes.byref(cpt)), "hd_shape_rule")
    return cpt.value


def autotune_clear():
    """Drop every tuned shape (back to the built-in rule)."""
    _lib.check(_lib.load().hd_autotune_clear(), "hd_autotune_clear")


class LazyGOE(LazyMatrix):
    """Lazy n x n matrix G ~ scale * GOE(n) (symmetric; diagonal entries
    N(0, 2 scale^2), off-diagonal N(0, scale^2)), G = (Q + Q')/sqrt(2) for a
    lazy Gaussian Q with N(0, scale^2) entries.  ``mv`` answers G x with two
    queries of Q (``hd_goe_step``), so t_max counts queries of Q (two per
    call)."""

    def __init__(self, n, t_max=None, seed=0, trial=0, scale=1.0, dtype=None,
                 device="cuda:0"):
        super().__init__(GINIBRE, n, t_max=t_max, seed=seed, trial=trial,
                         sigma=scale, dtype=dtype, device=device)
        self.scale = scale

    def mv(self, x):
        return self.goe_mv(x)

    def rmv(self, x):
        return self.goe_mv(x)

    def run(self, *args, **kwargs):
        raise TypeError("LazyGOE answers single queries (mv); the built-in "
                        "trajectories run on LazyMatrix")


def usv_mv(U, V, s, x, transpose=False):
    """y = Q x (or Q' x) for Q = U S V with U, V two Haar LazyMatrix handles
    of sizes m and n (same dtype and device) and S = diag(s) in R^{m x n}
    (s: min(m, n) entries) (``hd_usv_step``)."""
    torch = _torch()
    if U.device != V.device or U.dtype != V.dtype:
        raise ValueError("U and V must match in dtype and device")
    m, n = U.n, V.n
    x = U._vec(x, m if transpose else n)
    s = U._vec(s, min(m, n))
    y = torch.empty(n if transpose else m, dtype=U.dtype, device=U.device)
    U._sync_stream()
    V._sync_stream()
    _lib.check(_lib.load().hd_usv_step(
        U._h, V._h, ctypes.c_void_p(s.data_ptr()), 1 if transpose else 0,
        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())),
        "hd_usv_step")
    return y


class CLazyMatrix:
    """Lazy complex m x n random matrix on one GPU (``hd_c*``, Sec. 3.4).

    ensemble: GINIBRE (complex Gaussian entries, E|Q_ij|^2 = sigma^2) or HAAR
    (the unitary group U(n), m = n).  dtype: torch.complex64 or
    torch.complex128 (panel and vector storage).  ``mv``/``rmv`` answer
    Q x and Q^H x; ``gue_mv`` answers G x for G = (Q + Q^H) / sqrt(2) on a
    square Ginibre handle; ``run`` runs the fused Haar trajectory."""

    def __init__(self, ensemble, n, m=None, t_max=None, seed=0, trial=0,
                 sigma=1.0, dtype=None, device="cuda:0"):
        torch = _torch()
        dtype = torch.complex64 if dtype is None else dtype
        if dtype not in (torch.complex64, torch.complex128):
            raise TypeError("dtype must be complex64 or complex128")
        m = n if m is None else m
        t_max = min(m, n, 1024) if t_max is None else t_max
        self.ensemble, self.m, self.n, self.t_max = ensemble, m, n, t_max
        self.dtype = dtype
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().hd_cinit(
                ensemble, HD_F64 if dtype == torch.complex128 else HD_F32, m,
                n, t_max, seed, trial, sigma, _stream_ptr(self.device),
                ctypes.byref(h)), "hd_cinit")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().hd_cfree(h)
            self._h = None

    def _sync_stream(self):
        _lib.check(_lib.load().hd_cset_stream(self._h,
                                              _stream_ptr(self.device)),
                   "hd_cset_stream")

    def _vec(self, x, n):
        x = x.to(self.device, self.dtype).contiguous()
        if x.shape != (n,):
            raise ValueError("expected a vector of length %d" % n)
        return x

    def query(self, x, adjoint=False):
        torch = _torch()
        x = self._vec(x, self.m if adjoint else self.n)
        y = torch.empty(self.n if adjoint else self.m, dtype=self.dtype,
                        device=self.device)
        self._sync_stream()
        _lib.check(_lib.load().hd_cstep(self._h, 1 if adjoint else 0,
                                        ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr())),
                   "hd_cstep")
        return y

    def mv(self, x):
        return self.query(x, False)

    def rmv(self, x):
        return self.query(x, True)

    def gue_mv(self, x):
        torch = _torch()
        x = self._vec(x, self.n)
        y = torch.empty(self.n, dtype=self.dtype, device=self.device)
        self._sync_stream()
        _lib.check(_lib.load().hd_cgue_step(self._h,
                                            ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr())),
                   "hd_cgue_step")
        return y

    def run(self, x1, T, a, b, record=True):
        """T queries y_t = Q x_t with x_{t+1} = tanh(a |y_t|) e^{i arg y_t}
        + b x_t (Haar).  Returns X ((T+1) x n) and Y (T x n, or None)."""
        torch = _torch()
        X = torch.empty((T + 1, self.n), dtype=self.dtype, device=self.device)
        X[0] = self._vec(x1, self.n)
        Y = torch.empty((T, self.n), dtype=self.dtype,
                        device=self.device) if record else None
        self._sync_stream()
        _lib.check(_lib.load().hd_crun(
            self._h, T, float(a), float(b), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(Y.data_ptr()) if record else None), "hd_crun")
        return X, Y

    def reset(self, seed, trial=0):
        self._sync_stream()
        _lib.check(_lib.load().hd_creset(self._h, seed, trial), "hd_creset")

    def counts(self):
        t, r, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().hd_ccounts(self._h, ctypes.byref(t),
                                          ctypes.byref(r), ctypes.byref(l)),
                   "hd_ccounts")
        return t.value, r.value, l.value

    def status(self):
        return _lib.load().hd_cstatus(self._h)

    def profile(self, enable):
        self._sync_stream()
        _lib.check(_lib.load().hd_cprofile(self._h, 1 if enable else 0),
                   "hd_cprofile")

    def profile_read(self, kind):
        """(ms, launches, algorithmic bytes) of kind 0 (L1 dots), 1 (data
        pass) or 2 (output pass) since profiling started."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _lib.check(_lib.load().hd_cprofile_read(
            self._h, kind, ctypes.byref(ms), ctypes.byref(n),
            ctypes.byref(by)), "hd_cprofile_read")
        return ms.value, n.value, by.value
