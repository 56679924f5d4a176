"""The allocation-free trajectory entry point (hd_run_noalloc) against the
allocating one (hd_init + hd_run + hd_free) on the GPU.

Both run the same kernels in the same launch shapes on a fresh Q with the
same key, so their trajectories must agree to the parity bar (FP64 storage
1e-11, FP32 1e-4; in practice bit for bit).  Two calls in a row, the second
smaller than the first, check that a call does not see what the previous one
left in the shared static array.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2101_07464_amd as hd  # noqa: E402
from paper_2101_07464_amd import _lib, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def relerr(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _noalloc(ens, n, T, dtype, dyn, a, b, pattern, seed, x1, record):
    L = _lib.load()
    sig = 1.0 / np.sqrt(n) if ens == hd.GINIBRE else 1.0
    stream = torch.cuda.current_stream(DEV).cuda_stream
    cfg = _lib.HDConfig(ens, _lib.HD_F64 if dtype == torch.float64
                        else _lib.HD_F32, n, n, T, seed, 0, sig,
                        ctypes.c_void_p(stream))
    d = _lib.HDDynamics(hd._DYN[dyn], hd._PATTERN[pattern], a, b)
    need = ctypes.c_size_t()
    assert L.hd_noalloc_scratch_bytes(ctypes.byref(cfg),
                                      ctypes.byref(need)) == 0
    assert need.value <= _lib.HD_NOALLOC_SCRATCH_BYTES
    vp = ctypes.c_void_p
    if record:
        X = torch.empty((T + 1, n), dtype=dtype, device=DEV)
        Y = torch.empty((T, n), dtype=dtype, device=DEV)
        rc = L.hd_run_noalloc(ctypes.byref(cfg), ctypes.byref(d), T,
                              vp(x1.data_ptr()), None, None,
                              vp(X.data_ptr()), vp(Y.data_ptr()))
        assert rc == 0, _lib.strerror(rc)
        return X, Y
    xo = torch.empty(n, dtype=dtype, device=DEV)
    rc = L.hd_run_noalloc(ctypes.byref(cfg), ctypes.byref(d), T,
                          vp(x1.data_ptr()), None, vp(xo.data_ptr()), None,
                          None)
    assert rc == 0, _lib.strerror(rc)
    return xo, None


def _plain(ens, n, T, dtype, dyn, a, b, pattern, seed, x1, record):
    sig = 1.0 / np.sqrt(n) if ens == hd.GINIBRE else 1.0
    A = hd.LazyMatrix(ens, n, t_max=T, seed=seed, sigma=sig, dtype=dtype,
                      device=DEV)
    out = A.run(x1, T, dyn, a, b, pattern, record=record)
    torch.cuda.synchronize()
    assert A.status() == 0
    A.close()
    return out


CASES = [
    # (ensemble, n, T, dtype, map, a, b, pattern, seed, x1 scale, record)
    [(hd.HAAR, 20011, 40, torch.float32, "tanh", 1.0, 0.5, "Q", 3, None,
      True),
     (hd.HAAR, 3001, 16, torch.float64, "tanh", 2.0, 0.0, "alt", 4, None,
      True)],
    [(hd.GINIBRE, 9001, 30, torch.float32, "soft_hist", 0.1, 0.3, "alt", 5,
      1.0, True),
     (hd.GINIBRE, 2003, 12, torch.float64, "soft_hist", 0.1, 0.3, "alt", 6,
      1.0, False)],
]


@pytest.mark.parametrize("pair", CASES, ids=["haar", "gaussian"])
def test_noalloc_matches_allocating_run(pair):
    for ens, n, T, dtype, dyn, a, b, pat, seed, sc, rec in pair:
        print("noalloc case: ens %d n %d T %d %s %s" % (ens, n, T, dtype,
                                                        pat), flush=True)
        x1 = torch.from_numpy(inputs.x1_normal(n, seed=seed, scale=sc)).to(
            DEV, dtype)
        got = _noalloc(ens, n, T, dtype, dyn, a, b, pat, seed, x1, rec)
        torch.cuda.synchronize()
        ref = _plain(ens, n, T, dtype, dyn, a, b, pat, seed, x1, rec)
        ex = relerr(got[0], ref[0])
        ey = relerr(got[1], ref[1]) if rec else 0.0
        print("  x %.2e  y %.2e  bitwise %s" %
              (ex, ey, bool(torch.equal(got[0], ref[0]))), flush=True)
        assert ex < TOL[dtype] and ey < TOL[dtype]
