"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hd.h declares, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_2101_07464_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(hd_\w+)\s*\(",
                                 txt, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_symbol():
    L = _lib.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert _lib.strerror(code)


def _cfg(**kw):
    base = dict(ensemble=_lib.HD_HAAR, storage=_lib.HD_F32, m=64, n=64,
                t_max=8, seed=0, trial=0, sigma=1.0, stream=None)
    base.update(kw)
    return _lib.HDConfig(**base)


@pytest.mark.parametrize("kw", [
    dict(m=64, n=65),              # Haar must be square
    dict(t_max=0),
    dict(t_max=65),                # T <= min(m, n)
    dict(n=0, m=0),
    dict(storage=7),
    dict(ensemble=3),
    dict(ensemble=_lib.HD_GINIBRE, m=10, n=20, t_max=11),
    dict(ensemble=_lib.HD_GINIBRE, sigma=0.0),
])
def test_init_rejects_invalid_config(kw):
    h = ctypes.c_void_p()
    rc = _lib.load().hd_init(ctypes.byref(_cfg(**kw)), ctypes.byref(h))
    assert rc == _lib.HD_ERR_INVALID
    assert not h.value


def test_null_arguments():
    L = _lib.load()
    assert L.hd_init(None, None) == _lib.HD_ERR_INVALID
    assert L.hd_step(None, None, None) == _lib.HD_ERR_INVALID
    assert L.hd_apply_T(None, None, None) == _lib.HD_ERR_INVALID
    assert L.hd_status(None) == _lib.HD_ERR_INVALID
    assert L.hd_counts(None, None, None, None) == _lib.HD_ERR_INVALID
    assert L.hd_free(None) == _lib.HD_OK
    assert L.hd_batch_set_graph(None, 1) == _lib.HD_ERR_INVALID
    assert L.hd_goe_step(None, None, None) == _lib.HD_ERR_INVALID
    assert L.hd_usv_step(None, None, None, 0, None, None) == \
        _lib.HD_ERR_INVALID
    assert L.hd_run(None, None, 0, None, None, None, None, None) == \
        _lib.HD_ERR_INVALID


@pytest.mark.skipif("HD_CPT" in os.environ, reason="HD_CPT overrides shapes")
def test_builtin_shape_rule():
    L = _lib.load()
    cpt = ctypes.c_int32()
    assert L.hd_autotune_clear() == _lib.HD_OK
    for ens in (_lib.HD_GINIBRE, _lib.HD_HAAR):
        for st in (_lib.HD_F32, _lib.HD_F64):
            for n, want in [(1, 1), (65536, 1), ((1 << 18) - 1, 1),
                            (1 << 18, 2), ((1 << 19) - 1, 2), (1 << 19, 4),
                            (10 ** 7, 4)]:
                assert L.hd_shape_rule(ens, st, n, ctypes.byref(cpt)) == \
                    _lib.HD_OK
                assert cpt.value == want, (ens, st, n)
    assert L.hd_shape_rule(0, 5, 10, ctypes.byref(cpt)) == _lib.HD_ERR_INVALID
    assert L.hd_shape_rule(2, 0, 10, ctypes.byref(cpt)) == _lib.HD_ERR_INVALID
    assert L.hd_shape_rule(0, 0, 0, ctypes.byref(cpt)) == _lib.HD_ERR_INVALID
    assert L.hd_shape_rule(0, 0, 10, None) == _lib.HD_ERR_INVALID


def test_autotune_rejects_invalid_arguments():
    L = _lib.load()
    arr = (ctypes.c_int64 * 2)(4096, 1)
    H, F32 = _lib.HD_HAAR, _lib.HD_F32
    assert L.hd_autotune(H, F32, None, 1, 8, None, None) == \
        _lib.HD_ERR_INVALID
    assert L.hd_autotune(5, F32, arr, 1, 8, None, None) == \
        _lib.HD_ERR_INVALID
    assert L.hd_autotune(H, 7, arr, 1, 8, None, None) == _lib.HD_ERR_INVALID
    assert L.hd_autotune(H, F32, arr, 0, 8, None, None) == \
        _lib.HD_ERR_INVALID
    assert L.hd_autotune(H, F32, arr, 1, 1, None, None) == \
        _lib.HD_ERR_INVALID
    # the second length is shorter than the trajectory
    assert L.hd_autotune(H, F32, arr, 2, 8, None, None) == \
        _lib.HD_ERR_INVALID


def _state_header(**kw):
    """A state header as hd_export writes it (host byte order)."""
    import struct
    f = dict(magic=b"HDSTATE1", ensemble=_lib.HD_HAAR, storage=_lib.HD_F32,
             t_max=8, pstride=20, m=64, n=64, seed=0, trial=0, sigma=0.0,
             t=2, r=2, l=2, flag=0, pf=(0, 0), pending=(-1, -1),
             vcols=(2, 2), bcols=(0, 0), total=1 << 20)
    f.update(kw)
    return struct.pack("<8s4i2q2Id4i2i2i2i2iQ", f["magic"], f["ensemble"],
                       f["storage"], f["t_max"], f["pstride"], f["m"], f["n"],
                       f["seed"], f["trial"], f["sigma"], f["t"], f["r"],
                       f["l"], f["flag"], *f["pf"], *f["pending"],
                       *f["vcols"], *f["bcols"], f["total"])


def test_state_header_size():
    assert len(_state_header()) == 112


@pytest.mark.parametrize("kw", [
    dict(magic=b"HDSTATE0"),
    dict(m=65, n=65),              # sizes differ from cfg
    dict(t_max=9),
    dict(storage=_lib.HD_F64),
    dict(ensemble=_lib.HD_GINIBRE),
    dict(t=9),                     # beyond t_max
    dict(r=3),                     # more reflectors than queries
])
def test_import_rejects_malformed_state(kw):
    L = _lib.load()
    buf = _state_header(**kw) + bytes(256)
    h = ctypes.c_void_p()
    rc = L.hd_import(ctypes.byref(_cfg()), buf, len(buf), ctypes.byref(h))
    assert rc == _lib.HD_ERR_INVALID
    assert not h.value


def test_export_import_null_arguments():
    L = _lib.load()
    size = ctypes.c_size_t(0)
    h = ctypes.c_void_p()
    assert L.hd_export(None, None, ctypes.byref(size)) == _lib.HD_ERR_INVALID
    assert L.hd_import(None, b"x" * 200, 200, ctypes.byref(h)) == \
        _lib.HD_ERR_INVALID
    assert L.hd_import(ctypes.byref(_cfg()), None, 200, ctypes.byref(h)) == \
        _lib.HD_ERR_INVALID
    # shorter than the header
    assert L.hd_import(ctypes.byref(_cfg()), b"HDSTATE1", 8,
                       ctypes.byref(h)) == _lib.HD_ERR_INVALID


@pytest.mark.parametrize("trials,count", [
    ([], 0),                       # empty batch
    ([(10, 0, 0, 0)], 1),          # T = 0
    ([(10, 11, 0, 0)], 1),         # T > n
    ([(0, 1, 0, 0)], 1),           # n = 0
    ([(100, 5, 0, 0), (3, 4, 0, 1)], 2),
])
def test_batch_init_rejects_invalid_trials(trials, count):
    L = _lib.load()
    arr = (_lib.HDBatchTrial * max(len(trials), 1))(
        *[_lib.HDBatchTrial(*t) for t in trials])
    h = ctypes.c_void_p()
    rc = L.hd_batch_init(_lib.HD_F32, arr, count, None, ctypes.byref(h))
    assert rc == _lib.HD_ERR_INVALID
    assert not h.value


def test_noalloc_sizing_and_limit():
    """The allocation-free entry point sizes its layout on the host and
    refuses problems beyond its static array before touching the device."""
    L = _lib.load()
    need = ctypes.c_size_t()
    assert L.hd_noalloc_scratch_bytes(ctypes.byref(_cfg(n=1000, m=1000,
                                                         t_max=20)),
                                      ctypes.byref(need)) == _lib.HD_OK
    # two FP32 panels of 1024 x 20 plus vectors: well inside the array
    assert 2 * 1024 * 20 * 4 < need.value < _lib.HD_NOALLOC_SCRATCH_BYTES
    big = _cfg(n=1 << 20, m=1 << 20, t_max=64)
    assert L.hd_noalloc_scratch_bytes(ctypes.byref(big),
                                      ctypes.byref(need)) == _lib.HD_OK
    assert need.value > _lib.HD_NOALLOC_SCRATCH_BYTES
    dyn = _lib.HDDynamics(_lib.HD_DYN_TANH, _lib.HD_PATTERN_Q, 1.0, 0.5)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: refused first
    assert L.hd_run_noalloc(ctypes.byref(big), ctypes.byref(dyn), 4, fake,
                            None, None, None, None) == _lib.HD_ERR_TOO_LARGE
    assert L.hd_run_noalloc(None, ctypes.byref(dyn), 4, fake, None, None,
                            None, None) == _lib.HD_ERR_INVALID
    assert L.hd_run_noalloc(ctypes.byref(_cfg(t_max=0)), ctypes.byref(dyn),
                            4, fake, None, None, None,
                            None) == _lib.HD_ERR_INVALID
    assert L.hd_noalloc_scratch_bytes(None, ctypes.byref(need)) == \
        _lib.HD_ERR_INVALID
