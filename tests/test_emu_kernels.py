"""The library's runtime and kernel sources, emulated on the host under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/emu holds a host emulation of the HIP features the sources use: every
workgroup runs as cooperative fibers, barriers and wave-wide exchanges
(shuffles, DPP moves, permlane swaps) synchronise the fibers involved, and a
barrier some participant cannot reach aborts.  Device buffers are exact-size
host allocations, so any access beyond a buffer the runtime allocated, or
beyond a caller's vector, is reported by AddressSanitizer.

The normalising map x_{t+1} = y/||y|| + 0.1 x (the large single trial's
dynamics, switched off on the GPU after a fault whose cause was never shown)
runs here through exactly the launches hd_run would issue for it (Haar,
n = 4099, T = 30, FP32, the case of that fault): it must be clean under both
sanitizers and agree with the FP64 oracle.  A Gaussian trajectory with Q and
Q' alternating in the four-chunk launch shape covers the other ensemble and
the row-split column dots, the same in the one-chunk shape the workgroup
prologues of both passes (z = T'w, the reflector step), a small batch of unrolled-ISTA trials the
lockstep Gaussian batch and its reverse pass, and four ragged Haar trials the
Haar batch in one and four chunks per workgroup.  The complex path
(Sec. 3.4) runs mixed Q / Q^H
sequences with a zero query on U(n) and on a rectangular complex Ginibre
matrix, GUE steps, and a fused FP32 Haar trajectory.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2101_07464_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
EMU = os.path.join(ROOT, "tests", "emu")
CSRC = os.path.join(ROOT, "paper_2101_07464_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ of the ROCm toolchain not found")
    out = str(tmp_path_factory.mktemp("emu") / "emu_driver")
    cmd = [CLANG, "-std=c++17", "-O2", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(EMU, "shim"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-x", "c++", os.path.join(EMU, "driver.cpp"),
           "-x", "c++", os.path.join(CSRC, "hd_ista.hip"),
           "-x", "c++", os.path.join(CSRC, "hd_batch.hip"),
           "-x", "c++", os.path.join(CSRC, "hd_kernels.hip"),
           "-x", "c++", os.path.join(CSRC, "hd_cplx.hip"),
           "-x", "c++", os.path.join(EMU, "emu.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    return out


def _run(driver, tmp_path, ens, n, T, kind, a, b, pattern, seed, cpt, x1,
         extra_env=None):
    xf = str(tmp_path / "x1.bin")
    x1.astype(np.float32).tofile(xf)
    pre = str(tmp_path / "out")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", **(extra_env or {}))
    r = subprocess.run([driver, str(ens), str(n), str(T), str(kind), str(a),
                        str(b), str(pattern), str(seed), "0", "0", str(cpt),
                        xf, pre], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.split() == ["rc", "0", "status", "0"], r.stdout
    X = np.fromfile(pre + ".X", dtype=np.float32).reshape(T + 1, n)
    Y = np.fromfile(pre + ".Y", dtype=np.float32).reshape(T, n)
    return X.astype(np.float64), Y.astype(np.float64)


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_normalising_map_emulated(driver, tmp_path):
    n, T, seed = 4099, 30, 2
    x1 = inputs.x1_normal(n, seed=seed).astype(np.float32)
    X, Y = _run(driver, tmp_path, 1, n, T, 3, 0.0, 0.1, 0, seed, 0, x1)
    # mode B: the oracle answers the emulated run's own query vectors
    orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=seed)
    Yb = oracle.replay(orc, X[:-1], [False] * T)
    eb = max(relerr(y, yb) for y, yb in zip(Y, Yb))
    # mode A: the oracle's own FP64 trajectory of the same map
    orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=seed)
    Xo, _ = oracle.run_trajectory(orc, X[0], T, "normalize", 0.0, 0.1)
    ea = max(relerr(x, xo) for x, xo in zip(X, Xo))
    print("emulated normalising map: mode B %.2e  mode A %.2e" % (eb, ea))
    assert eb < 1e-4 and ea < 1e-4
    # the map's own invariant: x_{t+1} - 0.1 x_t has unit norm
    d = np.linalg.norm(X[1:] - 0.1 * X[:-1], axis=1)
    assert np.allclose(d, 1.0, atol=1e-5)


def test_gaussian_alternating_four_chunks_emulated(driver, tmp_path):
    n, T, seed = 2000, 8, 7
    x1 = inputs.x1_normal(n, seed=seed, scale=1.0).astype(np.float32)
    X, Y = _run(driver, tmp_path, 0, n, T, 2, 0.1, 0.3, 1, seed, 4, x1)
    orc = oracle.HDOracle(oracle.GINIBRE, n, tmax=T, seed=seed,
                          sigma=1.0 / np.sqrt(n))
    Yb = oracle.replay(orc, X[:-1], [t % 2 == 1 for t in range(T)])
    eb = max(relerr(y, yb) for y, yb in zip(Y, Yb))
    print("emulated Gaussian, four chunks: mode B %.2e" % eb)
    assert eb < 1e-4


def test_gaussian_alternating_one_chunk_emulated(driver, tmp_path):
    """One chunk per workgroup, where every workgroup of the data pass forms
    z = T'w and every workgroup of the random pass the reflector step in
    their prologues (the shape of the n = 65536 alternating workload).  Map
    x_{t+1} = tanh(y_t) + 0.5 x_t."""
    n, T, seed = 1100, 40, 3
    x1 = inputs.x1_normal(n, seed=seed).astype(np.float32)
    X, Y = _run(driver, tmp_path, 0, n, T, 1, 1.0, 0.5, 1, seed, 1, x1)
    orc = oracle.HDOracle(oracle.GINIBRE, n, tmax=T, seed=seed,
                          sigma=1.0 / np.sqrt(n))
    Yb = oracle.replay(orc, X[:-1], [t % 2 == 1 for t in range(T)])
    eb = max(relerr(y, yb) for y, yb in zip(Y, Yb))
    print("emulated Gaussian, one chunk: mode B %.2e" % eb)
    assert eb < 1e-4


def test_two_stage_reduction_emulated(driver, tmp_path):
    """The two-stage reduction of the partial rows (blocks of 256 rows x 32
    slots, then the block sums), which the library uses from 1024 rows per
    pass on, here forced for every reduction (HD_RED_TWO_STAGE=1) on a Haar
    trajectory with 264 one-chunk workgroups (two row blocks): Mode B
    against the oracle."""
    n, T = 66561, 4
    x1 = inputs.x1_normal(n, seed=1).astype(np.float32)
    X, Y = _run(driver, tmp_path, 1, n, T, 1, 1.0, 0.5, 0, 1, 1, x1,
                extra_env={"HD_RED_TWO_STAGE": "1"})
    orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=1)
    Yb = oracle.replay(orc, X[:-1], [False] * T)
    eb = max(relerr(y, yb) for y, yb in zip(Y, Yb))
    print("emulated two-stage reduction: mode B %.2e" % eb)
    assert eb < 1e-4


def test_ista_batch_emulated(driver, tmp_path):
    """Three lockstep unrolled-ISTA trials (m = 150, n = 300, 4 layers,
    FP32) and their reverse pass against the oracle's single-trial runs with
    the same keys."""
    C, n, m, L, seed, trial0 = 3, 300, 150, 4, 5, 10
    sig = 1.0 / np.sqrt(m)
    a32, t32 = float(np.float32(0.3)), float(np.float32(0.6))
    xs = np.stack([inputs.sparse_target(n, 0.8, 2.0, seed=0, trial=i)
                   for i in range(C)]).astype(np.float32)
    w = np.stack([inputs.noise(m, 0.1, seed=0, trial=i)
                  for i in range(C)]).astype(np.float32)
    g = np.random.default_rng(3).standard_normal((C, n)).astype(np.float32)
    xf, wf, out, gf, gout = (str(tmp_path / f) for f in
                             ("xs.bin", "w.bin", "X.bin", "g.bin", "gr.bin"))
    xs.tofile(xf)
    w.tofile(wf)
    g.tofile(gf)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([driver, "ista", str(m), str(n), str(L), str(C),
                        str(seed), str(trial0), "%.17g" % sig, "0.3", "0.6", xf,
                        wf, out, gf, gout], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.split() == ["rc", "0", "status", "0"], r.stdout
    X = np.fromfile(out, dtype=np.float32).reshape(C, L + 1, n)
    gr = np.fromfile(gout, dtype=np.float64).reshape(2, C, L)
    worst = worst_g = 0.0
    for i in range(C):
        orc = oracle.HDOracle(oracle.GINIBRE, n, m=m, tmax=4 * L - 1,
                              seed=seed, trial=trial0 + i, sigma=sig)
        y = orc.mv(xs[i].astype(np.float64)) + w[i]
        Xo, Uo, Vo = oracle.lista_forward(orc, np.zeros(n), y, [a32] * L,
                                          [t32] * L)
        worst = max(worst, max(relerr(a, b) for a, b in zip(X[i][1:],
                                                            Xo[1:])))
        da, dth, _ = oracle.lista_backward(orc, g[i].astype(np.float64),
                                           [a32] * L, [t32] * L, Uo, Vo)
        worst_g = max(worst_g, relerr(gr[0, i], da), relerr(gr[1, i], dth))
    print("emulated ISTA batch: layers %.2e, gradients %.2e"
          % (worst, worst_g))
    assert worst < 1e-4 and worst_g < 1e-4


def _crun_queries(driver, tmp_path, ens, m, n, f64, sigma, pattern, xs):
    dt = np.complex128 if f64 else np.complex64
    xf, yf = str(tmp_path / "cx.bin"), str(tmp_path / "cy.bin")
    np.concatenate([x.astype(dt) for x in xs]).tofile(xf)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, "cplx", str(ens), str(m), str(n), str(f64),
                        "3", "4", "%.17g" % sigma, pattern, xf, yf], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.split() == ["rc", "0", "status", "0"], r.stdout
    ys, o = np.fromfile(yf, dtype=dt).astype(np.complex128), 0
    out = []
    for c in pattern:
        L = m if c == "Q" else n
        out.append(ys[o:o + L])
        o += L
    return out


@pytest.mark.parametrize("ens,m,n,pattern", [
    (1, 1500, 1500, "QQHQQH"), (0, 1300, 900, "QHHQQH"), (0, 700, 700, "QGQG")])
def test_complex_queries_emulated(driver, tmp_path, ens, m, n, pattern):
    rng = np.random.default_rng(m + n)
    xs = [rng.standard_normal(m if c == "H" else n) +
          1j * rng.standard_normal(m if c == "H" else n) for c in pattern]
    xs[2] = np.zeros_like(xs[2])
    sig = 0.5 if ens == 0 else 1.0
    ys = _crun_queries(driver, tmp_path, ens, m, n, 1, sig, pattern, xs)
    tq = sum(2 if c == "G" else 1 for c in pattern)
    orc = oracle.CHDOracle(ens, n, m=m, tmax=tq, seed=3, trial=4, sigma=sig)
    for c, x, y in zip(pattern, xs, ys):
        if c == "G":
            want = (orc.mv(x) + orc.rmv(x)) / np.sqrt(2)
        else:
            want = orc.query(x, c == "H")
        assert np.abs(y - want).max() <= 1e-12 * max(np.abs(want).max(), 1)


def test_complex_haar_trajectory_emulated(driver, tmp_path):
    n, T, a, b = 2100, 12, 1.0, 0.1
    rng = np.random.default_rng(1)
    x1 = (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    x1.astype(np.complex64).tofile(str(tmp_path / "x1.bin"))
    pre = str(tmp_path / "run")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, "crun", str(n), str(T), str(a), str(b), "0",
                        "5", "6", str(tmp_path / "x1.bin"), pre], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr
    assert r.stdout.split() == ["rc", "0", "status", "0"], r.stdout
    X = np.fromfile(pre + ".X", dtype=np.complex64).reshape(T + 1, n)
    Y = np.fromfile(pre + ".Y", dtype=np.complex64).reshape(T, n)
    X, Y = X.astype(np.complex128), Y.astype(np.complex128)
    orc = oracle.CHDOracle(oracle.HAAR, n, tmax=T, seed=5, trial=6)
    for t in range(T):
        assert relerr(Y[t], orc.mv(X[t])) < 1e-5
        assert np.abs(oracle.f_ctanh(Y[t], X[t], a, b) - X[t + 1]).max() < 1e-6


@pytest.mark.parametrize("cpt", ["1", "4"])
def test_haar_batch_emulated(driver, tmp_path, cpt):
    """Four ragged FP32 Haar trials in one batch (hd_batch_run, tanh(2y)),
    one and four chunks per workgroup: every x_{t+1} equals the map of the
    oracle's answer to the emulated run's own x_t."""
    spec = [(1500, 9), (3000, 5), (700, 12), (2049, 7)]
    sf, xf, out = (str(tmp_path / f) for f in ("spec.bin", "x1.bin", "X.bin"))
    np.array(spec, dtype=np.int64).ravel().tofile(sf)
    np.concatenate([inputs.x1_normal(n, seed=0, trial=i).astype(np.float32)
                    for i, (n, T) in enumerate(spec)]).tofile(xf)
    env = dict(os.environ, HD_BATCH_CPT=cpt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, "batch", sf, xf, out], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.split() == ["rc", "0", "status", "0"], r.stdout
    X = np.fromfile(out, dtype=np.float32).astype(np.float64)
    o, worst = 0, 0.0
    for i, (n, T) in enumerate(spec):
        Xi = X[o:o + n * (T + 1)].reshape(T + 1, n)
        o += n * (T + 1)
        orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=0, trial=i)
        for t in range(T):
            worst = max(worst, np.abs(np.tanh(2 * orc.mv(Xi[t])) -
                                      Xi[t + 1]).max())
    assert worst < 1e-6


def test_haar_batch_shapes_emulated(driver, tmp_path):
    """The same batch switched between launch shapes in one process
    (hd_batch_set_shape 1 -> 4 -> 2, then the autotuner, then 1 again): the
    block map, partial-row counts and per-trial arguments follow each switch,
    so every run's trajectory satisfies x_{t+1} = tanh(2 Q x_t) against the
    oracle, and all runs agree to FP32 rounding."""
    spec = [(1500, 6), (3000, 4), (700, 7)]
    sf, xf, out = (str(tmp_path / f) for f in ("spec.bin", "x1.bin", "X.bin"))
    np.array(spec, dtype=np.int64).ravel().tofile(sf)
    np.concatenate([inputs.x1_normal(n, seed=0, trial=i).astype(np.float32)
                    for i, (n, T) in enumerate(spec)]).tofile(xf)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("HD_BATCH_CPT", None)
    r = subprocess.run([driver, "batch", sf, xf, out, "142a1"], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[:3] == ["shape 1 rc 0 status 0", "shape 4 rc 0 status 0",
                         "shape 2 rc 0 status 0"], r.stdout
    assert lines[3].startswith("tuned ")
    assert lines[4] == "shape 1 rc 0 status 0", r.stdout
    runs = [np.fromfile(out + ".%d" % k, dtype=np.float32).astype(np.float64)
            for k in range(4)]
    worst = 0.0
    o = 0
    for i, (n, T) in enumerate(spec):
        orc = oracle.HDOracle(oracle.HAAR, n, tmax=T, seed=0, trial=i)
        Xi = runs[0][o:o + n * (T + 1)].reshape(T + 1, n)
        for t in range(T):
            worst = max(worst, np.abs(np.tanh(2 * orc.mv(Xi[t])) -
                                      Xi[t + 1]).max())
        o += n * (T + 1)
    assert worst < 1e-6
    for k in range(1, 4):
        assert np.abs(runs[k] - runs[0]).max() < 1e-5
