"""Benchmark of the Householder Dice step on one MI355X.

A step is one whole trajectory of the workload: hd_reset (a fresh random
matrix, new Philox key) followed by T queries of eq. (dynamics) with the
workload's map f_t, all on the GPU, inputs resident in HBM.  The metric is
nominal element updates per second, W = n * sum_{t<=T} t per trajectory
(n the larger dimension), plus the roofline of the dominant panel kernel.

Timing: W warm-up steps, then K steps between two device synchronisations
(value, ms_per_step); then the same K steps once more with HIP events around
every panel launch, from which the dominant kernel's average duration and its
roofline fraction are taken (events perturb the launch stream, so that pass
is not timed).

Workloads (--workload):
  c4  (default) the large single trial: Haar n = 1e7, T = 200, Q-queries,
      FP32 panels and vectors (two panels of 8 GB), FP64 accumulation, norms
      and T; x_1 ~ N(0, I/n).  Its specified map x_{t+1} = y/||y|| + 0.1 x is
      switched off in the library, so x_{t+1} = tanh(y) + 0.1 x stands in
      (the same passes and bytes).  The line also carries the error of the
      first answers against the FP64 oracle (replaying the GPU's own query
      vectors), the Haar invariants over all 200 answers, and -- unless
      --no-extras -- the batched-vs-plain ratio of the batched workload and
      the reverse-over-forward time of the differentiated one.
  c2  Ginibre n = m = 65536, sigma = 1/sqrt(n), T = 100, queries
      Q, Q', Q, ...; x_{t+1} = soft(y_t, 0.1) + 0.3 x_{t-1}, x_1 ~ N(0, I),
      x_0 = 0; FP32 panels and vectors, FP64 accumulation, norms and T.
      Its panels (at most 52 MB) stay in the 256 MB Infinity Cache, so its
      roofline is flagged cache-resident.
  c1  Haar n = 1000, T = 20, FP64; x_{t+1} = tanh(y_t) + 0.5 x_t,
      x_1 ~ N(0, I/n).
  c3  4096 independent Haar trials, n log-uniform in [1e3, 1e5], T uniform
      in [10, 200] (tag-5 draws), x_{t+1} = tanh(2 y_t), x_1 ~ N(0, I/n),
      FP32, all trials in one batch (hd_batch_run); a step runs every trial
      to completion.  Also times the same kind of trials one handle at a time
      (a sample of them) for the batched-vs-plain comparison.
  c5  Differentiated unrolled ISTA: Gaussian Q (n = 262144, m = 131072,
      N(0, 1/m) entries), y = Q x* + 0.01 noise, x* Bernoulli(0.1)-Gaussian
      (sd 2), 50 layers with FP32 (a_t, theta_t) = (0.3, 0.6), loss
      ||x_51 - x*||^2; FP32 storage.  A step is --c5-trials trials, each a
      fresh Q: forward pass (101 queries) and reverse pass (98 queries);
      also timed forward-only, and the same trials as one lockstep batch
      (hd_ista_run + hd_ista_grad) against the trial-by-trial run.
  goe       50 GOE queries G x_t at n = 65536 (two queries of Q each).
  spectral  the spectral method of Sec. 2.2: n = 1e5, m = 2e5, 50 power
            steps of m D through the lazy Haar Q.
  lasso     the lasso experiment of Sec. 2.1: 1e5 ISTA trials at n = 1000,
            m = 500, T = 50 in one lockstep batch, beside the direct method
            (dense Q) on 20000 trials, with both mean squared error curves.
  cplx      complex HD (Sec. 3.4): U(1e7), T = 200, complex64, map
            tanh(|y|) e^{i arg y} + 0.1 x.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("HD n*t elem-updates/s and % HBM peak; batched/adjoint vs plain "
          "at err<=1e-4")
HBM_PEAK_GBS = 8000.0
KIND_NAMES = {0: "panel TDOT (k_tdot)", 1: "data-side GEMV-N (k_pass)",
              2: "random-side GEMV-N (k_pass / k_gin_pass)"}

WORKLOADS = {
    "c2": dict(name="ginibre_n65536_T100_alt_soft_fp32", ensemble="ginibre",
               n=65536, T=100, dyn="soft_hist", a=0.1, b=0.3, pattern="alt",
               f64=False, x1_scale=1.0, dense=True, modeb=100,
               title="Gaussian n=m=65536, T=100, Q and Q' alternating, FP32",
               dyn_text="x_{t+1} = soft(y_t, 0.1) + 0.3 x_{t-1}",
               cache_resident="cache-resident: the panels (at most 52 MB) "
                              "fit the 256 MB Infinity Cache, so this "
                              "fraction of the HBM peak measures latency, "
                              "not HBM bandwidth"),
    "c1": dict(name="haar_n1000_T20_tanh_fp64", ensemble="haar", n=1000,
               T=20, dyn="tanh", a=1.0, b=0.5, pattern="Q", f64=True,
               x1_scale=None, modeb=20,
               title="Haar n=1000, T=20, Q-queries, FP64",
               dyn_text="x_{t+1} = tanh(y_t) + 0.5 x_t",
               cache_resident="cache-resident: the panels (320 KB) fit the "
                              "L2, so this fraction measures launch "
                              "latency"),
    # the large single trial; its normalising map is switched off in the
    # library, so tanh(y) + 0.1 x stands in (same passes, same bytes)
    "c4": dict(name="haar_n1e7_T200_tanh_fp32", ensemble="haar", n=10000000,
               T=200, dyn="tanh", a=1.0, b=0.1, pattern="Q", f64=False,
               x1_scale=None, modeb=8,
               title="large single trial: Haar n=1e7, T=200, Q-queries, FP32 "
                     "(map tanh(y)+0.1x standing in for y/||y||+0.1x)",
               dyn_text="x_{t+1} = tanh(y_t) + 0.1 x_t (stand-in: the "
                        "specified y_t/||y_t|| + 0.1 x_t is switched off in "
                        "the library)"),
}

KERNEL_OF_KIND = {(0, "ginibre"): "k_tdot", (1, "ginibre"): "k_pass<data>",
                  (2, "ginibre"): "k_gin_pass", (0, "haar"): "k_tdot",
                  (1, "haar"): "k_pass<data>", (2, "haar"): "k_pass<random>"}


def kernel_sources_sha256(files=("hd_kernels.hip", "hd_device.hpp",
                                 "hd_internal.hpp")):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2101_07464_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


CPLX_SOURCES = ("hd_cplx.hip", "hd_device.hpp", "hd_internal.hpp")


def measured_traffic(workload, kernel, files=None):
    """HBM bytes per launch from a committed PMC summary under profiles/,
    or None when there is none for these kernel sources."""
    import glob
    sha = kernel_sources_sha256(files) if files else kernel_sources_sha256()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_pmc_traffic.md")):
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", "|", "`")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if (kv.get("workload") == workload and kv.get("kernel") == kernel and
                kv.get("kernel_sources_sha256") == sha):
            return float(kv["traffic_bytes_per_launch"])
    return None


C3 = dict(name="haar_batch4096_n1e3-1e5_T10-200_tanh2_fp32", count=4096,
          a=2.0, b=0.0, plain_sample=256)


def nominal_work(n, T):
    return n * T * (T + 1) / 2.0


def dense_direct(wl, x1, steps):
    """The direct method on the same GPU: draw the dense m x n Gaussian
    matrix (N(0, sigma^2) entries, torch's generator) and run the same T
    queries and map as plain matrix-vector products, in the workload's
    storage type.  Per step: the fill plus the T products."""
    import torch
    n, T = wl["n"], wl["T"]
    sig = 1.0 / np.sqrt(n)
    g = torch.Generator(device=x1.device)
    g.manual_seed(0)
    Q = torch.empty((n, n), dtype=x1.dtype, device=x1.device)

    def step():
        Q.normal_(0.0, sig, generator=g)
        x, xp = x1, torch.zeros_like(x1)
        for t in range(T):
            tr = wl["pattern"] == "alt" and t % 2 == 1
            y = torch.mv(Q.t(), x) if tr else torch.mv(Q, x)
            m = torch.clamp(torch.abs(y) - wl["a"], min=0.0)
            x, xp = torch.sign(y) * m + wl["b"] * xp, x
        return x

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    del Q
    torch.cuda.empty_cache()
    return {"ms_per_step": dt * 1e3,
            "method": "dense %dx%d Gaussian fill (torch) + %d torch.mv "
                      "products, same map, same storage type" % (n, n, T)}


def host_facts():
    """CPU model, logical CPUs and RAM of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "ram_bytes": ram}


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 oracle (single-threaded C) on the same workload: whole
    trajectories while they fit the time budget, else the first queries of
    one trajectory; elem-updates/s over what it finished."""
    import oracle
    from paper_2101_07464_amd import inputs
    n, T = wl["n"], wl["T"]
    ens = oracle.GINIBRE if wl["ensemble"] == "ginibre" else oracle.HAAR
    sig = 1.0 / np.sqrt(n) if ens == oracle.GINIBRE else 1.0
    f = oracle.DYNAMICS[wl["dyn"]]
    x1 = inputs.x1_normal(n, seed=0, scale=wl["x1_scale"])
    t0 = time.perf_counter()
    work, done, trial = 0.0, 0, 0
    while True:
        orc = oracle.HDOracle(ens, n, tmax=T, seed=0, trial=trial, sigma=sig)
        x, xp = x1.copy(), np.zeros(n)
        for t in range(T):
            tr = wl["pattern"] == "alt" and t % 2 == 1
            y = orc.query(x, tr)
            x, xp = f(y, x, xp, wl["a"], wl["b"]), x
            work += n * (t + 1)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        trial += 1
        del orc
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = dict(value=work / dt, unit="elem-updates/s", cores=1, kind="oracle",
               sample="%d queries (%d trajectories started) of the same "
                      "workload, FP64 C oracle (gcc -O3), single thread, "
                      "%.1f s" % (done, trial, dt))
    out.update(host_facts())
    return out


def batch_bytes(n, T, es=4):
    """Algorithmic bytes of one Haar trial, per query with k = t-1 reflectors
    per side: TDOT (k columns + x + the pending column), data pass (k columns
    + x + the new column), random pass (k columns + the new column + x_t
    read and x_{t+1} written by the fused map; y itself is not stored when
    the run does not record it)."""
    k = np.arange(T, dtype=np.float64)
    return float(es * np.sum(3.0 * n * k + 7.0 * n))


def run_batch(args, steps, warmup):
    """The batched workload; returns its result object."""
    import torch
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import inputs
    dev = "cuda:0"
    nb, Tb = inputs.ragged_batch(C3["count"])
    trials = [(int(n), int(T), 0, b) for b, (n, T) in enumerate(zip(nb, Tb))]
    x1 = [torch.from_numpy(inputs.x1_normal(n, seed=0, trial=b)).to(
        dev, torch.float32) for n, T, _, b in trials]
    W = float(sum(nominal_work(n, T) for n, T, _, _ in trials))
    by = sum(batch_bytes(n, T) for n, T, _, _ in trials)
    B = hd.HaarBatch(trials, dtype=torch.float32, device=dev)
    shape = {"chunks_per_workgroup": B.shape(), "source": "built-in"}
    if not args.no_autotune:
        # the library's tuner: one timed run of the whole batch per shape
        chosen, ms = B.autotune(x1, "tanh", C3["a"], C3["b"], reps=1)
        shape = {"chunks_per_workgroup": chosen, "source": "hd_batch_autotune",
                 "ms_per_run": {str(k): round(v, 2) for k, v in ms.items()}}
    for _ in range(warmup):
        B.run(x1, "tanh", C3["a"], C3["b"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.run(x1, "tanh", C3["a"], C3["b"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if B.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    # the same runs replayed from a recorded HIP graph (one submission per
    # run; recording needs a non-default stream)
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        B.set_graph(True)
        for _ in range(max(warmup, 1)):
            B.run(x1, "tanh", C3["a"], C3["b"])
        gs.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.run(x1, "tanh", C3["a"], C3["b"])
        gs.synchronize()
        elapsed_g = time.perf_counter() - t0
    if B.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    del B
    # plain: a sample of the same trials, one handle and hd_run each
    rs = np.random.default_rng(7).choice(len(trials), C3["plain_sample"],
                                         replace=False)
    Ws, tp = 0.0, 0.0
    for i in rs:
        n, T, s, k = trials[i]
        A = hd.LazyMatrix(hd.HAAR, n, t_max=T, seed=s, trial=k, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()   # the run only, not the allocation
        A.run(x1[i], T, "tanh", C3["a"], C3["b"], record=False)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t1
        Ws += nominal_work(n, T)
        del A
    plain = Ws / tp
    value = W * steps / elapsed
    gbs = by * steps / elapsed / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "elem-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": C3["name"], "trials": len(trials),
                   "elem_updates_per_step": W,
                   "algorithmic_bytes_per_step": by, "launch_shape": shape},
        "roofline": {"bound": "hbm", "kernel": "whole batched step",
                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS,
                     # counters were taken in the four-chunk shape
                     "traffic": (measured_traffic(C3["name"],
                                                  "whole batched step")
                                 if shape["chunks_per_workgroup"] == 4
                                 else None),
                     "traffic_unit": "bytes per batched step"},
        "plain_per_trial": {"value": plain, "unit": "elem-updates/s",
                            "sample": "%d of the trials, one handle each "
                                      "(hd_run), plan with the same kernels"
                                      % len(rs)},
        "batched_vs_plain": value / plain,
        "hipgraph_replay": {"value": W * steps / elapsed_g,
                            "unit": "elem-updates/s",
                            "ms_per_step": elapsed_g / steps * 1e3},
    }
    return out


C5 = dict(name="ista50_ginibre_n262144_m131072_fp32", n=262144, m=131072,
          L=50, a=0.3, theta=0.6)


def tune_shapes(args, hd, ens, lengths, dtype, k):
    """Launch shapes for the panels: measured by the library's autotuner
    (default) or the built-in rule.  Runs before any timed work."""
    lengths = sorted(set(int(v) for v in lengths))
    out = {"source": "rule"}
    if not args.no_autotune:
        rep = hd.autotune(ens, lengths, dtype, k=k)
        out = {"source": "autotune", "tuner_trajectory_queries": k,
               "tuner_us": {str(n): {str(c): round(us, 1)
                                     for c, us in t.items()}
                            for n, (_, t) in rep.items()}}
    out["chunks_per_workgroup"] = {str(n): hd.shape_rule(ens, n, dtype)
                                   for n in lengths}
    return out


GOE = dict(name="goe_n65536_K50_linear_fp32", n=65536, K=50)


def main_goe(args):
    """GOE queries (two queries of the lazy Gaussian each): x_{t+1} = G x_t
    for K steps, G ~ GOE(n) / sqrt(n), FP32."""
    import ctypes
    import torch
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import _lib, inputs
    dev = "cuda:0"
    n, K = GOE["n"], GOE["K"]
    shape = tune_shapes(args, hd, hd.GINIBRE, [n], torch.float32, 32)
    G = hd.LazyGOE(n, t_max=2 * K, seed=0, scale=1.0 / np.sqrt(n),
                   device=dev)
    x1 = torch.from_numpy(inputs.x1_normal(n, seed=0)).to(dev, torch.float32)
    buf = [torch.empty_like(x1), torch.empty_like(x1)]
    L = _lib.load()
    G._sync_stream()

    def step(i):
        G.reset(0, i)
        src = x1
        for t in range(K):
            dst = buf[t % 2]
            _lib.check(L.hd_goe_step(G._h, ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(dst.data_ptr())),
                       "hd_goe_step")
            src = dst

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if G.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    G.profile(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kinds = {k: G.profile_read(k) for k in (0, 1, 2)}
    G.profile(False)
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms, launches, nbytes = kinds[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    W = nominal_work(n, 2 * K)
    out = {
        "metric": METRIC, "value": W * args.steps / elapsed,
        "unit": "elem-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": GOE["name"], "n": n, "goe_queries": K,
                   "queries_of_Q": 2 * K, "elem_updates_per_step": W,
                   "launch_shape": shape},
        "roofline": {"bound": "hbm", "kernel": KIND_NAMES[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "launches": launches,
                     "avg_launch_us": ms * 1e3 / max(launches, 1),
                     "algorithmic_bytes_per_launch":
                         nbytes / max(launches, 1)},
    }
    print(json.dumps(out), flush=True)


def run_adjoint(args, steps, warmup, K):
    """The differentiated workload with K trials per step; returns its
    result object."""
    import torch
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import inputs
    dev = "cuda:0"
    n, m, L = C5["n"], C5["m"], C5["L"]
    sig = 1.0 / np.sqrt(m)
    xs = [torch.from_numpy(inputs.sparse_target(n, 0.1, 2.0, seed=0,
                                                trial=b)).to(dev, torch.float32)
          for b in range(K)]
    nz = [torch.from_numpy(inputs.noise(m, 0.01, seed=0, trial=b)).to(
        dev, torch.float32) for b in range(K)]
    a = [C5["a"]] * L
    th = [C5["theta"]] * L
    tq = 1 + 2 * L + 2 * (L - 1)
    shape = tune_shapes(args, hd, hd.GINIBRE, [n, m], torch.float32, 32)
    A = hd.LazyMatrix(hd.GINIBRE, n, m=m, t_max=tq, seed=0, sigma=sig,
                      device=dev)
    z = torch.zeros(n, device=dev)

    def trial(b, backward):
        A.reset(0, b)
        y = A.mv(xs[b]) + nz[b]
        X, U, V = A.lista_forward(a, th, z, y)
        if backward:
            A.lista_backward(a, th, U, V, 2.0 * (X[-1] - xs[b]))

    def timed(backward):
        for i in range(warmup):
            trial(i % K, backward)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for b in range(K):
                trial(b, backward)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_fb = timed(True)
    t_f = timed(False)
    if A.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    # the same K trials (same keys and inputs) as one lockstep batch
    # (hd_ista_run + hd_ista_grad)
    xs_b, nz_b = torch.stack(xs), torch.stack(nz)
    Bt = hd.IstaBatch(m, n, L, K, seed=0, trial0=0, sigma=sig, device=dev,
                      grad=True)

    def batch_step(backward):
        X = Bt.run(a, th, xs_b, nz_b)
        if backward:
            return X, Bt.grad(a, th, 2.0 * (X[:, -1] - xs_b))
        return X, None

    def timed_batch(backward):
        for _ in range(max(warmup, 1)):
            batch_step(backward)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch_step(backward)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tb_fb = timed_batch(True)
    tb_f = timed_batch(False)
    if Bt.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    # batched against per-trial gradients on sampled trials
    Xb, (gab, gtb, _) = batch_step(True)
    gerr = 0.0
    for b in sorted({0, K // 2, K - 1}):
        A.reset(0, b)
        y = A.mv(xs[b]) + nz[b]
        X1, U1, V1 = A.lista_forward(a, th, z, y)
        ga1, gt1, _ = A.lista_backward(a, th, U1, V1, 2.0 * (X1[-1] - xs[b]))
        for p_, q_ in ((gab[b], ga1), (gtb[b], gt1)):
            gerr = max(gerr, float((p_ - q_).abs().max() /
                                   q_.abs().max().clamp_min(1e-300)))
    del Xb, Bt
    W_fb = K * nominal_work(n, tq)
    W_f = K * nominal_work(n, 1 + 2 * L)
    out = {
        "metric": METRIC, "value": W_fb / t_fb, "unit": "elem-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": t_fb * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": C5["name"], "trials_per_step": K,
                   "queries_per_trial": tq, "elem_updates_per_step": W_fb,
                   "launch_shape": shape},
        "forward_only": {"value": W_f / t_f, "unit": "elem-updates/s",
                         "ms_per_step": t_f * 1e3,
                         "queries_per_trial": 1 + 2 * L},
        "adjoint_time_over_forward": t_fb / t_f,
        "batched": {"what": "the same trials in one lockstep batch "
                            "(hd_ista_run + hd_ista_grad)",
                    "ms_per_step": tb_fb * 1e3,
                    "forward_only_ms_per_step": tb_f * 1e3,
                    "value": W_fb / tb_fb, "unit": "elem-updates/s",
                    "batched_over_serial": t_fb / tb_fb,
                    "grad_max_rel_err_vs_serial": gerr,
                    "grad_trials_compared": sorted({0, K // 2, K - 1})},
    }
    return out


SPECTRAL = dict(name="spectral_n1e5_m2e5_K50_fp32", n=100_000, m=200_000,
                K=50)


def main_spectral(args):
    """Spectral method of Sec. 2.2: A = [I_n 0] Q, Q Haar of size
    m = 2n, measurements y = tanh|A' xi|, K power steps of m D (eq. (D_mtx))
    through the lazy Q (1 + 2K queries); a step is one whole run from a fresh
    Q (hd_reset) to x_{K+1}."""
    import torch
    import oracle
    import paper_2101_07464_amd as hd
    dev = "cuda:0"
    n, m, K = SPECTRAL["n"], SPECTRAL["m"], SPECTRAL["K"]
    rng = np.random.default_rng(0)
    xi_h = rng.standard_normal(n).astype(np.float32)
    x1_h = rng.standard_normal(n).astype(np.float32)
    xi = torch.from_numpy(xi_h).to(dev)
    x1 = torch.from_numpy(x1_h).to(dev)
    shape = tune_shapes(args, hd, hd.HAAR, [m], torch.float32, 32)
    A = hd.LazyMatrix(hd.HAAR, m, t_max=1 + 2 * K, seed=0, device=dev)

    def step(i):
        A.reset(0, i)
        return A.spectral_power(xi, x1, K)

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if A.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    A.profile(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kinds = {k: A.profile_read(k) for k in (0, 1, 2)}
    A.profile(False)
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms, launches, nbytes = kinds[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    W = nominal_work(m, 1 + 2 * K)
    out = {
        "metric": METRIC, "value": W * args.steps / elapsed,
        "unit": "elem-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": SPECTRAL["name"], "n": n, "m": m,
                   "power_steps": K, "queries": 1 + 2 * K,
                   "elem_updates_per_step": W, "launch_shape": shape},
        "roofline": {"bound": "hbm", "kernel": KIND_NAMES[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "launches": launches,
                     "avg_launch_us": ms * 1e3 / max(launches, 1),
                     "residency": "panels of at most 2 x 80 MB: largely "
                                  "cache-resident (256 MB Infinity Cache)"},
    }
    if not args.no_checks:
        z, X = step(0)
        torch.cuda.synchronize()
        orc = oracle.HDOracle(oracle.HAAR, m, tmax=1 + 2 * K, seed=0, trial=0)
        zo, Xo = oracle.spectral_power(orc, xi_h.astype(np.float64),
                                       x1_h.astype(np.float64), K)
        X = X.double().cpu().numpy()
        errs = [float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
                for a, b in zip(X, Xo)]
        # the iterates compare with the oracle's while each still brings a
        # new direction (above 1e-3 of its norm); after that they are
        # rounding-determined completions (any realisation is valid), and
        # what every realisation satisfies is checked instead: the Gram
        # matrix of the iterates of one symmetric D is a Hankel matrix, and
        # the Rayleigh quotients do not decrease
        newdir = [1.0]
        for k in range(1, len(Xo)):
            Qm, _ = np.linalg.qr(Xo[:k].T)
            r = Xo[k] - Qm @ (Qm.T @ Xo[k])
            newdir.append(float(np.linalg.norm(r) / np.linalg.norm(Xo[k])))
        kstar = next((k for k, e in enumerate(newdir) if e < 1e-3),
                     len(newdir))
        nrm = np.linalg.norm(X, axis=1)
        U = X @ X.T
        den = 0.5 * (np.outer(nrm[:-1], nrm[1:]) +
                     np.outer(nrm[1:], nrm[:-1]))
        hank = float(np.max(np.abs(U[:-1, 1:] - U[1:, :-1]) / den))
        rq = [float(X[k] @ X[k + 1] / (X[k] @ X[k])) for k in range(K)]
        mono = all(b >= a * (1 - 1e-3) for a, b in zip(rq, rq[1:]))
        c = float(abs(X[-1] @ xi_h) / np.linalg.norm(X[-1]) /
                  np.linalg.norm(xi_h))
        out["accuracy"] = {
            "oracle_iterates": {"iterates": kstar,
                                "max_rel_err": max(errs[:kstar]),
                                "tolerance": 1e-4,
                                "what": "x_1..x_k against the FP64 oracle "
                                        "while each iterate's new direction "
                                        "exceeds 1e-3 of its norm"},
            "hankel_gram_rel_err": hank, "rayleigh_nondecreasing": mono,
            "rayleigh_last": rq[-1], "cosine_with_signal": c}
    print(json.dumps(out), flush=True)


LASSO = dict(name="lasso_ista_n1000_m500_T50_trials1e5_fp32", n=1000, m=500,
             L=50, count=100_000, lam=2.0, tau=0.3, rho=0.2, sig_s=2.0,
             sig_w=0.1, direct_trials=20_000)


def ista_batch_bytes(n, m, L, es=4):
    """Algorithmic bytes of one trial of an ISTA batch run (2L + 1 queries):
    per query the TDOT streams the data side's reflector and basis columns
    and reads its input, the data pass streams the reflector columns, reads
    the input and writes the new column, the random pass streams the random
    side's reflector and basis columns and reads/writes its vectors."""
    dim = (n, m)
    kR = kL = 0
    total = 0
    for q in range(2 * L + 1):
        ds = 0 if (q == 0 or q % 2 == 1) else 1
        gs = 1 - ds
        kD, kG = (kR, kL) if ds == 0 else (kL, kR)
        if kR + kL > 0:
            total += (kD + kG + 1) * dim[ds]
        total += (kD + 2) * dim[ds]
        total += (kG + kD + 3) * dim[gs]
        if ds == 0:
            kR += 1
        else:
            kL += 1
    return total * es


def main_lasso(args):
    """The lasso experiment of Sec. 2.1 (the paper's first figure): 1e5
    independent trials of ISTA (eq. (ista)) on Gaussian Q (m = n/2,
    N(0, 1/m) entries), n = 1000, T = 50, lambda = 2, tau = 0.3,
    rho = 0.2, sigma_s = 2, sigma_w = 0.1, all trials in one lockstep batch
    (hd_ista_run).  A step runs every trial to the end.  Beside it, the
    direct method (dense Q drawn first, dense products, on the same GPU) on
    a sample of trials, with the mean squared error curves compared."""
    import torch
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import inputs
    dev = "cuda:0"
    c = LASSO
    n, m, L, C = c["n"], c["m"], c["L"], c["count"]
    sig = 1.0 / np.sqrt(m)
    xs_h, w_h = inputs.lasso_batch(C, n, m, 1 - c["rho"], c["sig_s"],
                                   c["sig_w"], seed=0)
    xs = torch.from_numpy(xs_h).to(dev, torch.float32)
    w = torch.from_numpy(w_h).to(dev, torch.float32)
    del xs_h, w_h
    a = [c["tau"]] * L
    th = [c["lam"] * c["tau"]] * L
    B = hd.IstaBatch(m, n, L, C, seed=0, trial0=0, sigma=sig, device=dev)
    for _ in range(args.warmup):
        X = B.run(a, th, xs, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X = B.run(a, th, xs, w)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if B.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    e_hd = ((X - xs.unsqueeze(1)).double().pow(2).sum(2) / n).mean(0)
    e_hd = e_hd.cpu().numpy()
    del X, B
    torch.cuda.empty_cache()
    # the direct method on a sample of trials (independent inputs)
    D = c["direct_trials"]
    xs2, w2 = inputs.lasso_batch(D, n, m, 1 - c["rho"], c["sig_s"],
                                 c["sig_w"], seed=1)
    xs2 = torch.from_numpy(xs2).to(dev, torch.float32)
    w2 = torch.from_numpy(w2).to(dev, torch.float32)
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    sq = torch.zeros(L + 1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for c0 in range(0, D, 4000):
        c1 = min(D, c0 + 4000)
        Q = torch.randn((c1 - c0, m, n), generator=g, device=dev) / np.sqrt(m)
        xstar = xs2[c0:c1]
        y = torch.bmm(Q, xstar.unsqueeze(2)).squeeze(2) + w2[c0:c1]
        x = torch.zeros_like(xstar)
        sq[0] += (x - xstar).double().pow(2).sum()
        for t in range(L):
            r = y - torch.bmm(Q, x.unsqueeze(2)).squeeze(2)
            v = x + c["tau"] * torch.bmm(r.unsqueeze(1), Q).squeeze(1)
            x = torch.sign(v) * torch.clamp(v.abs() - c["lam"] * c["tau"],
                                            min=0.0)
            sq[t + 1] += (x - xstar).double().pow(2).sum()
        del Q
    torch.cuda.synchronize()
    t_dir = time.perf_counter() - t1
    e_dir = (sq / (D * n)).cpu().numpy()
    per_trial_hd = elapsed / args.steps / C
    per_trial_dir = t_dir / D
    out = {
        "metric": "lasso ISTA trials/s (HD, lockstep batch)",
        "value": C * args.steps / elapsed,
        "unit": "trials/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": c["name"], "n": n, "m": m, "layers": L,
                   "trials": C, "queries_per_trial": 2 * L + 1},
        "roofline": {"bound": "hbm", "kernel": "whole batched step",
                     "achieved": C * ista_batch_bytes(n, m, L) /
                     (elapsed / args.steps) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": C * ista_batch_bytes(n, m, L) /
                     (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None,
                     "algorithmic_bytes_per_step":
                         C * ista_batch_bytes(n, m, L)},
        "mse_curve": {"hd": [round(float(v), 6) for v in e_hd],
                      "direct": [round(float(v), 6) for v in e_dir],
                      "max_abs_diff": float(np.max(np.abs(e_hd - e_dir))),
                      "direct_trials": D},
        "per_trial_ms": {"hd_batched": per_trial_hd * 1e3,
                         "direct_dense": per_trial_dir * 1e3,
                         "direct_over_hd": per_trial_dir / per_trial_hd},
    }
    print(json.dumps(out), flush=True)


CPLX = dict(name="unitary_haar_n1e7_T200_ctanh_c64", n=10_000_000, T=200,
            a=1.0, b=0.1, modeb=4)
CPLX_KINDS = {0: "k_cx_dots (L1: data dots | random draw dots)",
              1: "k_cx_pass<data> (data pass)",
              2: "k_cx_pass<haar out> (output pass, map fused)"}


def main_cplx(args):
    """Complex HD (Sec. 3.4) on the unitary group: one trial of T = 200
    queries y_t = Q x_t, Q Haar on U(1e7), x_{t+1} = tanh(|y_t|) e^{i arg y_t}
    + 0.1 x_t, complex64 storage (the complex counterpart of the large single
    trial).  A step is one whole trajectory from a fresh Q (hd_creset)."""
    import torch
    import oracle
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import inputs
    dev = "cuda:0"
    c = CPLX
    n, T = c["n"], c["T"]
    x1 = torch.from_numpy(inputs.cx1_normal(n, seed=0)).to(dev,
                                                          torch.complex64)
    A = hd.CLazyMatrix(hd.HAAR, n, t_max=T, seed=0, dtype=torch.complex64,
                       device=dev)

    def step(i, record=False):
        A.reset(0, i)
        return A.run(x1, T, c["a"], c["b"], record=record)

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if A.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    A.profile(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kinds = {k: A.profile_read(k) for k in (0, 1, 2)}
    A.profile(False)
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms, launches, nbytes = kinds[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    W = nominal_work(n, T)
    per_kernel = {CPLX_KINDS[k]: {
        "avg_launch_us": v[0] * 1e3 / max(v[1], 1),
        "frac": (v[2] / (v[0] * 1e-3) / 1e9 / HBM_PEAK_GBS) if v[0] else 0.0}
        for k, v in kinds.items()}
    out = {
        "metric": METRIC, "value": W * args.steps / elapsed,
        "unit": "elem-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": c["name"], "ensemble": "haar_unitary",
                   "n": n, "T": T, "pattern": "Q",
                   "dynamics": "tanh(|y|) e^{i arg y} + 0.1 x",
                   "elem_updates_per_step": W},
        "roofline": {"bound": "hbm", "kernel": CPLX_KINDS[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(c["name"], CPLX_KINDS[dom],
                                                 CPLX_SOURCES),
                     "launches": launches,
                     "avg_launch_us": ms * 1e3 / max(launches, 1),
                     "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
                     "per_kernel": per_kernel},
    }
    if not args.no_checks:
        X, Y = step(0, record=True)
        torch.cuda.synchronize()
        xn = torch.linalg.vector_norm(X[:T].to(torch.complex128), dim=1)
        yn = torch.linalg.vector_norm(Y.to(torch.complex128), dim=1)
        iso = float(((yn / xn) - 1).abs().max())
        q = c["modeb"]
        orc = oracle.CHDOracle(oracle.HAAR, n, tmax=T, seed=0, trial=0)
        Xh = X[:q].to(torch.complex128).cpu().numpy()
        Yh = Y[:q].to(torch.complex128).cpu().numpy()
        eb = max(float(np.abs(orc.mv(Xh[t]) - Yh[t]).max() /
                       np.abs(Yh[t]).max()) for t in range(q))
        out["accuracy"] = {
            "oracle_replay": {"queries": q, "max_rel_err": eb,
                              "tolerance": 1e-4},
            "unitary_isometry": {"answers": T, "max_err": iso,
                                 "what": "max_t | ||y_t|| / ||x_t|| - 1 |"}}
        del X, Y
    print(json.dumps(out), flush=True)


def stream_reference():
    """What plain streaming kernels reach on the same GPU, as context for
    the roofline fractions (which are taken against the 8 TB/s peak): a
    4 GiB float32 copy (torch.mul into another buffer, read + write bytes)
    and a 4 GiB read-only reduction (torch.sum), best of five each, timed
    with events on the current stream."""
    import torch
    n = 1 << 30
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    res = {}
    for name, fn, nbytes in (
            ("copy", lambda: torch.mul(src, 1.0, out=dst), 8 * n),
            ("read", lambda: torch.sum(src), 4 * n)):
        fn()
        best = None
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name + "_GBs"] = nbytes / (best * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    res["what"] = ("torch copy and sum of 4 GiB float32 on the same GPU, "
                   "best of five: the streaming rate plain kernels reach")
    return res


def copy_calibration():
    """A plain device copy of known size (read 1 GiB, write 1 GiB, five
    times) for scaling the PMC byte counters of the panel kernels."""
    import torch
    n = 1 << 28
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel": "torch.mul(src, 1.0, out=dst), float32",
                      "bytes_read_per_launch": n * 4,
                      "bytes_written_per_launch": n * 4, "launches": 5}),
          flush=True)


def single_trial_checks(hd, A, x1, wl, n_modeb):
    """Accuracy of the timed configuration: one more trajectory (key (0, 0),
    same launch shape) with every x_t and y_t recorded.  The FP64 oracle
    answers the GPU's own first n_modeb query vectors (per-step replay), and
    the whole trajectory is checked against what holds for any orthogonal Q
    (||y_t|| = ||x_t|| and Y'Y = X'X) or, for the Gaussian ensemble, only
    the replay is reported."""
    import torch
    import oracle
    n, T = wl["n"], wl["T"]
    A.reset(0, 0)
    X, Y = A.run(x1, T, wl["dyn"], wl["a"], wl["b"], wl["pattern"])
    torch.cuda.synchronize()
    if A.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    out = {}
    kb = min(n_modeb, T)
    Xh = X[:kb].double().cpu().numpy()
    Yh = Y[:kb].double().cpu().numpy()
    ens = oracle.GINIBRE if wl["ensemble"] == "ginibre" else oracle.HAAR
    sig = 1.0 / np.sqrt(n) if ens == oracle.GINIBRE else 1.0
    orc = oracle.HDOracle(ens, n, tmax=kb, seed=0, trial=0, sigma=sig)
    tr = [wl["pattern"] == "alt" and t % 2 == 1 for t in range(kb)]
    Yo = oracle.replay(orc, Xh, tr)
    del orc
    err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
              for a, b in zip(Yh, Yo))
    out["oracle_replay"] = {
        "queries": kb, "max_rel_err": err,
        "tolerance": 1e-11 if wl["f64"] else 1e-4,
        "what": "max over the first %d answers of max|y_gpu - y_oracle| / "
                "max|y_oracle|, the FP64 oracle answering the GPU's own "
                "query vectors" % kb}
    if wl["ensemble"] == "haar" and wl["pattern"] == "Q":
        iso, G = 0.0, None
        for r0 in range(0, T, 25):
            xs = X[r0:min(r0 + 25, T)].double()
            ys = Y[r0:min(r0 + 25, T)].double()
            nx = torch.linalg.vector_norm(xs, dim=1)
            ny = torch.linalg.vector_norm(ys, dim=1)
            iso = max(iso, float(torch.max(torch.abs(ny / nx - 1.0))))
        Xd = X[:T].double()
        Gx = Xd @ Xd.T
        del Xd
        Yd = Y[:T].double()
        Gy = Yd @ Yd.T
        del Yd
        gram = float(torch.max(torch.abs(Gy - Gx)) / torch.max(torch.abs(Gx)))
        out["haar_invariants"] = {
            "answers": T, "max_isometry_err": iso, "gram_rel_err": gram,
            "what": "max_t | ||y_t|| / ||x_t|| - 1 | and max|Y'Y - X'X| / "
                    "max|X'X| over every answer of the trajectory (both hold "
                    "for any orthogonal Q)"}
    del X, Y
    torch.cuda.empty_cache()
    return out


def run_single(args, wl):
    """One of the single-trial workloads (c1, c2, c4); returns its line."""
    import torch
    import paper_2101_07464_amd as hd
    from paper_2101_07464_amd import inputs

    n, T = wl["n"], wl["T"]
    dev = "cuda:0"
    dtype = torch.float64 if wl["f64"] else torch.float32
    ens = hd.GINIBRE if wl["ensemble"] == "ginibre" else hd.HAAR
    sig = 1.0 / np.sqrt(n) if ens == hd.GINIBRE else 1.0
    x1 = torch.from_numpy(inputs.x1_normal(n, seed=0, scale=wl["x1_scale"]))
    x1 = x1.to(dev, dtype)
    shape = tune_shapes(args, hd, ens, [n], dtype, min(T, 32))
    A = hd.LazyMatrix(ens, n, t_max=T, seed=0, sigma=sig, dtype=dtype,
                      device=dev)

    def step(i):
        A.reset(0, i)
        A.run(x1, T, wl["dyn"], wl["a"], wl["b"], wl["pattern"],
              record=False)

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if A.status() != 0:
        raise RuntimeError("device reported a non-finite reflector norm")
    # Kernel durations: the same steps again with HIP events recorded by the
    # dispatches of every panel launch (on the library's stream).  Events
    # add work between launches, so this pass is kept out of the timed
    # region above.
    A.profile(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kinds = {k: A.profile_read(k) for k in (0, 1, 2)}
    A.profile(False)
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms, launches, nbytes = kinds[dom]
    kname = KERNEL_OF_KIND[(dom, wl["ensemble"])]
    traffic = measured_traffic(wl["name"], kname)
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    W = nominal_work(n, T)
    out = {
        "metric": METRIC,
        "value": W * args.steps / elapsed,
        "unit": "elem-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl["f64"] else "f32",
        "data": "synthetic",
        "config": {"workload": wl["title"], "n": n, "T": T,
                   "ensemble": wl["ensemble"], "pattern": wl["pattern"],
                   "dynamics": wl["dyn_text"],
                   "precision": ("FP64 panels and vectors" if wl["f64"] else
                                 "FP32 panels and vectors, FP64 accumulation,"
                                 " norms, signs and T"),
                   "elem_updates_per_step": W, "launch_shape": shape},
        "roofline": {"bound": "hbm", "kernel": KIND_NAMES[dom],
                     "kernel_symbol": kname,
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_source": ("FETCH_SIZE + WRITE_SIZE per launch "
                                        "from the committed rocprofv3 PMC "
                                        "summary of these kernel sources "
                                        "(profiles/)" if traffic else
                                        "no PMC summary for these kernel "
                                        "sources"),
                     "launches": launches,
                     "avg_launch_us": ms * 1e3 / max(launches, 1),
                     "algorithmic_bytes_per_launch":
                         nbytes / max(launches, 1)},
    }
    for k in (0, 1, 2):
        kms, kl, kb = kinds[k]
        if kl:
            out["roofline"].setdefault("per_kernel", {})[
                KERNEL_OF_KIND[(k, wl["ensemble"])]] = {
                    "avg_launch_us": kms * 1e3 / kl,
                    "frac": kb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if wl.get("cache_resident"):
        out["roofline"]["residency"] = wl["cache_resident"]
    if not args.no_checks:
        out["accuracy"] = single_trial_checks(hd, A, x1, wl, wl["modeb"])
    A.close()
    del A
    torch.cuda.empty_cache()
    if not args.no_checks:
        out["roofline"]["stream_reference"] = stream_reference()
    if wl.get("dense", False):
        out["dense_direct"] = dense_direct(wl, x1, args.steps)
        out["vs_dense_direct"] = (out["dense_direct"]["ms_per_step"] /
                                  out["ms_per_step"])
    return out


def extras(args, out):
    """The batched and the differentiated workloads, reduced to their
    ratios against the plain per-trial launch and the forward-only run."""
    t0 = time.perf_counter()
    try:
        b = run_batch(args, args.extra_steps, 1)
        out["batched_vs_plain"] = b["batched_vs_plain"]
        out["batched"] = {
            "workload": b["config"]["workload"], "value": b["value"],
            "unit": b["unit"], "ms_per_step": b["ms_per_step"],
            "steps": b["steps"], "frac_hbm_whole_step": b["roofline"]["frac"],
            "launch_shape": b["config"]["launch_shape"],
            "plain_per_trial": b["plain_per_trial"],
            "hipgraph_replay_ms_per_step":
                b["hipgraph_replay"]["ms_per_step"]}
    except Exception as e:  # reported, not fatal for the headline line
        out["batched_error"] = repr(e)
    try:
        a = run_adjoint(args, args.extra_steps, 1, args.extra_c5_trials)
        out["adjoint_time_over_forward"] = a["adjoint_time_over_forward"]
        out["adjoint"] = {
            "workload": a["config"]["workload"], "value": a["value"],
            "unit": a["unit"], "ms_per_step": a["ms_per_step"],
            "trials_per_step": a["config"]["trials_per_step"],
            "forward_only": a["forward_only"], "batched": a["batched"]}
    except Exception as e:
        out["adjoint_error"] = repr(e)
    out["extras_wall_s"] = time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4",
                    choices=sorted(list(WORKLOADS) +
                                   ["c3", "c5", "goe", "spectral", "lasso",
                                    "cplx"]))
    ap.add_argument("--c5-trials", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only the plain copy used to scale PMC bytes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the recorded trajectory checked against the "
                         "oracle and the invariants")
    ap.add_argument("--no-extras", action="store_true",
                    help="c4 only: skip the batched and differentiated "
                         "ratios")
    ap.add_argument("--extra-steps", type=int, default=2)
    ap.add_argument("--extra-c5-trials", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in launch-shape rule instead of "
                         "timing the candidate shapes first")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU "
              "path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        print(json.dumps(run_batch(args, args.steps, args.warmup)),
              flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(run_adjoint(args, args.steps, args.warmup,
                                     args.c5_trials)), flush=True)
        return
    if args.workload == "goe":
        main_goe(args)
        return
    if args.workload == "spectral":
        main_spectral(args)
        return
    if args.workload == "lasso":
        main_lasso(args)
        return
    if args.workload == "cplx":
        main_cplx(args)
        return
    wl = WORKLOADS[args.workload]
    out = run_single(args, wl)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    if args.workload == "c4" and not args.no_extras:
        extras(args, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
