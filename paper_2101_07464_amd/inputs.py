"""Seeded synthetic inputs for the Householder Dice workloads.

This module only draws input vectors and workload shapes (initial conditions,
sparse targets, noise, ragged batch sizes).  It contains none of the method's
arithmetic: the random numbers that Householder Dice itself reveals are drawn
inside the library (and, independently, inside the oracle) from the Philox
stream keyed on (seed, trial).

Every generator is numpy's PCG64 seeded with (seed, trial, tag); the tags keep
the streams of different inputs apart.
"""
import numpy as np

TAG_X1 = 1        # initial condition x_1
TAG_SUPPORT = 2   # support of the sparse target x*
TAG_AMPL = 3      # amplitudes of x*
TAG_NOISE = 4     # observation noise
TAG_BATCH = 5     # ragged batch shapes


def rng(seed, trial, tag):
    return np.random.default_rng(np.random.SeedSequence([seed, trial, tag]))


def x1_normal(n, seed=0, trial=0, scale=None):
    """x_1 ~ N(0, scale^2 I_n); scale defaults to 1/sqrt(n) (x_1 ~ N(0, I/n))."""
    s = 1.0 / np.sqrt(n) if scale is None else scale
    return rng(seed, trial, TAG_X1).standard_normal(n) * s


def cx1_normal(n, seed=0, trial=0):
    """Complex x_1 with i.i.d. circular entries, E|x_i|^2 = 1 (real and
    imaginary parts N(0, 1/2))."""
    g = rng(seed, trial, TAG_X1).standard_normal((2, n))
    return (g[0] + 1j * g[1]) / np.sqrt(2.0)


def sparse_target(n, p_nonzero, sigma_s, seed=0, trial=0):
    """Bernoulli-Gaussian vector: entry nonzero with probability p_nonzero,
    nonzero entries N(0, sigma_s^2) (the prior of the lasso example)."""
    sup = rng(seed, trial, TAG_SUPPORT).random(n) < p_nonzero
    amp = rng(seed, trial, TAG_AMPL).standard_normal(n) * sigma_s
    return np.where(sup, amp, 0.0)


def noise(m, sigma_w, seed=0, trial=0):
    return rng(seed, trial, TAG_NOISE).standard_normal(m) * sigma_w


def ragged_batch(count, n_lo=1000, n_hi=100000, t_lo=10, t_hi=200, seed=0):
    """Per-trial (n_b, T_b): n_b log-uniform in [n_lo, n_hi], T_b uniform in
    [t_lo, t_hi]."""
    g = rng(seed, 0, TAG_BATCH)
    u = g.random(count)
    n = np.floor(n_lo * (n_hi / n_lo) ** u).astype(np.int64)
    n = np.clip(n, n_lo, n_hi)
    T = g.integers(t_lo, t_hi + 1, size=count).astype(np.int64)
    return n, T


def lasso_batch(count, n, m, p_nonzero, sigma_s, sigma_w, seed=0):
    """Inputs of `count` lasso trials at once: rows of x* (count x n,
    Bernoulli-Gaussian as sparse_target) and of the noise w (count x m,
    N(0, sigma_w^2)), drawn from streams of their own (seeded with
    (seed, 2^32, tag), apart from every per-trial stream)."""
    def g(tag):
        return np.random.default_rng(np.random.SeedSequence([seed, 1 << 32,
                                                             tag]))
    sup = g(TAG_SUPPORT).random((count, n)) < p_nonzero
    amp = g(TAG_AMPL).standard_normal((count, n)) * sigma_s
    w = g(TAG_NOISE).standard_normal((count, m)) * sigma_w
    return np.where(sup, amp, 0.0), w
