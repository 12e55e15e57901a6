"""Seeded synthetic workloads shaped like the paper's datasets.

This module holds no arithmetic of the method: it only draws raw samples
(uint8 images, float features or bit vectors) and labels with numpy's PCG64.
Both the GPU path and the CPU oracle consume what it returns; the
preprocessing (quantisation, thermometer encoding), encryption and everything
after it are implemented separately on each side.

Shapes follow the paper's datasets (Sec. 4.1), which are not available here:
MNIST (28x28 grey digits, 10 classes), HAM10000 (28x28x3 skin images, 7
skewed classes), Wisconsin breast cancer (30 real features, 2 classes 357/212).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def tiny(seed: int = 0, n_train: int = 32, n_test: int = 16):
    """8x8 uint8 images, uniform over 0..255; labels alternate 0/1."""
    g = _rng(seed)
    n = n_train + n_test
    X = g.integers(0, 256, size=(n, 64), dtype=np.uint8)
    y = (np.arange(n) % 2).astype(np.int64)
    return X[:n_train], y[:n_train], X[n_train:], y[n_train:]


def _blob_templates(g, l, h, w, channels, blobs=3):
    """Per-class templates made of isotropic Gaussian blobs (centres uniform in
    the middle of the image, std 2-4 px, peak 0.6-1.0 of full scale)."""
    yy, xx = np.mgrid[0:h, 0:w]
    tmpl = np.zeros((l, h, w, channels), np.float64)
    for c in range(l):
        for _ in range(blobs):
            cy, cx = g.uniform(6, h - 6), g.uniform(6, w - 6)
            sd = g.uniform(2.0, 4.0)
            peak = 255.0 * g.uniform(0.6, 1.0)
            col = g.uniform(0.3, 1.0, size=channels) if channels > 1 else np.ones(1)
            bump = peak * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sd * sd))
            tmpl[c] += bump[:, :, None] * col[None, None, :]
    return np.minimum(tmpl, 255.0)


def _images(g, tmpl, labels, noise):
    out = tmpl[labels] + g.normal(0.0, noise, size=tmpl[labels].shape)
    return np.clip(np.rint(out), 0, 255).astype(np.uint8).reshape(len(labels), -1)


def mnist_like(seed: int = 1, per_class_train: int = 100, per_class_test: int = 100, noise: float = 30.0):
    """28x28 uint8 images, 10 balanced classes, blob templates plus N(0, 30^2) noise."""
    g = _rng(seed)
    l = 10
    tmpl = _blob_templates(g, l, 28, 28, 1)
    ytr = np.repeat(np.arange(l), per_class_train)
    yte = np.repeat(np.arange(l), per_class_test)
    g.shuffle(ytr)
    g.shuffle(yte)
    return _images(g, tmpl, ytr, noise), ytr, _images(g, tmpl, yte, noise), yte


HAM_PRIORS = (0.67, 0.11, 0.11, 0.05, 0.03, 0.02, 0.01)


def ham_like(seed: int = 3, n_train: int = 10000, n_test: int = 1000, noise: float = 30.0):
    """28x28x3 uint8 images, 7 classes with the skewed priors of HAM10000."""
    g = _rng(seed)
    l = len(HAM_PRIORS)
    tmpl = _blob_templates(g, l, 28, 28, 3)

    def labels(n):
        counts = [int(round(p * n)) for p in HAM_PRIORS]
        counts[0] += n - sum(counts)
        y = np.concatenate([np.full(k, c) for c, k in enumerate(counts)]).astype(np.int64)
        g.shuffle(y)
        return y

    ytr, yte = labels(n_train), labels(n_test)
    return _images(g, tmpl, ytr, noise), ytr, _images(g, tmpl, yte, noise), yte


def wisconsin_like(seed: int = 4, n0: int = 357, n1: int = 212):
    """30 float32 features per sample from per-class Gaussians N(mu_c, I)."""
    g = _rng(seed)
    mu0 = g.normal(0.0, 1.0, 30)
    mu1 = mu0 + 0.8 * g.normal(0.0, 1.0, 30)
    y = np.concatenate([np.zeros(n0, np.int64), np.ones(n1, np.int64)])
    g.shuffle(y)
    X = np.where(y[:, None] == 0, mu0, mu1) + g.normal(0.0, 1.0, (len(y), 30))
    return X.astype(np.float32), y


def prototype_bits(seed: int, n: int, s: int, l: int, flip: float = 0.1):
    """Bit vectors from per-class Bernoulli(0.5) prototypes with `flip` noise."""
    g = _rng(seed)
    proto = g.integers(0, 2, size=(l, s), dtype=np.uint8)
    y = g.integers(0, l, size=n).astype(np.int64)
    flips = (g.random((n, s)) < flip).astype(np.uint8)
    return proto[y] ^ flips, y


def batched_jobs(seed: int = 2, njobs: int = 256):
    """Shapes of the uneven training jobs: n ~ U{32..2000}, s ~ U{128..2352},
    a ~ U{8..12}, l ~ U{2..10}, ring degree 2048 or 4096."""
    g = _rng(seed)
    jobs = []
    for j in range(njobs):
        jobs.append(dict(
            n=int(g.integers(32, 2001)), s=int(g.integers(128, 2353)), a=int(g.integers(8, 13)),
            l=int(g.integers(2, 11)), N=int(g.choice([2048, 4096])), seed=int(g.integers(0, 2**62)),
        ))
    return jobs


def poisson_arrivals(seed: int, qps: float, count: int):
    """Arrival times (s) of a Poisson process with rate qps."""
    g = _rng(seed)
    return np.cumsum(g.exponential(1.0 / qps, size=count))
