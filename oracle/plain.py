"""Plaintext WiSARD and client-side steps of the oracle (numpy, plain loops).

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark use it.

* quantisation and thermometer encoding (Sec. 2.4.2-2.4.3)
* f_comp and the Integer WiSARD: training (Alg. 4), evaluation (Alg. 2)
* activations used with PD-act (Sec. 3.2, 3.5.1) and ArgMax
* the layout map from a plaintext model W to the decrypted cells of the
  Homomorphic WiSARD H (Def. 2 with the IVP encoding of Alg. 5)
"""
from __future__ import annotations

import numpy as np

from . import ceil_log2, permutation


# -- client preprocessing ------------------------------------------------------

def thermometer(x: int, size: int) -> list[int]:
    """T_size(x): t_i = 1 for i < x, 0 otherwise (Sec. 2.4.3)."""
    return [1 if i < x else 0 for i in range(size)]


def quantize_u8(v: np.ndarray, levels: int) -> np.ndarray:
    """Linear quantisation of uint8 values to [0, levels]:
    min(levels, floor(v * (levels + 1) / 256)) (Sec. 2.4.2 with r = 256/(levels+1))."""
    v = np.asarray(v, np.int64)
    return np.minimum(levels, (v * (levels + 1)) // 256)


def quantize_minmax(x: np.ndarray, levels: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Min-max scaling to [0, 1] then floor(x * (levels + 1)) clipped to levels (per feature)."""
    x = np.asarray(x, np.float64)
    span = np.where(hi > lo, hi - lo, 1.0)
    u = np.clip((x - lo) / span, 0.0, 1.0)
    return np.minimum(levels, np.floor(u * (levels + 1)).astype(np.int64))


def encode(levels_arr: np.ndarray, size: int) -> np.ndarray:
    """Thermometer-encode every value of each sample; value v occupies bits
    [v*size, (v+1)*size) of the sample's bit vector."""
    lv = np.asarray(levels_arr).reshape(len(levels_arr), -1)
    n, m = lv.shape
    out = np.zeros((n, m * size), np.uint8)
    for i in range(n):
        for v in range(m):
            out[i, v * size:(v + 1) * size] = thermometer(int(lv[i, v]), size)
    return out


# -- WiSARD (Def. 1, Alg. 2, Alg. 4) ---------------------------------------------

def f_comp(t, d: int, a: int) -> int:
    """Address of tuple d: sum_i t[i + a d] 2^i over the tuple's bits, LSB
    first (Def. 1; the printed upper bound is read as exclusive)."""
    s = len(t)
    addr = 0
    for i in range(min(a, s - a * d)):
        addr += int(t[i + a * d]) << i
    return addr


def train_integer(X: np.ndarray, y: np.ndarray, l: int, a: int, pi: np.ndarray) -> np.ndarray:
    """Integer WiSARD training (Alg. 4): W[L_i][j][f_comp(pi(T_i), j)] += 1."""
    n, s = X.shape
    k = -(-s // a)
    W = np.zeros((l, k, 1 << a), np.int64)
    for i in range(n):
        t = X[i][pi]
        for j in range(k):
            W[int(y[i]), j, f_comp(t, j, a)] += 1
    return W


def act_bin(x, thr: int = 0):
    """binarisation / bleaching threshold: 1 if x > thr else 0"""
    return (np.asarray(x) > thr).astype(np.int64)


def act_log(x):
    """floor(log2(x + 1)) on non-negative integers"""
    x = np.asarray(x, np.int64)
    out = np.zeros_like(x)
    v = x + 1
    while np.any(v > 1):
        out += (v > 1)
        v = v >> 1
    return out


def act_blog(x, cap: int = 4):
    """min(floor(log2(x + 1)), cap)"""
    return np.minimum(act_log(x), cap)


def activate(x, kind: str = "bin", thr: int = 0, cap: int = 4):
    if kind == "bin":
        return act_bin(x, thr)
    if kind == "log":
        return act_log(x)
    if kind == "blog":
        return act_blog(x, cap)
    if kind == "none":
        return np.asarray(x, np.int64)
    raise ValueError(kind)


def argmax_lowest(u) -> int:
    """ArgMax with ties going to the lowest class index."""
    u = list(u)
    best = 0
    for c in range(1, len(u)):
        if u[c] > u[best]:
            best = c
    return best


def ram_scores(W: np.ndarray, x: np.ndarray, a: int, pi: np.ndarray) -> np.ndarray:
    """u[c][j] = W[c][j][f_comp(pi(x), j)] (the per-RAM cells Alg. 2 sums)."""
    l, k, _ = W.shape
    t = x[pi]
    out = np.zeros((l, k), np.int64)
    for c in range(l):
        for j in range(k):
            out[c, j] = W[c, j, f_comp(t, j, a)]
    return out


def predict(W, x, a, pi, kind="bin", thr=0, cap=4) -> int:
    """Alg. 2 with an activation applied to every selected cell, ArgMax lowest."""
    u = ram_scores(W, x, a, pi)
    return argmax_lowest(activate(u, kind, thr, cap).sum(axis=1))


def pd_act_predict(u_cells, kind="bin", thr=0, cap=4) -> int:
    """PD-act on the client: decrypted per-RAM cells u[c][j] -> f_act -> sum -> ArgMax."""
    return argmax_lowest(activate(np.asarray(u_cells), kind, thr, cap).sum(axis=1))


# -- layout of the homomorphic model -----------------------------------------------

def model_row(d: int, z: int, L: int, l: int) -> int:
    """Row of H that holds tree leaf d of a RAM with z tree bits: with z >= L,
    leaf d = c + 2^L w (class c < l) is row w l + c, so a row holds
    l 2^(z-L) = l 2^a / N ciphertexts (Def. 2); with z < L row d is leaf d."""
    if z < L:
        return d
    c, w = d % (1 << L), d >> L
    return w * l + c if c < l else -1


def expected_model_cells(W: np.ndarray, s: int, l: int, a: int, N: int, layout: int = 0) -> np.ndarray:
    """Decrypted content of H (shape [k0][k1][N]) implied by a plaintext Integer
    WiSARD W.  Layout 0 (label-pruned): with m = c + 2^L addr, tree leaf
    d = m mod 2^z_j of RAM j holds W[c][j][addr] at coefficient m >> z_j, and
    leaf d is row model_row(d) of H[j].  Layout 1 (class-packed): with
    m = addr + 2^a_j c, row m mod 2^z_j holds it at coefficient m >> z_j.
    Layout 2 (several RAMs per row, when 2^(L+a) < N): RAM j's layout-1 row
    sits at offset (j mod r) 2^(L+a) of row j / r, r = N / 2^(L+a); the
    result has shape [ceil(k0 / r)][1][N].  Every other cell is 0."""
    L = ceil_log2(l)
    logN = N.bit_length() - 1
    k0 = -(-s // a)
    nb_full = L + a
    z0 = nb_full - min(nb_full, logN)
    if layout == 0:
        k1 = l << (z0 - L) if z0 >= L else 1 << z0
    else:
        k1 = 1 << z0
    if layout == 2:
        one = expected_model_cells(W, s, l, a, N, layout=1)
        r = N >> nb_full if nb_full < logN else 1
        if r == 1:
            return one
        out = np.zeros((-(-k0 // r), 1, N), np.int64)
        for j in range(k0):
            off = (j % r) << nb_full
            out[j // r, 0, off:off + (1 << nb_full)] = one[j, 0, :1 << nb_full]
        return out
    out = np.zeros((k0, k1, N), np.int64)
    for j in range(k0):
        aj = min(a, s - j * a)
        nb = L + aj
        z = nb - min(nb, logN)
        for c in range(l):
            for addr in range(1 << aj):
                if layout == 0:
                    m = c + (addr << L)
                    out[j, model_row(m % (1 << z), z, L, l), m >> z] = W[c, j, addr]
                else:
                    m = addr + (c << aj)
                    out[j, m % (1 << z), m >> z] = W[c, j, addr]
    return out


__all__ = [
    "thermometer", "quantize_u8", "quantize_minmax", "encode", "f_comp", "train_integer",
    "act_bin", "act_log", "act_blog", "activate", "argmax_lowest", "ram_scores", "predict",
    "pd_act_predict", "model_row", "expected_model_cells", "permutation",
]
