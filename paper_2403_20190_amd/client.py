"""Client-side steps around the encrypted path (numpy, vectorised).

* preprocessing: linear / min-max quantisation (Sec. 2.4.2) and thermometer
  encoding (Sec. 2.4.3) of each sample on its own;
* label bits, LSB first (Alg. 6 feeds them before the tuple bits);
* PD-act (Sec. 3.5.1): decrypted per-RAM cells -> activation -> sum ->
  ArgMax, ties to the lowest class.
"""
from __future__ import annotations

import numpy as np


def ceil_log2(l: int) -> int:
    return max(0, int(l - 1).bit_length())


def quantize_u8(v, levels: int) -> np.ndarray:
    """uint8 -> level in [0, levels]: min(levels, floor(v (levels+1) / 256))."""
    v = np.asarray(v, np.int64)
    return np.minimum(levels, (v * (levels + 1)) // 256)


def quantize_minmax(x, levels: int, lo, hi) -> np.ndarray:
    """Per-feature min-max scaling to [0, 1], then min(levels, floor(u (levels+1)))."""
    x = np.asarray(x, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    span = np.where(hi > lo, hi - lo, 1.0)
    u = np.clip((x - lo) / span, 0.0, 1.0)
    return np.minimum(levels, np.floor(u * (levels + 1)).astype(np.int64))


def thermometer(levels, size: int) -> np.ndarray:
    """Thermometer code of every value: value v of a sample becomes bits
    [v*size, (v+1)*size) with bit i set iff i < level."""
    lv = np.asarray(levels, np.int64)
    lv = lv.reshape(lv.shape[0], -1)
    bits = (np.arange(size)[None, None, :] < lv[:, :, None]).astype(np.uint8)
    return bits.reshape(lv.shape[0], -1)


def label_bits(y, l: int) -> np.ndarray:
    L = ceil_log2(l)
    y = np.asarray(y, np.int64)
    return ((y[:, None] >> np.arange(L)[None, :]) & 1).astype(np.uint8).reshape(len(y), L)


def activate(x, kind: str = "bin", thr: int = 0, cap: int = 4) -> np.ndarray:
    """bin: x > thr; log: floor(log2(x+1)); blog: min(floor(log2(x+1)), cap)."""
    x = np.asarray(x, np.int64)
    if kind == "bin":
        return (x > thr).astype(np.int64)
    lg = np.zeros_like(x)
    nz = x > 0
    lg[nz] = np.floor(np.log2(x[nz] + 1)).astype(np.int64)
    # exact correction where float rounding could move across a power of two
    lg = np.where((1 << (lg + 1)) <= x + 1, lg + 1, lg)
    lg = np.where((1 << lg) > x + 1, lg - 1, lg)
    if kind == "log":
        return lg
    if kind == "blog":
        return np.minimum(lg, cap)
    if kind == "none":
        return x
    raise ValueError(kind)


def pd_act_predict(cells, kind: str = "bin", thr: int = 0, cap: int = 4) -> np.ndarray:
    """cells[n][l][k0] decrypted RAM cells -> predicted class per sample."""
    scores = activate(cells, kind, thr, cap).sum(axis=2)
    return np.argmax(scores, axis=1)  # numpy takes the first maximum: the lowest index


def save_checkpoint(path, model, class_count=None, **meta):
    """Write a model (and its class counter) with integer metadata to an .npz
    file: the parameters, the shape, and the number of samples trained so far
    (the cursor to resume from).  Training adds each sample's contribution, so
    resuming is training the remaining samples into the loaded model (or
    merging with hw_rlwe_add a model trained on them elsewhere)."""
    import numpy as np
    arrays = {"model": model.detach().cpu().numpy()}
    if class_count is not None:
        arrays["class_count"] = class_count.detach().cpu().numpy()
    for k, v in meta.items():
        arrays["meta_" + k] = np.asarray(int(v), np.int64)
    np.savez(path, **arrays)


def load_checkpoint(path, device="cuda"):
    """(model, class_count or None, meta) from save_checkpoint; loaded
    without unpickling."""
    import numpy as np
    import torch
    with np.load(path, allow_pickle=False) as z:
        model = torch.from_numpy(z["model"]).to(device)
        cnt = torch.from_numpy(z["class_count"]).to(device) if "class_count" in z.files else None
        meta = {k[len("meta_"):]: int(z[k]) for k in z.files if k.startswith("meta_")}
    return model, cnt, meta
