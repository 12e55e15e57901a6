"""The training entry point that allocates no device memory
(hw_wisard_train_encrypted_noalloc) against hw_wisard_train_encrypted on the
same ciphertexts: the same model and class-counter bits, on calls in a row
whose later ones are smaller (the fixed scratch keeps the previous call's
contents, which must not leak into the next), across two parameter sets that
share the one scratch array, and its refusal of a shape whose one-sample
workspace exceeds that array."""
import numpy as np
import pytest

from gpu_helpers import Pair, host_u32, zeros_u32
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu


def both_paths(pair, xr, yr, n, class_count=True):
    """(model, counter) from the allocating and the no-allocation entry points"""
    import torch
    out = []
    for fn in (pair.ctx.train, pair.ctx.train_noalloc):
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        cnt = zeros_u32(2, pair.nq, pair.N) if class_count else None
        fn(pair.shape, xr, yr, n, H, cnt)
        torch.cuda.synchronize()
        out.append((host_u32(H), None if cnt is None else host_u32(cnt)))
    return out


def test_noalloc_equals_allocating_path_on_consecutive_calls():
    from paper_2403_20190_amd import hwisard as HW
    # call 1: MNIST-shaped parameters and shape (196 RAMs, 5-level tree), three
    # samples; one sample's workspace is 213 MB, so the call runs three
    # sub-batches through the scratch
    X, y = synth.prototype_bits(31, 3, 2352, 10, flip=0.1)
    big = Pair(2048, 2, 1024, 2352, 10, 12, X, y, seed=31)
    assert (big.k0 + 1) * (2 ** 5 + 1) * big.ctx.rlwe_words * 4 <= HW.NOALLOC_SCRATCH_BYTES
    xr, yr = big.encrypt_dev(), big.encrypt_labels_dev()
    (H0, c0), (H1, c1) = both_paths(big, xr, yr, 3)
    assert np.array_equal(H0, H1) and np.array_equal(c0, c1)
    assert H0.any()
    # call 2, smaller: one different sample on the same context
    X2, y2 = synth.prototype_bits(32, 1, 2352, 10, flip=0.1)
    small = Pair(2048, 2, 1024, 2352, 10, 12, X2, y2, seed=32)
    xr2, yr2 = small.encrypt_dev(), small.encrypt_labels_dev()
    (H0, c0), (H1, c1) = both_paths(small, xr2, yr2, 1)
    assert np.array_equal(H0, H1) and np.array_equal(c0, c1)
    # call 3, smaller still, on another parameter set (N = 1024, one prime)
    # that shares the device's scratch: a ragged last tuple, no class counter
    X3, y3 = synth.prototype_bits(33, 5, 100, 3, flip=0.2)
    tiny = Pair(1024, 1, 64, 100, 3, 8, X3, y3, seed=33)
    xr3, yr3 = tiny.encrypt_dev(), tiny.encrypt_labels_dev()
    (H0, _), (H1, _) = both_paths(tiny, xr3, yr3, 5, class_count=False)
    assert np.array_equal(H0, H1)
    # and one more call of the first, larger shape after the small ones
    (H0, c0), (H1, c1) = both_paths(big, xr, yr, 2)
    assert np.array_equal(H0, H1) and np.array_equal(c0, c1)


def test_noalloc_accumulates_in_place_and_refuses_oversized_shapes():
    import torch

    from paper_2403_20190_amd import hwisard as HW
    X, y = synth.prototype_bits(34, 4, 128, 2, flip=0.1)
    pair = Pair(1024, 1, 64, 128, 2, 8, X, y, seed=34)
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    # two calls into the same model equal one call over all samples
    Hsplit = zeros_u32(pair.k0, pair.k1, 2, 1, 1024)
    pair.ctx.train_noalloc(pair.shape, xr[:2 * 128], yr[:2], 2, Hsplit, None)
    pair.ctx.train_noalloc(pair.shape, xr[2 * 128:], yr[2:], 2, Hsplit, None)
    Hone = zeros_u32(pair.k0, pair.k1, 2, 1, 1024)
    pair.ctx.train(pair.shape, xr, yr, 4, Hone, None)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(Hsplit), host_u32(Hone))
    # the HAM-shaped set: (393 RAM blocks) x (8 + 1 slots) x 96 KiB > 256 MiB per sample
    ctx = HW.Context(4096, 3, 16384)
    sh = HW.shape(4704, 7, 12, 5)
    k0, k1, _ = ctx.dims(sh)
    H = zeros_u32(k0, k1, 2, 3, 4096)
    # full-sized inputs, so that even a launch would stay in bounds
    x = zeros_u32(4704, ctx.rgsw_words)
    yl = zeros_u32(3, ctx.rgsw_words)
    with pytest.raises(HW.HwError) as e:
        ctx.train_noalloc(sh, x, yl, 1, H, None)
    assert e.value.status == HW.HW_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert not host_u32(H).any()  # nothing was enqueued
