"""Schedule variants of the tuned kernels compute the same bits (each forced
in turn, compared with the oracle or with variant 0 on ragged sizes), and
online tuning settles on a variant without changing any result."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import Pair, dev, host_u32, zeros_u32
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu


def _hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2), (4096, 3)])
def test_ntt_variants_identical(N, nq):
    HW = _hw()
    ctx = HW.Context(N, nq, 64)
    rng = np.random.default_rng(3)
    count = 37  # not a multiple of any tile
    a = np.stack([np.stack([rng.integers(0, q, N) for q in ctx.primes]) for _ in range(count)]).astype(np.uint32)
    outs = []
    for v in range(4):
        ctx.tune_set("ntt", v)
        ctx.tune_set("ntt_inverse", 3 - v)
        A = dev(a)
        ctx.ntt(A, count, False)
        outs.append(host_u32(A))
        ctx.ntt(A, count, True)
        assert np.array_equal(host_u32(A), a), v
    for v in range(1, 4):
        assert np.array_equal(outs[v], outs[0]), v


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384)])
def test_encrypt_rgsw_variants_match_oracle(N, nq, p):
    HW = _hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(9, sk)
    sk_o = orc.keygen(9)
    bits = np.array([1, 0, 1], np.uint8)
    ref = None
    for v in range(3):
        ctx.tune_set("encrypt_rgsw", v)
        rg = zeros_u32(len(bits), ctx.rgsw_words)
        ctx.encrypt_rgsw_bits(sk, dev(bits), 41, 7, rg)
        got = host_u32(rg)
        if ref is None:
            ref = got
            exp = zeros_u32(len(bits), ctx.rgsw_words)
            ctx.rgsw_export(rg, len(bits), exp)
            canon = host_u32(exp).reshape(len(bits), 2 * 5 * nq, 2, nq, N)
            for k, b in enumerate(bits):
                assert np.array_equal(canon[k], orc.enc_rgsw(sk_o, int(b), 41, 7 + k)), k
        assert np.array_equal(got, ref), v


@pytest.mark.parametrize("N,nq,s,l,a", [(1024, 1, 23, 3, 11), (4096, 3, 30, 5, 12)])
def test_train_and_infer_variants_identical(N, nq, s, l, a):
    """An encrypted tree level (z > L), a ragged last tuple and the class
    counter, every variant of training (grid order, tree levels in the
    chain's workgroup or staged one launch per level), batched training and
    inference forced in turn (N = 4096 adds the occupancy-4 builds)."""
    X, y = synth.prototype_bits(5, 4 if N == 1024 else 2, s, l, flip=0.2)
    pair = Pair(N, nq, 64, s, l, a, X, y, seed=5)
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    ctx = pair.ctx
    nv = ctx.tune_get("train")[2]
    assert nv == (8 if N == 4096 else 4)
    Hs, Cs, Ss = [], [], []
    for v in range(nv):
        ctx.tune_set("train", v)
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C = zeros_u32(2, pair.nq, pair.N)
        ctx.train(pair.shape, xr, yr, pair.n, H, C)
        Hs.append(host_u32(H))
        Cs.append(host_u32(C))
    for v in range(1, nv):
        assert np.array_equal(Hs[0], Hs[v]) and np.array_equal(Cs[0], Cs[v]), v
    rams = list(range(pair.k0)) if N == 1024 else [pair.k0 - 1]  # N = 4096: the ragged RAM
    Ho = pair.oracle_train(rams)
    for j in rams:
        assert np.array_equal(Hs[0][j], Ho[j]), j
    for v in range(ctx.tune_get("train_batch")[2]):
        ctx.tune_set("train_batch", v)
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C = zeros_u32(2, pair.nq, pair.N)
        ctx.batch_train([(pair.shape, xr, yr, pair.n, H, C)])
        assert np.array_equal(host_u32(H), Hs[0]) and np.array_equal(host_u32(C), Cs[0]), v
    Hd = dev(Hs[0])
    nv = ctx.tune_get("infer")[2]
    assert nv == (4 if N == 4096 else 2)
    for v in range(nv):
        ctx.tune_set("infer", v)
        sc = zeros_u32(pair.n, pair.l, pair.k0, pair.nq * (pair.N + 1))
        cs = zeros_u32(pair.n, pair.l, pair.nq * (pair.N + 1))
        ctx.infer(pair.shape, Hd, xr, pair.n, sc, cs)
        Ss.append((host_u32(sc), host_u32(cs)))
    for v in range(1, nv):
        assert np.array_equal(Ss[0][0], Ss[v][0]) and np.array_equal(Ss[0][1], Ss[v][1]), v


def test_online_tuning_settles_and_keeps_results():
    import torch
    HW = _hw()
    ctx = HW.Context(2048, 2, 64)
    v, t, n = ctx.tune_get("ntt")
    assert (v, t, n) == (-1, 0, 4)
    rng = np.random.default_rng(4)
    count = 8192  # x 2 primes: large enough to be timed
    a = rng.integers(0, min(ctx.primes), (count, 2, 2048)).astype(np.uint32)
    A = dev(a)
    ref = None
    for it in range(12):
        ctx.ntt(A, count, False)
        torch.cuda.synchronize()
        if ref is None:
            ref = host_u32(A)
        else:
            assert np.array_equal(host_u32(A), ref), it
        ctx.ntt(A, count, True)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(A), a)
    v, t, n = ctx.tune_get("ntt")
    assert 0 <= v < 4 and t >= 2 * 4
    assert HW.tune_variant_name("ntt", v) is not None
    assert set(ctx.schedule()) == set(HW.TUNED_KERNELS)
    ctx.tune_set("ntt", -1)  # forget and tune again
    assert ctx.tune_get("ntt")[:2] == (-1, 0)
    with pytest.raises(HW.HwError):
        ctx.tune_set("ntt", 4)
    with pytest.raises(HW.HwError):
        ctx.tune_set("nope", 0)
