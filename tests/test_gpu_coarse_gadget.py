"""GPU parity of the RGSW gadget of 2 balanced digits of 15 bits per prime
(hw_params log_base = 15, digits = 2, on rings of two or more primes; the
digit size of the paper's HE1 TFHE parameter set, Sec. 4), bit for bit
against the oracle's context of the same gadget:

* contexts refuse that gadget on one prime, and every other gadget;
* RGSW encryption (both row schedules) and the external product at
  (2048, 2), (4096, 3) and (2048, 3);
* training (every schedule: grid orders, tree levels fused or staged; the
  class counter) and inference on the MNIST parameter set (N = 2048, two
  primes, p = 2^10, 10 classes, 12-bit tuples: an encrypted tree level and
  a ragged last tuple), every RAM; at N = 4096 with three primes on the
  ragged RAM; batched training and batched inference equal the per-call
  results;
* a ring-key bootstrap with a key of that gadget;
* PackingKeySwitching keeps its own gadget of 5 digits of 6 bits on such a
  context (key rows and a packed RLWE);
* FM-act on such a context with a key-switched bootstrapping key."""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as P
from gpu_helpers import Pair, dev, host_u32, host_u64, zeros_u32, zeros_u64
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu

G = (15, 2)


def _hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


def ctx_pair(N, nq, p):
    HW = _hw()
    return HW.Context(N, nq, p, log_base=15, digits=2), O.Ctx(N, nq, p, log_base=15, digits=2)


def test_contexts_accept_only_the_built_gadgets():
    HW = _hw()
    c = HW.Context(2048, 2, 1024, log_base=15, digits=2)
    assert c.rgsw_words == 2 * 2 * 2 * c.rlwe_words
    assert c.tune_get("encrypt_rgsw")[2] == 2  # 1 or 2 rows per workgroup: 5 divides no 4 nq
    for N, nq, lb, dg in [(1024, 1, 15, 2), (2048, 2, 15, 3), (2048, 2, 10, 3), (2048, 2, 6, 2), (4096, 3, 23, 1)]:
        with pytest.raises(HW.HwError):
            HW.Context(N, nq, 64, log_base=lb, digits=dg)


@pytest.mark.parametrize("N,nq,p", [(2048, 2, 1024), (4096, 3, 16384), (2048, 3, 1024)])
def test_rgsw_and_external_product_bit_exact(N, nq, p):
    ctx, orc = ctx_pair(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(11, sk)
    sk_o = orc.keygen(11)
    bits = np.array([1, 0, 1], np.uint8)
    want_rg = [orc.enc_rgsw(sk_o, int(b), 21, 5 + k) for k, b in enumerate(bits)]
    assert want_rg[0].shape == (2 * 2 * nq, 2, nq, N)
    rg = None
    for v in range(2):
        ctx.tune_set("encrypt_rgsw", v)
        r = zeros_u32(len(bits), ctx.rgsw_words)
        ctx.encrypt_rgsw_bits(sk, dev(bits), 21, 5, r)
        exp = zeros_u32(len(bits), ctx.rgsw_words)
        ctx.rgsw_export(r, len(bits), exp)
        got = host_u32(exp).reshape(len(bits), *want_rg[0].shape)
        for k in range(len(bits)):
            assert np.array_equal(got[k], want_rg[k]), (v, k)
        rg = r
    rng = np.random.default_rng(nq * N + 1)
    rin = np.stack([np.stack([np.stack([rng.integers(0, q, N) for q in orc.primes]) for _ in range(2)])
                    for _ in bits]).astype(np.uint32)
    rout = zeros_u32(len(bits), 2, nq, N)
    ctx.external_product(rg, dev(rin), len(bits), rout)
    got = host_u32(rout)
    want = [None] * len(bits)
    O._parallel(lambda k: want.__setitem__(k, orc.extprod(want_rg[k], rin[k])), range(len(bits)))
    for k in range(len(bits)):
        assert np.array_equal(got[k], want[k]), k


def mnist_pair(n=3, seed=13):
    X, y = synth.prototype_bits(seed, n, 30, 10, flip=0.2)
    return Pair(2048, 2, 1024, 30, 10, 12, X, y, seed=seed, gadget=G)


def test_training_and_inference_mnist_params_bit_exact():
    """three 12-bit tuples over 30 bits (the last one 6 bits), 10 classes:
    nb = 16 > log2 N = 11, so z = 5 > L = 4 (an encrypted tree level)"""
    pair = mnist_pair()
    ctx = pair.ctx
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    nv = ctx.tune_get("train")[2]
    Hs, Cs = [], []
    for v in range(nv):
        ctx.tune_set("train", v)
        H = zeros_u32(pair.k0, pair.k1, 2, 2, 2048)
        cnt = zeros_u32(2, 2, 2048)
        ctx.train(pair.shape, xr, yr, pair.n, H, cnt)
        Hs.append(host_u32(H))
        Cs.append(host_u32(cnt))
    for v in range(1, nv):
        assert np.array_equal(Hs[v], Hs[0]) and np.array_equal(Cs[v], Cs[0]), v
    Ho = pair.oracle_train(range(pair.k0))
    assert np.array_equal(Hs[0], Ho)
    cnt_o = np.zeros((2, 2, 2048), np.uint32)
    pair.orc.class_count(pair.l, pair.yo, pair.n, cnt_o)
    assert np.array_equal(Cs[0], cnt_o)
    W = P.train_integer(pair.X, pair.y, pair.l, pair.a, pair.pi)
    dec = zeros_u64(pair.k0 * pair.k1, 2048)
    ctx.decrypt_rlwe(pair.sk, dev(Hs[0]), pair.k0 * pair.k1, dec)
    assert np.array_equal(host_u64(dec).reshape(pair.k0, pair.k1, 2048).astype(np.int64),
                          P.expected_model_cells(W, pair.s, pair.l, pair.a, 2048))
    # batched training: the same model
    Hb = zeros_u32(pair.k0, pair.k1, 2, 2, 2048)
    Cb = zeros_u32(2, 2, 2048)
    ctx.batch_train([(pair.shape, xr, yr, pair.n, Hb, Cb)])
    assert np.array_equal(host_u32(Hb), Hs[0]) and np.array_equal(host_u32(Cb), Cs[0])
    # inference of two test samples, every (label, RAM) against the oracle
    Xt, _ = synth.prototype_bits(99, 2, 30, 10, flip=0.3)
    nt = len(Xt)
    xt = pair.encrypt_dev(Xt, seed_x=71)
    Hd = dev(Hs[0])
    lw = pair.orc.lwe_words
    scores = []
    for v in range(ctx.tune_get("infer")[2]):
        ctx.tune_set("infer", v)
        sc = zeros_u32(nt, pair.l, pair.k0, lw)
        ctx.infer(pair.shape, Hd, xt, nt, sc, None)
        scores.append(host_u32(sc))
    for v in range(1, len(scores)):
        assert np.array_equal(scores[v], scores[0]), v
    jobs = [(i, c, j) for i in range(nt) for c in range(pair.l) for j in range(pair.k0)]
    want = {}

    def one(job):
        i, c, j = job
        want[job] = pair.orc.infer_one(pair.s, pair.l, pair.a, pair.pi, Ho,
                                       lambda k: pair.xo(i, k, Xt, 71, "test"), j, c)

    O._parallel(one, jobs)
    got = scores[0].reshape(nt, pair.l, pair.k0, 2, 2049)
    for job in jobs:
        assert np.array_equal(got[job], want[job]), job
    # batched inference: the same scores
    HW = _hw()
    sb = zeros_u32(nt, pair.l, pair.k0, lw)
    HW.batch_run([ctx], [dict(kind="infer", shape=pair.shape, x=xt, n=nt, model=Hd, scores=sb)])
    assert np.array_equal(host_u32(sb), scores[0])
    dl = zeros_u64(nt * pair.l * pair.k0)
    ctx.decrypt_lwe(pair.sk, dev(scores[0]), nt * pair.l * pair.k0, dl)
    cells = host_u64(dl).reshape(nt, pair.l, pair.k0).astype(np.int64)
    for i in range(nt):
        assert np.array_equal(cells[i], P.ram_scores(W, Xt[i], pair.a, pair.pi))


def test_training_n4096_three_primes_ragged_ram_bit_exact():
    X, y = synth.prototype_bits(4, 2, 30, 5, flip=0.2)
    pair = Pair(4096, 3, 16384, 30, 5, 12, X, y, seed=4, gadget=G)
    H = zeros_u32(pair.k0, pair.k1, 2, 3, 4096)
    pair.ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    rams = [pair.k0 - 1]
    Ho = pair.oracle_train(rams)
    assert np.array_equal(host_u32(H)[rams[0]], Ho[rams[0]])


def test_ring_key_bootstrap_bit_exact():
    N, nq, p, n = 2048, 2, 1024, 24
    ctx, orc = ctx_pair(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(17, sk)
    sk_o = orc.keygen(17)
    bsk = zeros_u32(ctx.pbs_key_words(n))
    ctx.pbs_keygen(sk, 33, n, bsk)
    bsk_o = orc.pbs_keygen(sk_o, 33, n)
    rng = np.random.default_rng(5)
    ms = [p // 8, 3 * p // 8, 5 * p // 8, 7 * p // 8]
    X = np.stack([B.encrypt_short(orc, sk_o, m, n, p, rng) for m in ms])
    out = zeros_u32(len(ms), orc.lwe_words)
    V = orc.Q // 8
    ctx.pbs(bsk, n, dev(X), len(ms), V, out)
    want = [None] * len(ms)
    O._parallel(lambda j: want.__setitem__(j, orc.pbs(bsk_o, X[j], n, V)), range(len(ms)))
    got = host_u32(out).reshape(len(ms), nq, N + 1)
    for j in range(len(ms)):
        assert np.array_equal(got[j], want[j]), j
    assert [B.phase(orc, sk_o, w) < orc.Q // 2 for w in want] == [True, True, False, False]


def test_packing_keeps_its_own_gadget():
    N, nq, p = 1024, 2, 64
    ctx, orc = ctx_pair(N, nq, p)
    assert orc.pks_ctx().digits == 5 and orc.pks_ctx().log_base == 6
    sk = zeros_u32(N)
    ctx.keygen(23, sk)
    sk_o = orc.keygen(23)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(sk, 98, key)
    K_o = orc.pks_keygen(sk_o, 98)
    exp = zeros_u32(ctx.pks_key_words)
    ctx.pks_key_export(key, exp)
    assert np.array_equal(host_u32(exp).reshape(K_o.shape), K_o)
    k = 7
    rng = np.random.default_rng(7)
    lwes = np.stack([np.stack([rng.integers(0, q, N + 1) for q in orc.primes]) for _ in range(k)]).astype(np.uint32)
    out = zeros_u32(1, 2, nq, N)
    ctx.pack_lwe(key, dev(lwes[None]), k, 1, out)
    assert np.array_equal(host_u32(out)[0], orc.pack_lwe(K_o, lwes))


def test_fm_act_two_primes_bit_exact():
    """FM-act on a context of that gadget: a key-switched bootstrapping key
    (its RGSW in the context's gadget), PackingKeySwitching in its own
    5 x 6 gadget, bit for bit against the oracle (2 RAMs of 4 cells, p = 8,
    a 32-coefficient LWE key), and every activated cell decrypting to
    [cell >= T]"""
    N, T, n = 1024, 2, 32
    rng = np.random.default_rng(31)
    X = rng.integers(0, 2, (6, 2)).astype(np.uint8)
    y = np.array([0, 1, 0, 0, 1, 1])
    pair = Pair(N, 2, 8, 2, 2, 1, X, y, seed=19, gadget=G)
    ctx, orc = pair.ctx, pair.orc
    H = zeros_u32(pair.k0, pair.k1, 2, 2, N)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    Ho = pair.oracle_train(range(pair.k0))
    assert np.array_equal(host_u32(H), Ho)
    key = ctx.pbs_ks_keygen(pair.sk, 43, n)
    ko = orc.pbs_ks_keygen(pair.sk_o, 43, n)
    assert ko.gctx is orc  # the context's own gadget
    pks = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 9, pks)
    K_o = orc.pks_keygen(pair.sk_o, 9)
    out = zeros_u32(*H.shape)
    ctx.fm_act(pair.shape, key, 0, pks, H, "ge", T, 3, out)
    want = B.fm_act(orc, ko, n, K_o, Ho, B.fm_cells(N, 2, 1), T, 8)
    got = host_u32(out)
    assert np.array_equal(got, want)
    W = P.train_integer(pair.X, pair.y, 2, 1, pair.pi)
    cells = P.expected_model_cells(W, 2, 2, 1, N)
    dec = [[B.decode(orc, pair.sk_o, orc.extract_lwe(want[j, r], k), 8) for k in range(4)]
           for j in range(pair.k0) for r in range(pair.k1)]
    assert dec == [[int(v >= T) for v in cells[j, r, :4]] for j in range(pair.k0) for r in range(pair.k1)]
