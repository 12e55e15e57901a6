"""GPU parity of the programmable bootstrapping and the OTF-act functions
(Activate as [m >= T], log and b-log; EncryptedArgMax; Sec. 2.5.3,
Sec. 3.5.2, Alg. 7).

Against the oracle, bit for bit: the bootstrapping key, single bootstraps
over the whole key (N = 1024), and the activation and argmax circuits at
p = 8 (their bootstraps in sequence take the oracle about a minute).  At the
Wisconsin-shaped parameter set (N = 2048, two primes, p = 512) every output
is checked by decryption: [m >= T] on both sides of the thresholds, log
and b-log (Sec. 2.4.2) on both sides of every power of two, the argmax
with ties to the lowest index, and OTF-act end to end (inference,
activation of every RAM score, class sums, EncryptedArgMax) against the
plaintext Alg. 2 with the bin activation."""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as P
from gpu_helpers import Pair, dev, host_u32, host_u64, zeros_u32, zeros_u64
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu


def hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


def setup(N, nq, p, key_seed=41, bsk_seed=42):
    HW = hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(key_seed, sk)
    s = orc.keygen(key_seed)
    bsk = None
    if bsk_seed is not None:
        bsk = zeros_u32(ctx.pbs_key_words(N))
        ctx.pbs_keygen(sk, bsk_seed, N, bsk)
    return HW, ctx, orc, sk, s, bsk


def lwes(orc, s, ms, p, seed):
    rng = np.random.default_rng(seed)
    return np.stack([B.encrypt_short(orc, s, int(m), orc.N, p, rng) for m in ms])


def test_key_and_single_bootstraps_bit_exact():
    HW, ctx, orc, sk, s, bsk = setup(1024, 1, 8)
    # key rows of the first coefficients against the oracle's RGSW
    exp = zeros_u32(6, ctx.rgsw_words)
    ctx.rgsw_export(bsk[: 6 * ctx.rgsw_words], 6, exp)
    ok = orc.pbs_keygen(s, 42, 3)
    assert np.array_equal(host_u32(exp).reshape(6, *ok[0].shape), np.stack(ok))
    bsk_o = orc.pbs_keygen(s, 42, 1024)
    X = lwes(orc, s, [0, 3, 5], 8, 1)
    out = zeros_u32(3, orc.lwe_words)
    V = orc.Q // 8
    ctx.pbs(bsk, 1024, dev(X), 3, V, out)
    want = [None] * 3
    O._parallel(lambda j: want.__setitem__(j, orc.pbs(bsk_o, X[j], 1024, V)), range(3))
    got = host_u32(out).reshape(3, 1, 1025)
    for j in range(3):
        assert np.array_equal(got[j], want[j]), j


@pytest.mark.parametrize("N,nq,p,n", [(2048, 2, 1024, 96), (4096, 3, 16384, 48)])
def test_single_bootstraps_bit_exact_larger_rings(N, nq, p, n):
    """the blind rotation at the two- and three-prime rings, over the first n
    key coefficients (LWE masks zero past them), bit for bit"""
    HW, ctx, orc, sk, s, _ = setup(N, nq, p, bsk_seed=None)
    bsk = zeros_u32(ctx.pbs_key_words(n))
    ctx.pbs_keygen(sk, 52, n, bsk)
    exp = zeros_u32(4, ctx.rgsw_words)
    ctx.rgsw_export(bsk[: 4 * ctx.rgsw_words], 4, exp)
    bsk_o = orc.pbs_keygen(s, 52, n)
    assert np.array_equal(host_u32(exp).reshape(4, *bsk_o[0].shape), np.stack(bsk_o[:4]))
    X = lwes_n(orc, s, [p // 8, 3 * p // 8, 5 * p // 8], p, 9, n)  # phases Q/8, 3Q/8, 5Q/8
    out = zeros_u32(3, orc.lwe_words)
    V = orc.Q // 8
    ctx.pbs(bsk, n, dev(X), 3, V, out)
    want = [None] * 3
    O._parallel(lambda j: want.__setitem__(j, orc.pbs(bsk_o, X[j], n, V)), range(3))
    got = host_u32(out).reshape(3, nq, N + 1)
    for j in range(3):
        assert np.array_equal(got[j], want[j]), j
    # V for a phase in [0, Q/2), -V above
    assert [B.phase(orc, s, w) < orc.Q // 2 for w in want] == [True, True, False]


def lwes_n(orc, s, ms, p, seed, n):
    rng = np.random.default_rng(seed)
    return np.stack([B.encrypt_short(orc, s, int(m), n, p, rng) for m in ms])


def test_activate_and_argmax_circuits_bit_exact():
    HW, ctx, orc, sk, s, bsk = setup(1024, 1, 8)
    bsk_o = orc.pbs_keygen(s, 42, 1024)
    X = lwes(orc, s, [2, 3], 8, 2)
    out = zeros_u32(2, orc.lwe_words)
    ctx.activate_ge(bsk, 1024, dev(X), 2, 3, 4, out)
    U = lwes(orc, s, [1, 2], 8, 3)  # scores of two classes at p_in = 8
    am = zeros_u32(1, orc.lwe_words)
    ctx.encrypted_argmax(bsk, 1024, dev(U), 1, 2, 3, am)
    want = [None] * 3
    jobs = [lambda: B.activate_ge(orc, bsk_o, 1024, X[0], 3, 16), lambda: B.activate_ge(orc, bsk_o, 1024, X[1], 3, 16),
            lambda: B.argmax(orc, bsk_o, 1024, [U[0], U[1]], 8)]
    O._parallel(lambda j: want.__setitem__(j, jobs[j]()), range(3))
    got = host_u32(out).reshape(2, 1, 1025)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    assert np.array_equal(host_u32(am).reshape(1, 1025), want[2])
    assert [B.decode(orc, s, got[j], 16) for j in range(2)] == [0, 1]
    assert B.decode(orc, s, want[2], 4) == 1


def test_log_activations_bit_exact():
    """log at m = 3 and at m = p - 1 (m + 1 wraps to 0), b-log with cap 1"""
    HW, ctx, orc, sk, s, bsk = setup(1024, 1, 8)
    bsk_o = orc.pbs_keygen(s, 42, 1024)
    X = lwes(orc, s, [3, 7, 5], 8, 6)
    out = zeros_u32(3, orc.lwe_words)
    ctx.activate(bsk, 1024, dev(X[:2]), 2, "log", 0, 4, out[:2])
    ctx.activate(bsk, 1024, dev(X[2:]), 1, "blog", 1, 4, out[2:])
    want = [None] * 3
    jobs = [lambda: B.activate_log(orc, bsk_o, 1024, X[0], 16), lambda: B.activate_log(orc, bsk_o, 1024, X[1], 16),
            lambda: B.activate_log(orc, bsk_o, 1024, X[2], 16, 1)]
    O._parallel(lambda j: want.__setitem__(j, jobs[j]()), range(3))
    got = host_u32(out).reshape(3, 1, 1025)
    for j in range(3):
        assert np.array_equal(got[j], want[j]), j
    assert [B.decode(orc, s, got[j], 16) for j in range(3)] == [2, 3, 1]


def decrypt_at(HW, N, nq, p, sk, lwe_dev, count):
    """GPU decryption with plaintext modulus p (same primes and key)"""
    c = HW.Context(N, nq, p)
    out = zeros_u64(count)
    c.decrypt_lwe(sk, lwe_dev, count, out)
    return host_u64(out).astype(np.int64)


def test_activate_and_argmax_by_decryption_wisconsin_params():
    HW, ctx, orc, sk, s, bsk = setup(2048, 2, 512)
    ms = np.array([0, 1, 2, 99, 100, 101, 255, 256, 257, 258, 300, 510, 511, 77, 400, 128])
    X = dev(lwes(orc, s, ms, 512, 4))
    for T in (1, 101, 257, 511):
        out = zeros_u32(len(ms), orc.lwe_words)
        ctx.activate_ge(bsk, 2048, X, len(ms), T, 7, out)
        assert np.array_equal(decrypt_at(HW, 2048, 2, 128, sk, out, len(ms)), (ms >= T).astype(np.int64)), T
    ml = np.array([0] + [v for i in range(1, 10) for v in ((1 << i) - 2, (1 << i) - 1) if v > 0])  # 2^i - 1 = m + 1 - 1
    XL = dev(lwes(orc, s, ml, 512, 8))
    for kind, cap in (("log", 0), ("blog", 2), ("blog", 4)):
        out = zeros_u32(len(ml), orc.lwe_words)
        ctx.activate(bsk, 2048, XL, len(ml), kind, cap, 7, out)
        want = P.act_log(ml) if kind == "log" else P.act_blog(ml, cap)
        assert np.array_equal(decrypt_at(HW, 2048, 2, 128, sk, out, len(ml)), want), (kind, cap)
    rng = np.random.default_rng(5)
    for l in (2, 3):
        S = rng.integers(0, 64, (12, l))
        S[0] = 7  # a tie of every class
        S[1, :2] = [40, 40]
        U = dev(np.stack([lwes(orc, s, row, 128, 10 + j) for j, row in enumerate(S)]))
        idx = zeros_u32(len(S), orc.lwe_words)
        ctx.encrypted_argmax(bsk, 2048, U, len(S), l, 7, idx)
        L = (l - 1).bit_length()
        got = decrypt_at(HW, 2048, 2, 1 << (L + 1), sk, idx, len(S))
        assert np.array_equal(got, np.argmax(S, axis=1)), l


def test_log_activations_by_decryption_mnist_modulus():
    """log and b-log (cap 4, the paper's MNIST activation) at p = 2^10"""
    HW, ctx, orc, sk, s, bsk = setup(2048, 2, 1024)
    ml = np.array([0, 1, 2, 3, 14, 15, 16, 30, 31, 62, 63, 126, 127, 510, 511, 1022, 1023])
    X = dev(lwes(orc, s, ml, 1024, 11))
    for kind, cap in (("log", 0), ("blog", 4)):
        out = zeros_u32(len(ml), orc.lwe_words)
        ctx.activate(bsk, 2048, X, len(ml), kind, cap, 6, out)
        want = P.act_log(ml) if kind == "log" else P.act_blog(ml, cap)
        assert np.array_equal(decrypt_at(HW, 2048, 2, 64, sk, out, len(ml)), want), kind


def test_otf_act_end_to_end_wisconsin_shape():
    """Inference scores of a Wisconsin-shaped model (s = 480, l = 2, a = 8,
    60 RAMs), every score activated with bin(thr) = [count > thr] by the
    bootstrapped circuit, summed per class, EncryptedArgMax: the decrypted
    class index equals Alg. 2 with the bin activation, computed in the clear."""
    from paper_2403_20190_amd import client as CL
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)
    pair = Pair(2048, 2, 512, 480, 2, 8, bits[:24], yw[:24], seed=12)
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    H = zeros_u32(pair.k0, pair.k1, 2, 2, 2048)
    pair.ctx.train(pair.shape, xr, yr, pair.n, H, None)
    tb = bits[100:104]
    xt = pair.encrypt_dev(tb, seed_x=66)
    nt, l, k0 = len(tb), 2, pair.k0
    sc = zeros_u32(nt, l, k0, pair.orc.lwe_words)
    pair.ctx.infer(pair.shape, H, xt, nt, sc, None)
    bsk = zeros_u32(pair.ctx.pbs_key_words(2048))
    pair.ctx.pbs_keygen(pair.sk, 43, 2048, bsk)
    thr = 1
    act = zeros_u32(nt * l * k0, pair.orc.lwe_words)
    pair.ctx.activate_ge(bsk, 2048, sc, nt * l * k0, thr + 1, 7, act)  # p_out = 128 > 2 * 60
    sums = zeros_u32(nt, l, pair.orc.lwe_words)
    pair.ctx.class_sums(act, nt, l, k0, sums)
    idx = zeros_u32(nt, pair.orc.lwe_words)
    pair.ctx.encrypted_argmax(bsk, 2048, sums, nt, l, 7, idx)
    HW = hw()
    got = decrypt_at(HW, 2048, 2, 4, pair.sk, idx, nt)
    W = P.train_integer(pair.X, pair.y, pair.l, pair.a, pair.pi)
    want = [P.predict(W, tb[i], pair.a, pair.pi, "bin", thr) for i in range(nt)]
    assert list(got) == want
    # the activated scores themselves
    cells = decrypt_at(HW, 2048, 2, 128, pair.sk, act, nt * l * k0).reshape(nt, l, k0)
    for i in range(nt):
        assert np.array_equal(cells[i], (P.ram_scores(W, tb[i], pair.a, pair.pi) > thr).astype(np.int64))
