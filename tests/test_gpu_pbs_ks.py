"""GPU parity of the bootstrap through a key switch to a binary LWE key
(hw_pbs_ks_keygen, hw_boot_key with a key-switching key; the TFHE setting
of Sec. 2.5.3 keeps an LWE key in B^n beside the ring key).

* Against the oracle, bit for bit: the LWE key, the key's RGSW rows (on
  rings of two and three primes in the coarser gadget of 2 digits of 15 bits
  per prime) and every key-switching word (rebuilt from the contraction
  layout's signed bytes), and bootstraps of full-mask ciphertexts at the one-, two- and
  three-prime rings (the key switch's digits, its int8 matrix-core
  contraction, the switch to 2N and the one-CMUX-per-bit blind rotation all
  feed those bits).
* By decryption at the Wisconsin-shaped parameters with an LWE key of 1024
  coefficients: [m >= T], log and EncryptedArgMax, and FM-act of a
  Wisconsin-shaped model through inference and EncryptedArgMax."""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as P
from gpu_helpers import Pair, dev, host_u32, host_u64, zeros_u32, zeros_u64

pytestmark = pytest.mark.gpu


def hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


def setup(N, nq, p, n, key_seed=41, ks_seed=71):
    HW = hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(key_seed, sk)
    s = orc.keygen(key_seed)
    key = ctx.pbs_ks_keygen(sk, ks_seed, n)
    return HW, ctx, orc, sk, s, key


def ksk_words(key, N):
    """the 32-bit key-switching words [N 6][n + 1] from the signed-byte layout"""
    n = key.n
    kd = N * O.KS_DIGITS
    raw = key.ksk.cpu().numpy().view(np.int8).reshape(-1, kd)[: 4 * (n + 1)].astype(np.int64)
    w = np.zeros((n + 1, kd), np.int64)
    for l in range(4):
        w += raw[l * (n + 1):(l + 1) * (n + 1)] << (8 * l)
    return (w % (1 << 32)).astype(np.uint32).T


def test_key_bit_exact():
    N, n = 1024, 64
    HW, ctx, orc, sk, s, key = setup(N, 1, 8, n)
    ko = orc.pbs_ks_keygen(s, 71, n)
    assert np.array_equal(key.lwe_key.cpu().numpy(), ko.s1)
    exp = zeros_u32(4, ctx.rgsw_words)
    ctx.rgsw_export(key.bsk[: 4 * ctx.rgsw_words], 4, exp)
    assert np.array_equal(host_u32(exp).reshape(4, *ko.bsk[0].shape), np.stack(ko.bsk[:4]))
    assert np.array_equal(ksk_words(key, N), ko.ksk)
    raw = key.ksk.cpu().numpy().view(np.int8).reshape(-1, N * O.KS_DIGITS)
    assert not raw[4 * (n + 1):].any()  # padding rows of the contraction


@pytest.mark.parametrize("N,nq,p,n", [(1024, 1, 8, 64), (2048, 2, 1024, 48), (4096, 3, 16384, 24)])
def test_bootstraps_bit_exact(N, nq, p, n):
    HW, ctx, orc, sk, s, key = setup(N, nq, p, n)
    ko = orc.pbs_ks_keygen(s, 71, n)
    if nq >= 2:  # RGSW of 2 digits of 15 bits per prime: 5 of them fill 2 of the 5-digit layout
        assert ko.bsk[0].shape == (2 * 2 * nq, 2, nq, N)
        exp = zeros_u32(2, ctx.rgsw_words)
        ctx.rgsw_export(key.bsk[: 2 * ctx.rgsw_words], 2, exp)
        assert np.array_equal(host_u32(exp).reshape(5, *ko.bsk[0].shape), np.stack(ko.bsk[:5]))
    rng = np.random.default_rng(N + n)
    ms = [p // 8, 3 * p // 8, 5 * p // 8, 7 * p // 8, int(rng.integers(0, p))]
    X = np.stack([B.encrypt_short(orc, s, m, N, p, rng) for m in ms])  # full masks
    out = zeros_u32(len(ms), orc.lwe_words)
    V = orc.Q // 8
    ctx.pbs(key, 0, dev(X), len(ms), V, out)
    want = [None] * len(ms)
    O._parallel(lambda j: want.__setitem__(j, orc.pbs(ko, X[j], 0, V)), range(len(ms)))
    got = host_u32(out).reshape(len(ms), nq, N + 1)
    for j in range(len(ms)):
        assert np.array_equal(got[j], want[j]), j
    assert [B.phase(orc, s, w) < orc.Q // 2 for w in want[:4]] == [True, True, False, False]


def decrypt_at(HW, N, nq, p, sk, lwe_dev, count):
    c = HW.Context(N, nq, p)
    out = zeros_u64(count)
    c.decrypt_lwe(sk, lwe_dev, count, out)
    return host_u64(out).astype(np.int64)


def test_circuits_by_decryption_wisconsin_params():
    HW, ctx, orc, sk, s, key = setup(2048, 2, 512, 1024)
    ms = np.array([0, 1, 2, 6, 7, 99, 100, 101, 255, 256, 257, 510, 511])
    rng = np.random.default_rng(12)
    X = dev(np.stack([B.encrypt_short(orc, s, int(m), 2048, 512, rng) for m in ms]))
    out = zeros_u32(len(ms), orc.lwe_words)
    ctx.activate(key, 0, X, len(ms), "ge", 100, 7, out)
    assert np.array_equal(decrypt_at(HW, 2048, 2, 128, sk, out, len(ms)), (ms >= 100).astype(np.int64))
    ctx.activate(key, 0, X, len(ms), "log", 0, 7, out)
    assert np.array_equal(decrypt_at(HW, 2048, 2, 128, sk, out, len(ms)), P.act_log(ms))
    S = np.array([[3, 9], [9, 3], [5, 5], [0, 63], [40, 39]])
    U = dev(np.stack([np.stack([B.encrypt_short(orc, s, int(v), 2048, 128, rng) for v in row]) for row in S]))
    idx = zeros_u32(len(S), orc.lwe_words)
    ctx.encrypted_argmax(key, 0, U, len(S), 2, 7, idx)
    assert np.array_equal(decrypt_at(HW, 2048, 2, 4, sk, idx, len(S)), np.argmax(S, axis=1))


def test_fm_act_with_the_key_switched_bootstrap():
    """log FM-act of a Wisconsin-shaped model (2 RAMs of 512 cells) with the
    key-switched bootstrap: every coefficient decrypts to log of its cell,
    and inference on it gives Alg. 2 with log"""
    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import synth
    HW = hw()
    N, s_, a, l, lp = 2048, 16, 8, 2, 6
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)[:, :s_]
    pair = Pair(N, 2, 512, s_, l, a, bits[:60], yw[:60], seed=23)
    ctx = pair.ctx
    H = zeros_u32(pair.k0, pair.k1, 2, 2, N)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    key = ctx.pbs_ks_keygen(pair.sk, 73, 1024)
    pks = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 45, pks)
    act = zeros_u32(*H.shape)
    ctx.fm_act(pair.shape, key, 0, pks, H, "log", 0, lp, act)
    W = P.train_integer(pair.X, pair.y, l, a, pair.pi)
    cells = P.expected_model_cells(W, s_, l, a, N)
    cp = HW.Context(N, 2, 1 << lp)
    dec = zeros_u64(pair.k0 * pair.k1, N)
    cp.decrypt_rlwe(pair.sk, act, pair.k0 * pair.k1, dec)
    assert np.array_equal(host_u64(dec).reshape(cells.shape).astype(np.int64), P.act_log(cells))
    tb = bits[[70, 71, 72, 73, 74, 112, 175, 192]]
    nt = len(tb)
    xt = pair.encrypt_dev(tb, seed_x=67)
    sc = zeros_u32(nt, l, pair.k0, ctx.lwe_words)
    ctx.infer(pair.shape, act, xt, nt, sc, None)
    sums = zeros_u32(nt, l, ctx.lwe_words)
    ctx.class_sums(sc, nt, l, pair.k0, sums)
    idx = zeros_u32(nt, ctx.lwe_words)
    ctx.encrypted_argmax(key, 0, sums, nt, l, lp, idx)
    want = [P.predict(W, tb[i], a, pair.pi, "log") for i in range(nt)]
    assert sorted(set(want)) == [0, 1]
    assert list(decrypt_at(HW, N, 2, 4, pair.sk, idx, nt)) == want
