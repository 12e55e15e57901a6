"""Pins of the oracle's bootstrap through a key switch to a binary LWE key
(Ctx.pbs_ks_keygen, Ctx.key_switch, Ctx.pbs with a KsKey; the TFHE setting
of Sec. 2.5.3 keeps an LWE key in B^n beside the ring key), on a
128-coefficient ring with n = 64:

* the LWE key is binary; every key-switching row decrypts under it to
  s_k 2^(28 - 4j) plus an error within the error distribution's range, whose
  spread is that of 2^13 x the context's Gaussian plus a 13-bit uniform;
* a key-switched ciphertext decrypts under the LWE key, at modulus 2^32, to
  round(2^32 phase / Q) of the input within a bound set by the digits'
  rounding and the key's errors;
* the bootstrap returns V or -V by the half of the circle of the switched
  phase computed from the key-switched ciphertext;
* the activation and argmax circuits decrypt to their plaintext values
  with this key, also on a two-prime ring, where the key's RGSW use the
  coarser gadget of 2 digits of 15 bits per prime.
"""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as PL

N, P_MOD, NL = 128, 512, 64


@pytest.fixture(scope="module")
def setup():
    ctx = O.Ctx(N, 1, P_MOD)
    s = ctx.keygen(5)
    key = ctx.pbs_ks_keygen(s, 91, NL)
    return ctx, s, key


def signed32(x):
    x = int(x) % (1 << 32)
    return x - (1 << 32) if x >= 1 << 31 else x


def test_lwe_key_and_ksk_rows(setup):
    ctx, s, key = setup
    assert key.s1.dtype == np.uint8 and set(key.s1.tolist()) <= {0, 1} and 16 < int(key.s1.sum()) < 48
    assert key.ksk.shape == (N * O.KS_DIGITS, NL + 1) and len(key.bsk) == NL
    errs = []
    for r in range(0, N * O.KS_DIGITS, 1):
        k, j = divmod(r, O.KS_DIGITS)
        row = key.ksk[r].astype(np.int64)
        dot = int(np.dot(row[:NL], key.s1.astype(np.int64)))
        e = signed32(int(row[NL]) - dot - int(s[k]) * (1 << (28 - 4 * j)))
        assert abs(e) <= 41 * 8192 + 4096, (k, j, e)
        errs.append(e)
    errs = np.array(errs, np.float64)
    sd_want = np.sqrt((3.2 * 8192) ** 2 + 8192 ** 2 / 12)  # Gaussian part and the uniform fill
    assert abs(errs.mean()) < 4 * sd_want / np.sqrt(len(errs))
    assert 0.9 * sd_want < errs.std() < 1.1 * sd_want


def test_key_switch_keeps_the_phase(setup):
    ctx, s, key = setup
    rng = np.random.default_rng(7)
    sd = np.sqrt(N * O.KS_DIGITS * (16 ** 2 / 12) * ((3.2 * 8192) ** 2 + 8192 ** 2 / 12) + N * (2 / 3) * 128 ** 2 / 3)
    for m in [int(v) for v in rng.integers(0, P_MOD, 24)]:
        x = B.encrypt_short(ctx, s, m, N, P_MOD, rng)
        ks = ctx.key_switch(key, x).astype(np.int64)
        ph = signed32(int(ks[NL]) - int(np.dot(ks[:NL], key.s1.astype(np.int64))))
        want = (B.phase(ctx, s, x) * (1 << 32) + ctx.Q // 2) // ctx.Q
        err = signed32(ph - want)
        assert abs(err) < 6 * sd, (m, err)


def test_bootstrap_sign_of_the_switched_phase(setup):
    ctx, s, key = setup
    rng = np.random.default_rng(8)
    V = ctx.Q // 8
    sh = 32 - (N.bit_length())  # 2^32 -> 2N
    for m in [int(v) for v in rng.integers(0, P_MOD, 16)] + [0, 1, 255, 256, 511]:
        x = B.encrypt_short(ctx, s, m, N, P_MOD, rng)
        ks = ctx.key_switch(key, x)
        t = [((int(v) + (1 << (sh - 1))) >> sh) % (2 * N) for v in ks]
        sw = (t[NL] - sum(t[i] * int(key.s1[i]) for i in range(NL))) % (2 * N)
        ph = B.phase(ctx, s, ctx.pbs(key, x, 0, V))
        want = V if sw < N else ctx.Q - V
        assert min((ph - want) % ctx.Q, (want - ph) % ctx.Q) < ctx.Q // 64, (m, sw)


def test_circuits_with_the_key_switched_bootstrap(setup):
    ctx, s, key = setup
    cases = [("ge", m, T) for m, T in ((99, 100), (100, 100), (511, 511), (3, 1))] + \
            [("log", m, 0) for m in (0, 1, 6, 7, 255, 511)] + [("blog", m, 2) for m in (2, 3, 100)]

    def one(c):
        kind, m, T = c
        x = B.encrypt_short(ctx, s, m, N, P_MOD, np.random.default_rng(6000 + m + 7 * T))
        if kind == "ge":
            return B.decode(ctx, s, B.activate_ge(ctx, key, 0, x, T, 128), 128)
        return B.decode(ctx, s, B.activate_log(ctx, key, 0, x, 64, T if kind == "blog" else None), 64)

    got = [None] * len(cases)
    O._parallel(lambda i: got.__setitem__(i, one(cases[i])), range(len(cases)))
    for (kind, m, T), g in zip(cases, got):
        want = int(m >= T) if kind == "ge" else (int(PL.act_log(m)) if kind == "log" else int(PL.act_blog(m, T)))
        assert g == want, (kind, m, T)
    u = [B.encrypt_short(ctx, s, v, N, 128, np.random.default_rng(61 + v)) for v in (9, 40, 40)]
    assert B.decode(ctx, s, B.argmax(ctx, key, 0, u, 128), 4) == 1


def test_two_prime_ring_uses_the_coarser_gadget_and_stays_correct():
    """on a ring of two primes the key-switched key's RGSW use 2 digits of 15
    bits per prime; the threshold and log circuits still decrypt right"""
    ctx = O.Ctx(1024, 2, 512)
    s = ctx.keygen(5)
    key = ctx.pbs_ks_keygen(s, 91, 64)
    assert (key.gctx.digits, key.gctx.log_base) == (O.BSK_DIGITS, O.BSK_LOG_BASE) == (2, 15)
    assert key.bsk[0].shape == (2 * 2 * 2, 2, 2, 1024)
    cases = [("ge", 99, 100), ("ge", 100, 100), ("ge", 511, 511), ("log", 6, 0), ("log", 255, 0), ("log", 511, 0)]

    def one(c):
        kind, m, T = c
        x = B.encrypt_short(ctx, s, m, 1024, 512, np.random.default_rng(7 + m))
        if kind == "ge":
            return B.decode(ctx, s, B.activate_ge(ctx, key, 0, x, T, 128), 128)
        return B.decode(ctx, s, B.activate_log(ctx, key, 0, x, 64), 64)

    got = [None] * len(cases)
    O._parallel(lambda i: got.__setitem__(i, one(cases[i])), range(len(cases)))
    assert got == [int(m >= T) if k == "ge" else int(PL.act_log(m)) for k, m, T in cases]
