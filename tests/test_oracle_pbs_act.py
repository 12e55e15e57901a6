"""Pins of the oracle's bootstrapped activation and EncryptedArgMax
(oracle.pbs; Sec. 2.5.3, Sec. 3.5.2) against plaintext definitions, on a
small ring (N = 128, one prime) so that every bootstrap blind-rotates over
the whole key, as it does at full size:

* the modulus switch stays within its rounding bound of the exact phase;
* a bootstrap with the constant test polynomial V returns V or -V by the
  half of the circle the switched phase lies in;
* the bit extraction returns the binary digits of the message, least
  significant first, across the carry boundaries of a 9-bit count;
* activate_ge decrypts to [m >= T] on both sides of every threshold tried;
* activate_log decrypts to floor(log2(m + 1)) and, with a cap, to
  min(floor(log2(m + 1)), cap) (Sec. 2.4.2) on both sides of every power of
  two, m = p - 1 (where m + 1 wraps to 0) included;
* argmax decrypts to the index of the largest score, ties to the lowest.
"""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as PL

N, P_MOD = 128, 512


@pytest.fixture(scope="module")
def setup():
    ctx = O.Ctx(N, 1, P_MOD)
    s = ctx.keygen(5)
    bsk = ctx.pbs_keygen(s, 77, N)
    return ctx, s, bsk


def run_all(fn, items):
    out = [None] * len(items)
    O._parallel(lambda i: out.__setitem__(i, fn(items[i])), range(len(items)))
    return out


def test_modswitch_within_rounding_bound(setup):
    ctx, s, _ = setup
    rng = np.random.default_rng(3)
    bound = (sum(abs(int(v)) for v in s) + 1) / 2
    for _ in range(40):
        m = int(rng.integers(0, P_MOD))
        x = B.encrypt_short(ctx, s, m, N, P_MOD, rng)
        ms = ctx.modswitch(x, N)
        assert ms.min() >= 0 and ms.max() < 2 * N
        sw = (int(ms[N]) - sum(int(ms[k]) * int(s[k]) for k in range(N))) % (2 * N)
        exact = B.phase(ctx, s, x) * 2 * N / ctx.Q
        d = (sw - exact + N) % (2 * N) - N
        assert abs(d) <= bound


def test_pbs_sign_of_the_switched_phase(setup):
    ctx, s, bsk = setup
    rng = np.random.default_rng(4)
    V = ctx.Q // 8
    ms_ = [int(v) for v in rng.integers(0, P_MOD, 12)] + [0, 1, 255, 256, 511]

    def one(m):
        x = B.encrypt_short(ctx, s, m, N, P_MOD, rng_for(m))
        ms = ctx.modswitch(x, N)
        sw = (int(ms[N]) - sum(int(ms[k]) * int(s[k]) for k in range(N))) % (2 * N)
        ph = B.phase(ctx, s, ctx.pbs(bsk, x, N, V))
        return sw, ph

    def rng_for(m):
        return np.random.default_rng(1000 + m)

    for sw, ph in run_all(one, ms_):
        want = V if sw < N else ctx.Q - V
        dist = min((ph - want) % ctx.Q, (want - ph) % ctx.Q)
        assert dist < ctx.Q // 64, (sw, ph)


def test_bits_are_the_binary_digits(setup):
    ctx, s, bsk = setup
    ms_ = list(range(0, 8)) + [127, 128, 129, 255, 256, 257, 383, 510, 511, 341]

    def one(m):
        x = B.encrypt_short(ctx, s, m, N, P_MOD, np.random.default_rng(2000 + m))
        return [B.decode(ctx, s, e, P_MOD) for e in B.bits(ctx, bsk, N, x, P_MOD)]

    for m, got in zip(ms_, run_all(one, ms_)):
        assert got == [(m >> k) & 1 for k in range(9)], m


def test_activate_ge_on_both_sides_of_the_threshold(setup):
    ctx, s, bsk = setup
    cases = []
    for T in (1, 2, 100, 256, 257, 511, 512):
        for m in (T - 1, T, T + 1, 0, 511):
            if 0 <= m < P_MOD:
                cases.append((m, T))
    cases = sorted(set(cases))

    def one(mT):
        m, T = mT
        x = B.encrypt_short(ctx, s, m, N, P_MOD, np.random.default_rng(3000 + 600 * T + m))
        return B.decode(ctx, s, B.activate_ge(ctx, bsk, N, x, T, 128), 128)

    for (m, T), got in zip(cases, run_all(one, cases)):
        assert got == int(m >= T), (m, T)


def test_argmax_index_with_ties_to_the_lowest(setup):
    ctx, s, bsk = setup
    p_in = 128
    cases = [(3, 5), (5, 3), (4, 4), (0, 0), (60, 59), (0, 63), (2, 7, 7), (9, 1, 9), (0, 0, 1), (40, 41, 39)]

    def one(scores):
        rng = np.random.default_rng(4000 + sum(scores) * 7 + len(scores))
        u = [B.encrypt_short(ctx, s, v, N, p_in, rng) for v in scores]
        L = (len(scores) - 1).bit_length()
        return B.decode(ctx, s, B.argmax(ctx, bsk, N, u, p_in), 1 << (L + 1))

    for sc, got in zip(cases, run_all(one, cases)):
        assert got == int(np.argmax(sc)), sc


def test_log_and_bounded_log_activations(setup):
    ctx, s, bsk = setup
    ms = sorted({0, 1, 2, 3} | {v for i in range(3, 10) for v in ((1 << i) - 2, (1 << i) - 1, (1 << i)) if v < P_MOD})
    cases = [(m, cap) for m in ms for cap in (None, 1, 4)]

    def one(mc):
        m, cap = mc
        x = B.encrypt_short(ctx, s, m, N, P_MOD, np.random.default_rng(5000 + m))
        return B.decode(ctx, s, B.activate_log(ctx, bsk, N, x, 64, cap), 64)

    for (m, cap), got in zip(cases, run_all(one, cases)):
        want = int(PL.act_log(m)) if cap is None else int(PL.act_blog(m, cap))
        assert got == want, (m, cap)
