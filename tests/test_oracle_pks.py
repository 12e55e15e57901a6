"""Pins of the oracle's PackingKeySwitching (Sec. 2.5.1 building block; the
PD-act return value of Alg. 7): with a noiseless key the packed RLWE's phase
is exactly sum_i phase_i X^i, computed here independently from the LWE
definition; with a real key the packed RLWE decrypts to the LWE messages;
key rows decrypt to s_j G_r."""
import numpy as np
import pytest

import oracle as O


def _lwe_phases(c, s, lwes):
    """phase_i = b_i - sum_j a_ij s_j mod q_g for every prime g (Python ints)"""
    k = lwes.shape[0]
    out = np.zeros((c.nq, k), np.int64)
    for g, q in enumerate(c.primes):
        for i in range(k):
            a = [int(x) for x in lwes[i, g, :c.N]]
            acc = int(lwes[i, g, c.N])
            for j in range(c.N):
                acc -= a[j] * int(s[j])
            out[g, i] = acc % q
    return out


@pytest.mark.parametrize("N,nq", [(64, 2), (32, 3), (1024, 1)])
def test_noiseless_key_packs_phases_exactly(N, nq):
    c = O.Ctx(N, nq, 16)
    s = c.keygen(3)
    rng = np.random.default_rng(N + nq)
    k = N // 2 + 3
    lwes = np.zeros((k, nq, N + 1), np.uint32)
    for g, q in enumerate(c.primes):
        lwes[:, g, :] = rng.integers(0, q, (k, N + 1))
    K = np.zeros((N, c.D, 2, nq, N), np.uint32)  # (0, s_j G_r): no mask, no error
    for j in range(N):
        for r in range(c.D):
            g, t = divmod(r, 5)
            q = c.primes[g]
            K[j, r, 1, g, 0] = (int(s[j]) * pow(64, t, q)) % q
    out = c.pack_lwe(K, lwes)
    assert not out[0].any()
    want = _lwe_phases(c, s, lwes)
    for g in range(nq):
        assert np.array_equal(out[1, g, :k].astype(np.int64), want[g]), g
        assert not out[1, g, k:].any()


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (64, 2, 256)])
def test_packing_decrypts_to_lwe_messages(N, nq, p):
    c = O.Ctx(N, nq, p)
    s = c.keygen(4)
    K = c.pks_keygen(s, 77)
    rng = np.random.default_rng(p)
    k = 24
    msgs = rng.integers(0, p, k)
    lwes = []
    for i, m in enumerate(msgs):
        mu = rng.integers(0, p, N).astype(np.uint64)
        mu[0] = m
        lwes.append(c.extract_lwe0(c.enc_rlwe(s, mu, 5, i)))
    lwes = np.stack(lwes)
    assert [c.dec_lwe(s, x) for x in lwes] == list(msgs)
    out = c.pack_lwe(K, lwes)
    dec = c.dec_rlwe(s, out)
    assert np.array_equal(dec[:k], msgs.astype(np.uint64)) and not dec[k:].any()


def test_key_rows_decrypt_to_gadget_times_secret():
    c = O.Ctx(64, 2, 16)
    s = c.keygen(6)
    K = c.pks_keygen(s, 9)
    for j in (0, 5, 63):
        for r in (0, 4, 7):
            g, t = divmod(r, 5)
            for i, q in enumerate(c.primes):
                a = K[j, r, 0, i].astype(np.uint64)
                sl = np.array([(int(x) + q) % q for x in s], np.uint64)
                ph = (K[j, r, 1, i].astype(np.int64) - c.negmul(i, a, sl).astype(np.int64)) % q
                ph = np.where(ph > q // 2, ph - q, ph)
                want = np.zeros(64, np.int64)
                if i == g:
                    want[0] = int(s[j]) * pow(64, t, q)
                    want[0] = want[0] - q if want[0] > q // 2 else want[0]
                assert np.abs(ph - want).max() <= 41, (j, r, i)


def test_packing_on_a_two_digit_context_keeps_its_own_gadget():
    """on a context whose RGSW use 2 digits of 15 bits, the key has the 5 nq
    rows of base-64 digits per coordinate and packing still decrypts to
    the LWE messages; RLWE and LWE ciphertexts are the same under both"""
    c = O.Ctx(64, 2, 256, log_base=15, digits=2)
    c6 = O.Ctx(64, 2, 256)
    assert c.primes == c6.primes and c.D == 4 and c6.D == 10
    s = c.keygen(4)
    assert np.array_equal(s, c6.keygen(4))
    K = c.pks_keygen(s, 77)
    assert K.shape == (64, 10, 2, 2, 64)
    assert np.array_equal(K, c6.pks_keygen(s, 77))
    rng = np.random.default_rng(5)
    msgs = rng.integers(0, 256, 20)
    lwes = []
    for i, m in enumerate(msgs):
        mu = rng.integers(0, 256, 64).astype(np.uint64)
        mu[0] = m
        ct = c.enc_rlwe(s, mu, 5, i)
        assert np.array_equal(ct, c6.enc_rlwe(s, mu, 5, i))
        lwes.append(c.extract_lwe0(ct))
    out = c.pack_lwe(K, np.stack(lwes))
    dec = c.dec_rlwe(s, out)
    assert np.array_equal(dec[:20], msgs.astype(np.uint64)) and not dec[20:].any()
