"""Pins of the oracle's TFHE building blocks (Sec. 2.5.1, Alg. 3, Alg. 5):
noiseless special cases that must hold bit-exactly, decryption semantics of
every gate including negacyclic signs, brute force of IVP and VP over every
index on small rings, CRT decoding and noise health."""
import itertools

import numpy as np
import pytest

import oracle as O

# a small ring so brute force over indices stays cheap; 30-bit primes = 1 mod 2N
SMALL = dict(N=16, nq=2, p=16)


def rand_rlwe(c, rng):
    return np.stack([np.stack([rng.integers(0, q, c.N) for q in c.primes]) for _ in range(2)]).astype(np.uint32)


@pytest.mark.parametrize("N,nq,gadget", [(16, 1, (6, 5)), (16, 2, (6, 5)), (1024, 1, (6, 5)), (2048, 2, (6, 5)),
                                         (64, 3, (6, 5)), (16, 2, (15, 2)), (2048, 2, (15, 2)), (64, 3, (15, 2))])
def test_trivial_rgsw_is_identity(N, nq, gadget):
    """G [.] c = c and 0 [.] c = 0 bit-exactly: fixes row order, digit order, sides
    (both gadgets: 5 digits of 6 bits, and 2 of 15 bits on two or more primes)."""
    c = O.Ctx(N, nq, 64, log_base=gadget[0], digits=gadget[1])
    rng = np.random.default_rng(N + nq)
    ct = rand_rlwe(c, rng)
    assert np.array_equal(c.extprod(c.trivial_rgsw(1), ct), ct)
    assert not c.extprod(c.trivial_rgsw(0), ct).any()
    # CMUX with trivial selectors is exact selection
    d1 = rand_rlwe(c, rng)
    assert np.array_equal(c.cmux(c.trivial_rgsw(1), d1, ct), d1)
    assert np.array_equal(c.cmux(c.trivial_rgsw(0), d1, ct), ct)


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384)])
def test_enc_dec_roundtrip(N, nq, p):
    c = O.Ctx(N, nq, p)
    s = c.keygen(1)
    rng = np.random.default_rng(p)
    mu = rng.integers(0, p, N).astype(np.uint64)
    ct = c.enc_rlwe(s, mu, 3, 5)
    assert np.array_equal(c.dec_rlwe(s, ct), mu)
    mx, _ = c.noise_rlwe(s, ct, mu)
    assert mx <= 41
    # RGSW row 0 decrypts like an RLWE of m * g_{0,0} = m in coefficient 0 (gadget in b)
    rg = c.enc_rgsw(s, 1, 3, 9)
    assert rg.shape == (2 * 5 * nq, 2, nq, N)


def test_crt_decode_rounding():
    c = O.Ctx(16, 2, 16)
    s = np.zeros(16, np.int32)  # zero key: the phase is b itself
    Q, d = c.Q, c.delta
    for mu in [0, 1, 7, 15]:
        for off in [0, 1, -1, d // 2 - 1, -(d // 2) + 1]:
            phi = (mu * d + off) % Q
            ct = np.zeros((2, 2, 16), np.uint32)
            for i, q in enumerate(c.primes):
                ct[1, i, 0] = phi % q
            assert c.dec_rlwe(s, ct)[0] == mu
    # the half-way point rounds up: phi = floor(Q/2)/p*... checked against the formula
    for phi in [Q // 2, Q - 1, Q // 32, Q // 32 - 1]:
        ct = np.zeros((2, 2, 16), np.uint32)
        for i, q in enumerate(c.primes):
            ct[1, i, 0] = phi % q
        assert c.dec_rlwe(s, ct)[0] == ((16 * phi + Q // 2) // Q) % 16


def test_extprod_decrypts_to_product():
    c = O.Ctx(1024, 1, 64)
    s = c.keygen(2)
    rng = np.random.default_rng(0)
    mu = rng.integers(0, 64, 1024).astype(np.uint64)
    ct = c.enc_rlwe(s, mu, 5, 0)
    for m in (0, 1):
        out = c.extprod(c.enc_rgsw(s, m, 6, m), ct)
        assert np.array_equal(c.dec_rlwe(s, out), (m * mu) % 64)


def test_cmux_cdemux_semantics():
    c = O.Ctx(1024, 1, 64)
    s = c.keygen(3)
    rng = np.random.default_rng(1)
    m1 = rng.integers(0, 64, 1024).astype(np.uint64)
    m0 = rng.integers(0, 64, 1024).astype(np.uint64)
    d1, d0 = c.enc_rlwe(s, m1, 7, 0), c.enc_rlwe(s, m0, 7, 1)
    for bit in (0, 1):
        C = c.enc_rgsw(s, bit, 8, bit)
        assert np.array_equal(c.dec_rlwe(s, c.cmux(C, d1, d0)), m1 if bit else m0)
        o0, o1 = c.cdemux(C, d1)
        assert np.array_equal(c.dec_rlwe(s, o0), m1 * (1 - bit))
        assert np.array_equal(c.dec_rlwe(s, o1), m1 * bit)


def _negacyclic_shift(v, e, p):
    N = len(v)
    out = np.zeros(N, np.int64)
    for j in range(N):
        t = (j + e) % (2 * N)
        if t < N:
            out[t] = (out[t] + v[j]) % p
        else:
            out[t - N] = (out[t - N] - v[j]) % p
    return out


def test_blind_rotate_semantics_with_wrap():
    c = O.Ctx(16, 2, 16)
    s = c.keygen(4)
    rng = np.random.default_rng(2)
    v = rng.integers(0, 16, 16).astype(np.uint64)
    ct = c.enc_rlwe(s, v, 9, 0)
    exps = [3, 7, 11, -5]
    for bits in itertools.product([0, 1], repeat=4):
        Cs = [c.enc_rgsw(s, b, 10, 4 * sum(x << i for i, x in enumerate(bits)) + t) for t, b in enumerate(bits)]
        out = c.blind_rotate(ct, Cs, exps)
        tot = sum(b * e for b, e in zip(bits, exps))
        assert np.array_equal(c.dec_rlwe(s, out).astype(np.int64), _negacyclic_shift(v.astype(np.int64), tot, 16))


def _bits_rgsw(c, s, m, nb, seed, ct0):
    return [c.enc_rgsw(s, (m >> u) & 1, seed, ct0 + u) for u in range(nb)]


@pytest.mark.parametrize("nb", [3, 5, 6])
def test_ivp_one_hot_brute_force(nb):
    """IVP output decrypts to zero everywhere except cell m, which holds f(m) (Alg. 5)."""
    c = O.Ctx(**SMALL)  # log2 N = 4 -> nb = 5, 6 exercise the CDEMUX tree (z = 1, 2)
    s = c.keygen(5)
    z = nb - min(nb, c.logN)
    for m in range(1 << nb):
        val = 1 + (m % 13)
        Cs = _bits_rgsw(c, s, m, nb, 11, 100 * m)
        out = c.ivp(Cs, c.trivial_rlwe(val))
        assert out.shape[0] == 1 << z
        dec = np.stack([c.dec_rlwe(s, o) for o in out])
        want = np.zeros_like(dec)
        want[m % (1 << z), m >> z] = val
        assert np.array_equal(dec, want), m


@pytest.mark.parametrize("N,nb,l", [(8, 6, 3), (16, 6, 3), (8, 7, 5), (16, 5, 2)])
def test_pruned_ivp_brute_force(N, nb, l):
    """The IVP with only the tree nodes that lead to a class below l: for
    every index m = c + 2^L addr with c < l, the live leaves decrypt to the
    one-hot table of the full IVP (Alg. 5), the leaf count is k1 of
    Definition 2, and a non-live leaf is never written.  Also the external
    products it saves: live leaves - 1 instead of 2^z - 1."""
    c = O.Ctx(N, 1, 16)
    s = c.keygen(8)
    L = O.ceil_log2(l)
    z = nb - min(nb, c.logN)
    live = [d for d in range(1 << z) if O.leaf_row(d, z, l) >= 0]
    assert len(live) == (l << (z - L) if z >= L else 1 << z)
    assert sorted(O.leaf_row(d, z, l) for d in live) == list(range(len(live)))
    for m in range(1 << nb):
        if m % (1 << L) >= l:
            continue
        val = 1 + (m % 7)
        Cs = _bits_rgsw(c, s, m, nb, 21, 100 * m)
        full = c.ivp(Cs, c.trivial_rlwe(val))
        pr = c.ivp_pruned(Cs, l, c.trivial_rlwe(val))
        for d in range(1 << z):
            if d in live:
                want = np.zeros(N, np.int64)
                if d == m % (1 << z):
                    want[m >> z] = val
                assert np.array_equal(c.dec_rlwe(s, pr[d]), want), (m, d)
                assert np.array_equal(c.dec_rlwe(s, full[d]), want), (m, d)
            else:
                assert not pr[d].any(), (m, d)


def test_vp_inverts_ivp_brute_force():
    """VP(bits(m'), IVP(bits(m), x)) decrypts to x [m' = m] (Alg. 3 read as the inverse of Alg. 5),
    with the low bits given in the clear like the label bits of Alg. 7."""
    c = O.Ctx(8, 1, 16)  # log2 N = 3
    s = c.keygen(6)
    nb, n_clear = 5, 1  # z = 2 > number of cleartext bits: one encrypted tree level
    for m in range(1 << nb):
        lut = c.ivp(_bits_rgsw(c, s, m, nb, 12, 50 * m), c.trivial_rlwe(5))
        for mp in range(1 << nb):
            rg = _bits_rgsw(c, s, mp, nb, 13, 1000 + 50 * mp)
            clear = [(mp >> u) & 1 for u in range(nb)]
            rg = [None if u < n_clear else rg[u] for u in range(nb)]
            lwe = c.vp(rg, clear, lut)
            assert c.dec_lwe(s, lwe) == (5 if mp == m else 0), (m, mp)


def test_extract_lwe_coefficient_zero():
    c = O.Ctx(1024, 1, 64)
    s = c.keygen(7)
    rng = np.random.default_rng(3)
    mu = rng.integers(0, 64, 1024).astype(np.uint64)
    ct = c.enc_rlwe(s, mu, 14, 0)
    for e in [0, -1, -37, -1023]:
        lwe = c.extract_lwe0(c.rotate(ct, e))
        assert c.dec_lwe(s, lwe) == _negacyclic_shift(mu.astype(np.int64), e, 64)[0]
    # LWE addition adds messages
    l2 = c.lwe_add(c.extract_lwe0(ct), c.extract_lwe0(c.rotate(ct, -1)))
    assert c.dec_lwe(s, l2) == (int(mu[0]) + int(mu[1])) % 64


def test_noise_health_after_chain():
    """Noise after a full rotation chain stays far below Delta/2 (margin >= 2^4)."""
    c = O.Ctx(2048, 2, 1024)
    s = c.keygen(8)
    Cs = _bits_rgsw(c, s, 0b10110110101, 11, 15, 0)
    out = c.ivp(Cs, c.trivial_rlwe(1))
    mu = np.zeros(2048, np.uint64)
    mu[0b10110110101] = 1
    mx, _ = c.noise_rlwe(s, out[0], mu)
    assert mx * 16 < c.delta / 2


def _psi(q, N):
    """psi = g^((q-1)/2N) for the smallest quadratic non-residue g >= 2 (Euler's
    criterion), a primitive 2N-th root of unity mod q: psi^N = -1."""
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    psi = pow(g, (q - 1) // (2 * N), q)
    assert pow(psi, N, q) == q - 1
    return psi


def _brv(k, bits):
    return int(format(k, "0%db" % bits)[::-1], 2)


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2)])
def test_rgsw_rows_draw_a_by_its_evaluations(N, nq):
    """An RGSW row's uniform a is drawn as its values at the points
    psi^(2 brv(k) + 1): evaluating the oracle's coefficient-form a there by
    Horner's rule (brute force, no transform) gives back draw k.  RLWE
    ciphertexts draw a by its coefficients."""
    c = O.Ctx(N, nq, 64)
    s = c.keygen(5)
    seed, ct = 77, 3
    rows = 2 * 5 * nq
    rg = c.enc_rgsw(s, 0, seed, ct)  # bit 0: no gadget term on the a side
    logN = N.bit_length() - 1
    for r in (0, rows - 1):
        for i, q in enumerate(c.primes):
            a = [int(v) for v in rg[r, 0, i]]
            psi = _psi(q, N)
            for k in (0, 1, 2, N // 2 + 3, N - 1):
                x = pow(psi, 2 * _brv(k, logN) + 1, q)
                acc = 0
                for coef in reversed(a):
                    acc = (acc * x + coef) % q
                assert acc == O.uniform_mod(seed, ((ct * rows + r) * nq + i) * N + k, q), (r, i, k)
    rl = c.enc_rlwe(s, np.zeros(N, np.uint64), seed, ct)
    for i, q in enumerate(c.primes):
        for k in (0, 5, N - 1):
            assert int(rl[0, i, k]) == O.uniform_mod(seed, (ct * nq + i) * N + k, q)


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2)])
def test_rlwe_error_draw_order(N, nq):
    """The error of an encryption of 0, b - a s recomputed with the
    schoolbook product (no transform), is coefficient by coefficient the CDT
    sample of error draw 8 (k mod N/8) + floor(k / (N/8)) of the row."""
    c = O.Ctx(N, nq, 64)
    s = c.keygen(9)
    seed, ct = 41, 2
    rl = c.enc_rlwe(s, np.zeros(N, np.uint64), seed, ct)
    T = O.cdt_table(3.2)
    q = c.primes[0]
    a = rl[0, 0].astype(np.uint64)
    b = rl[1, 0].astype(np.int64)
    sk = np.array([(int(v) + q) % q for v in s], np.uint64)
    e = (b - O.negmul_schoolbook(q, a, sk).astype(np.int64)) % q
    e = np.where(e > q // 2, e - q, e)
    for k in (0, 1, N // 8 - 1, N // 8, N // 8 + 1, N // 2 + 5, N - 1):
        pos = 8 * (k % (N // 8)) + k // (N // 8)
        assert e[k] == O.cdt_sample(T, O.w64(seed, 4, ct * N + pos)), k
