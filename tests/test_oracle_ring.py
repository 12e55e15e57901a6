"""Pins of the oracle's ring arithmetic: parameter primes by brute force,
NTT-based negacyclic products against schoolbook products (two independent
schoolbooks), monomial rotation and the gadget decomposition identity."""
import numpy as np
import pytest

import oracle as O


def _is_prime_py(n):
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    d = 3
    while d * d <= n:
        if n % d == 0:
            return False
        d += 2
    return True


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2), (4096, 3)])
def test_primes_rule_brute_force(N, nq):
    ps = O.find_primes(N, nq)
    assert ps == sorted(ps, reverse=True)
    for q in ps:
        assert q < 2**30 and (q - 1) % (2 * N) == 0 and _is_prime_py(q)
    # no larger candidate q = 1 mod 2N below 2^30 is prime, and none is skipped between them
    cands = [q for q in range(2**30 - 1, ps[-1] - 1, -1) if q % (2 * N) == 1]
    assert [q for q in cands if _is_prime_py(q)] == ps


def test_known_prime_values():
    # values the rule gives (checked by brute force above); fixed here so a change is visible
    assert O.find_primes(1024, 1) == [1073707009]
    assert O.find_primes(2048, 2) == [1073692673, 1073668097]
    assert O.find_primes(4096, 3) == [1073692673, 1073668097, 1073651713]


def _school_py(a, b, q):
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] = (out[k] + a[i] * b[j]) % q
            else:
                out[k - N] = (out[k - N] - a[i] * b[j]) % q
    return out


@pytest.mark.parametrize("N,q", [(8, 17), (16, 97), (32, 193)])
def test_ntt_vs_schoolbook_tiny(N, q):
    c = O.Ctx(N, 1, 4, primes=[q])
    rng = np.random.default_rng(N)
    for _ in range(20):
        a = rng.integers(0, q, N).astype(np.uint64)
        b = rng.integers(0, q, N).astype(np.uint64)
        want = _school_py([int(x) for x in a], [int(x) for x in b], q)
        assert c.negmul(0, a, b).tolist() == want
        assert O.negmul_schoolbook(q, a, b).tolist() == want


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2)])
def test_ntt_vs_schoolbook_large(N, nq):
    c = O.Ctx(N, nq, 64)
    rng = np.random.default_rng(7)
    for i, q in enumerate(c.primes):
        a = rng.integers(0, q, N).astype(np.uint64)
        b = rng.integers(0, q, N).astype(np.uint64)
        assert np.array_equal(c.negmul(i, a, b), O.negmul_schoolbook(q, a, b))


def test_x_to_the_n_is_minus_one():
    c = O.Ctx(16, 1, 4, primes=[97])
    xk = np.zeros(16, np.uint64)
    xk[15] = 1  # X^15 * X = X^16 = -1
    x1 = np.zeros(16, np.uint64)
    x1[1] = 1
    out = c.negmul(0, xk, x1)
    assert out[0] == 96 and out[1:].sum() == 0


def test_rotation_is_monomial_product():
    c = O.Ctx(32, 2, 16, primes=[193, 257])
    rng = np.random.default_rng(3)
    ct = np.stack([np.stack([rng.integers(0, q, 32) for q in c.primes])
                   for _ in range(2)]).astype(np.uint32)
    for e in [0, 1, 5, 31, 32, 33, 63, 64, -1, -7, -33, 100]:
        got = c.rotate(ct, e)
        em = e % 64
        mono = np.zeros(32, np.uint64)
        for p in range(2):
            for i, q in enumerate(c.primes):
                mono[:] = 0
                if em < 32:
                    mono[em] = 1
                else:
                    mono[em - 32] = q - 1
                want = O.negmul_schoolbook(q, ct[p, i].astype(np.uint64), mono)
                assert np.array_equal(got[p, i].astype(np.uint64), want)


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2), (4096, 3)])
def test_decomposition_identity(N, nq):
    c = O.Ctx(N, nq, 64)
    rng = np.random.default_rng(nq)
    poly = np.stack([rng.integers(0, q, N) for q in c.primes]).astype(np.uint32)
    # include the extreme residues
    for i, q in enumerate(c.primes):
        poly[i, :6] = [0, 1, q - 1, (q - 1) // 2, (q + 1) // 2, q // 3]
    dig = c.decompose(poly).reshape(nq, 5, N).astype(np.int64)
    assert dig[:, :4].min() >= -32 and dig[:, :4].max() <= 31
    assert np.abs(dig[:, 4]).max() <= 32
    for i, q in enumerate(c.primes):
        v = poly[i].astype(np.int64)
        centered = np.where(v > (q - 1) // 2, v - q, v)
        recon = sum(dig[i, j] * (64 ** j) for j in range(5))
        assert np.array_equal(recon, centered)


@pytest.mark.parametrize("N,nq", [(2048, 2), (4096, 3)])
def test_decomposition_identity_coarse_gadget(N, nq):
    """2 balanced digits of 15 bits per prime (the gadget offered on rings of
    two or more primes): digit bounds and exact reconstruction of the
    centred residue, extreme residues included"""
    c = O.Ctx(N, nq, 64, log_base=15, digits=2)
    rng = np.random.default_rng(10 + nq)
    poly = np.stack([rng.integers(0, q, N) for q in c.primes]).astype(np.uint32)
    for i, q in enumerate(c.primes):
        poly[i, :6] = [0, 1, q - 1, (q - 1) // 2, (q + 1) // 2, q // 3]
    dig = c.decompose(poly).reshape(nq, 2, N).astype(np.int64)
    assert dig[:, 0].min() >= -(1 << 14) and dig[:, 0].max() < (1 << 14)
    assert np.abs(dig[:, 1]).max() <= (1 << 14)
    for i, q in enumerate(c.primes):
        v = poly[i].astype(np.int64)
        centered = np.where(v > (q - 1) // 2, v - q, v)
        assert np.array_equal(dig[i, 0] + dig[i, 1] * (1 << 15), centered)
