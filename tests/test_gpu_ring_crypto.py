"""GPU parity: NTT, keys, encryption, decryption and the external product of
the HIP library against the CPU oracle, bit-exact (integer arithmetic)."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import dev, host_u32, host_u64, zeros_u32, zeros_u64

pytestmark = pytest.mark.gpu

SETS = [(1024, 1), (1024, 3), (2048, 2), (2048, 1), (4096, 3), (4096, 2)]


def _hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


def rand_polys(rng, primes, count, N):
    return np.stack([np.stack([rng.integers(0, q, N) for q in primes]) for _ in range(count)]).astype(np.uint32)


@pytest.mark.parametrize("N,nq", SETS)
def test_ntt_roundtrip_and_negacyclic_products(N, nq):
    import torch
    HW = _hw()
    ctx = HW.Context(N, nq, 64)
    orc = O.Ctx(N, nq, 64)
    assert ctx.primes == orc.primes
    rng = np.random.default_rng(N + nq)
    count = 37
    a, b = rand_polys(rng, ctx.primes, count, N), rand_polys(rng, ctx.primes, count, N)
    A, B = dev(a), dev(b)
    ctx.ntt(A, count, False)
    ctx.ntt(B, count, False)
    q = torch.tensor(ctx.primes, dtype=torch.int64, device="cuda").view(1, nq, 1)
    Pm = ((A.long() & 0xFFFFFFFF) * (B.long() & 0xFFFFFFFF) % q).to(torch.int32)
    ctx.ntt(Pm, count, True)
    ctx.ntt(A, count, True)
    got = host_u32(Pm)
    assert np.array_equal(host_u32(A), a)
    for c in [0, 1, count - 1]:
        for i in range(nq):
            want = orc.negmul(i, a[c, i].astype(np.uint64), b[c, i].astype(np.uint64))
            assert np.array_equal(got[c, i].astype(np.uint64), want), (c, i)


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384)])
def test_keygen_and_rlwe_encryption_bit_exact(N, nq, p):
    HW = _hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(123, sk)
    sk_o = orc.keygen(123)
    assert np.array_equal(host_u32(sk).view(np.int32), sk_o)
    rng = np.random.default_rng(p)
    count = 5
    msg = rng.integers(0, p, (count, N)).astype(np.uint64)
    out = zeros_u32(count, 2, nq, N)
    ctx.encrypt_rlwe(sk, dev(msg), count, 77, 3, out)
    got = host_u32(out)
    for c in range(count):
        assert np.array_equal(got[c], orc.enc_rlwe(sk_o, msg[c], 77, 3 + c)), c
    # zero message pointer encrypts zeros
    out0 = zeros_u32(1, 2, nq, N)
    ctx.encrypt_rlwe(sk, None, 1, 78, 0, out0)
    assert np.array_equal(host_u32(out0)[0], orc.enc_rlwe(sk_o, None, 78, 0))


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384)])
def test_rgsw_encryption_bit_exact(N, nq, p):
    HW = _hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(5, sk)
    sk_o = orc.keygen(5)
    bits = np.array([1, 0, 1, 1, 0], np.uint8)
    rg = zeros_u32(len(bits), ctx.rgsw_words)
    ctx.encrypt_rgsw_bits(sk, dev(bits), 31, 100, rg)
    exp = zeros_u32(len(bits), ctx.rgsw_words)
    ctx.rgsw_export(rg, len(bits), exp)
    got = host_u32(exp).reshape(len(bits), 10 * nq, 2, nq, N)
    for k in range(len(bits)):
        assert np.array_equal(got[k], orc.enc_rgsw(sk_o, int(bits[k]), 31, 100 + k)), k


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384)])
def test_decryption(N, nq, p):
    HW = _hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk_o = orc.keygen(9)
    sk = zeros_u32(N)
    ctx.keygen(9, sk)
    rng = np.random.default_rng(N)
    mu = rng.integers(0, p, N).astype(np.uint64)
    ct_enc = orc.enc_rlwe(sk_o, mu, 4, 0)
    ct_rand = rand_polys(rng, orc.primes, 2, N).reshape(1, 2, nq, N)
    cts = np.concatenate([ct_enc[None], ct_rand]).astype(np.uint32)
    out = zeros_u64(2, N)
    ctx.decrypt_rlwe(sk, dev(cts), 2, out)
    got = host_u64(out)
    assert np.array_equal(got[0], mu)
    assert np.array_equal(got[1], orc.dec_rlwe(sk_o, cts[1]))  # arbitrary phases: CRT rounding parity
    lwes = np.stack([orc.extract_lwe0(orc.rotate(ct_enc, -e)) for e in range(5)]
                    + [rng.integers(0, 2**30, (nq, N + 1)).astype(np.uint32) % np.array(orc.primes, np.uint32)[:, None]])
    outl = zeros_u64(len(lwes))
    ctx.decrypt_lwe(sk, dev(lwes), len(lwes), outl)
    gl = host_u64(outl)
    assert list(gl[:5]) == [int(mu[e]) for e in range(5)]  # coefficient 0 of X^{-e} m is m_e
    assert gl[5] == orc.dec_lwe(sk_o, lwes[5])


@pytest.mark.parametrize("N,nq,p", [(1024, 1, 64), (2048, 2, 1024), (4096, 3, 16384), (2048, 3, 1024)])
def test_external_product_bit_exact(N, nq, p):
    HW = _hw()
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk_o = orc.keygen(11)
    sk = zeros_u32(N)
    ctx.keygen(11, sk)
    rng = np.random.default_rng(nq * N)
    count = 3
    bits = np.array([1, 0, 1], np.uint8)
    rg = zeros_u32(count, ctx.rgsw_words)
    ctx.encrypt_rgsw_bits(sk, dev(bits), 21, 0, rg)
    rin = rand_polys(rng, orc.primes, 2 * count, N).reshape(count, 2, nq, N)
    rout = zeros_u32(count, 2, nq, N)
    ctx.external_product(rg, dev(rin), count, rout)
    got = host_u32(rout)

    def one(k):
        return orc.extprod(orc.enc_rgsw(sk_o, int(bits[k]), 21, k), rin[k])

    want = [None] * count
    O._parallel(lambda k: want.__setitem__(k, one(k)), range(count))
    for k in range(count):
        assert np.array_equal(got[k], want[k]), k
