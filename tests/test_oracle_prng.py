"""Pins of the oracle's random draws: Philox4x32-10 against published
known-answer vectors, the 64-bit draw layout, the Gaussian CDT against an
independent computation of the distribution, and sampler statistics."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLD, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert O.philox4x32_10(ctr, key) == [int(x, 16) for x in v["out"]]


def test_w64_layout():
    # even index -> words 0,1 of block index/2; odd -> words 2,3; key = seed, ctr = (blk, domain, 0)
    seed, dom = 0x0123456789ABCDEF, 3
    for idx in [0, 1, 2, 3, 12345, 2**33 + 7]:
        blk = idx >> 1
        o = O.philox4x32_10([blk & 0xFFFFFFFF, blk >> 32, dom, 0], [seed & 0xFFFFFFFF, seed >> 32])
        want = (o[2] | (o[3] << 32)) if idx & 1 else (o[0] | (o[1] << 32))
        assert O.w64(seed, dom, idx) == want


def test_w32_layout():
    # word index mod 4 of block index / 4; key = seed, ctr = (blk, domain, 0)
    seed, dom = 0x0123456789ABCDEF, 3
    for idx in [0, 1, 2, 3, 4, 7, 12345, 2**34 + 6]:
        blk = idx >> 2
        o = O.philox4x32_10([blk & 0xFFFFFFFF, blk >> 32, dom, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert O.w32(seed, dom, idx) == o[idx & 3]


def test_uniform_residue_rule():
    """Accepted words (below floor(2^32/q) q) give w mod q; the rejected ones
    (found by search: about 3e-5 of them at q near 2^30) take the 64-bit
    fallback draw of domain 5.  Accepted words are exactly uniform: every
    residue has floor(2^32/q) preimages below the limit."""
    q = 1073707009
    lim = (2**32 // q) * q
    seed = 91
    rejected = [x for x in range(300000) if O.w32(seed, 3, x) >= lim]
    assert rejected, "expected a rejected word among 300000 draws"
    for x in rejected[:5]:
        assert O.uniform_mod(seed, x, q) == O.w64(seed, 5, x) % q
    for x in [0, 1, 2, 3, 99, 123457]:
        if x not in rejected:
            assert O.uniform_mod(seed, x, q) == O.w32(seed, 3, x) % q
    # small prime: the rejection rate is (2^32 mod q) / 2^32 and the limit is a multiple of q
    q2 = 12289
    lim2 = (2**32 // q2) * q2
    assert lim2 % q2 == 0 and 2**32 - lim2 == 2**32 % q2 < q2
    vals = [O.uniform_mod(7, x, q2) for x in range(20000)]
    assert min(vals) >= 0 and max(vals) < q2
    # a crude uniformity check: the mean of 20000 residues within 5 sigma of (q - 1) / 2
    mean = sum(vals) / len(vals)
    sd = (q2 / 12 ** 0.5) / len(vals) ** 0.5
    assert abs(mean - (q2 - 1) / 2) < 5 * sd


def test_cdt_table_matches_distribution():
    sigma = 3.2
    T = O.cdt_table(sigma)
    assert T[41] == 2**63
    # strictly increasing until the double-precision CDF reaches 1 (tail mass < 2^-53), then 2^63
    sat = next(k for k in range(42) if int(T[k]) == 2**63)
    assert sat > 20  # > 6 sigma of support is represented
    assert all(T[k] < T[k + 1] for k in range(sat - 1)) and all(int(T[k]) == 2**63 for k in range(sat, 42))
    # independent computation of P(|X| <= k) with math.fsum
    rho = [math.exp(-x * x / (2 * sigma * sigma)) for x in range(42)]
    Z = math.fsum([rho[0]] + [2 * r for r in rho[1:]])
    for k in range(41):
        P = math.fsum([rho[0]] + [2 * r for r in rho[1:k + 1]]) / Z
        assert abs(int(T[k]) / 2**63 - P) < 1e-14
    # P(|X| <= 0) = 1/Z
    assert abs(int(T[0]) / 2**63 - 1 / Z) < 1e-15


def test_cdt_sampler_rule():
    T = O.cdt_table(3.2)
    # explicit boundary cases of the rule "smallest k with (w >> 1) < T[k]"
    assert O.cdt_sample(T, 0) == 0
    assert O.cdt_sample(T, 1) == 0  # magnitude 0 ignores the sign bit
    w = int(T[0]) << 1  # (w >> 1) == T[0] -> magnitude 1, positive
    assert O.cdt_sample(T, w) == 1
    assert O.cdt_sample(T, w | 1) == -1
    sat = next(k for k in range(42) if int(T[k]) == 2**63)
    assert O.cdt_sample(T, 2**64 - 1) == -sat


def test_gaussian_statistics():
    c = O.Ctx(1024, 1, 64)
    s = c.keygen(11)
    # fresh RLWE noise is exactly e: gather it over many encryptions of 0
    noise = []
    for ct in range(24):
        enc = c.enc_rlwe(s, None, 99, ct)
        _, nz = c.noise_rlwe(s, enc, np.zeros(1024, np.uint64))
        noise.append(nz)
    e = np.concatenate(noise)
    assert np.all(e == np.round(e)) and np.abs(e).max() <= 41
    assert abs(e.mean()) < 0.1
    assert abs(e.var() / 3.2**2 - 1) < 0.05


def test_ternary_key():
    c = O.Ctx(2048, 2, 1024)
    s = c.keygen(5)
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    assert np.all(np.abs(counts / 2048 - 1 / 3) < 0.05)
    # definition: s_k = (w64(seed, KEY=1, k) mod 3) - 1
    for k in [0, 1, 7, 2047]:
        assert s[k] == O.w64(5, 1, k) % 3 - 1


def test_permutation_fisher_yates():
    s, seed = 37, 42
    pi = O.permutation(seed, s)
    assert sorted(pi.tolist()) == list(range(s))
    # re-derive with the stated rule in Python
    ref = list(range(s))
    for k in range(s - 1, 0, -1):
        j = O.w64(seed, 2, s - 1 - k) % (k + 1)
        ref[k], ref[j] = ref[j], ref[k]
    assert pi.tolist() == ref
    assert O.permutation(seed, 1).tolist() == [0]
