"""Pins of the oracle's WiSARD layer: the paper's worked examples (Sec. 2.4.3,
Fig. 1, Fig. 2), encrypted training against the plaintext Integer WiSARD
(Alg. 4 vs Alg. 6, cell by cell), PD-act inference against Alg. 2, and the
additivity of the encrypted model."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import plain as P
from paper_2403_20190_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EX = json.load(open(os.path.join(GOLD, "paper_examples.json")))


def test_thermometer_examples():
    for case in EX["thermometer"]["cases"]:
        assert P.thermometer(case["x"], case["size"]) == case["bits"]
    assert P.encode(np.array([[3, 1]]), 4).tolist() == [[1, 1, 1, 0, 1, 0, 0, 0]]


def test_quantize_levels():
    v = np.arange(256)
    q = P.quantize_u8(v, 2)
    assert q.min() == 0 and q.max() == 2 and np.all(np.diff(q) >= 0)
    assert (q == 0).sum() == 86 and (q == 2).sum() == 85  # floor(3v/256)


def test_figure1_permutation_and_score():
    f = EX["figure1"]
    x = np.array(f["input"])
    t = x[np.array(f["perm"])]
    assert t.tolist() == f["address_bits"]
    W = np.array([f["rams"]])  # one discriminator
    # the figure labels cells as written strings t0 t1 (MSB first); read those
    drawn = ["".join(str(int(b)) for b in t[2 * j:2 * j + 2]) for j in range(2)]
    assert drawn == f["marked_cells_as_drawn"]
    assert sum(W[0, j, int(drawn[j], 2)] for j in range(2)) == f["score"]
    # with the LSB-first f_comp of Def. 1 the score of this discriminator is the same
    u = P.ram_scores(W, x, 2, np.array(f["perm"]))
    assert u.sum() == f["score"]


@pytest.mark.parametrize("key", ["figure2a", "figure2b"])
def test_figure2_scores(key):
    f = EX[key]
    W = np.array([f["rams"]])
    u = P.ram_scores(W, np.array(f["input"]), 2, np.arange(4))
    assert P.act_bin(u, f["threshold"]).sum() == f["score"]


def test_activations():
    x = np.array([0, 1, 2, 3, 4, 7, 8, 100])
    assert P.act_log(x).tolist() == [0, 1, 1, 2, 2, 3, 3, 6]
    assert P.act_blog(x, 2).tolist() == [0, 1, 1, 2, 2, 2, 2, 2]
    assert P.act_bin(x, 2).tolist() == [0, 0, 0, 1, 1, 1, 1, 1]
    assert P.argmax_lowest([1, 3, 3, 2]) == 1


def test_train_integer_counts():
    rng = np.random.default_rng(0)
    X = rng.integers(0, 2, (30, 10)).astype(np.uint8)
    y = rng.integers(0, 3, 30)
    pi = O.permutation(9, 10)
    W = P.train_integer(X, y, 3, 4, pi)
    assert W.shape == (3, 3, 16)
    assert W.sum() == 30 * 3
    for c in range(3):
        assert W[c].sum() == 3 * (y == c).sum()


class Micro:
    """Small encrypted WiSARD: exercises a ragged last tuple, an encrypted
    CDEMUX/CMUX tree level (z > L) and cleartext label bits in the chain."""

    def __init__(self, N, s, l, a, n, p=64, nq=1, seed=0, layout=0, gadget=(6, 5)):
        self.c = O.Ctx(N, nq, p, log_base=gadget[0], digits=gadget[1])
        self.s, self.l, self.a, self.n = s, l, a, n
        self.layout = layout
        self.L = O.ceil_log2(l)
        self.k0 = -(-s // a)
        self.k1 = self.c.k1(s, l, a, layout)
        X, y = synth.prototype_bits(seed, n, s, l, flip=0.2)
        self.X, self.y = X, y
        self.sk = self.c.keygen(100 + seed)
        self.pi = O.permutation(200 + seed, s)
        self.xr = self.c.enc_rgsw_bits(self.sk, X.reshape(-1), 300 + seed, 0).reshape(n, s, -1)
        yb = np.array([[(v >> u) & 1 for u in range(self.L)] for v in y]).reshape(-1)
        if self.L:
            self.yr = self.c.enc_rgsw_bits(self.sk, yb, 400 + seed, 0).reshape(n, self.L, -1)
        else:  # l = 1: no label bits
            self.yr = np.zeros((n, 0, self.xr.shape[-1]), np.uint32)

    def train(self, idx=None):
        idx = list(range(self.n)) if idx is None else list(idx)
        H = np.zeros((self.k0, self.k1, 2, self.c.nq, self.c.N), np.uint32)
        self.c.train(self.s, self.l, self.a, self.pi, lambda i, k: self.xr[idx[i], k],
                     lambda i, u: self.yr[idx[i], u], len(idx), H, layout=self.layout)
        return H


CONFIGS = [
    dict(N=32, s=5, l=200, a=2, n=5),  # L = 8 > z = 5: label bits in the tree and the chain; l not a power of two
    dict(N=16, s=3, l=2, a=1, n=4),    # one-bit tuples: nb = 2 <= log N, no tree
    dict(N=16, s=14, l=3, a=4, n=6),   # nb = 6, log N = 4: z = 2 = L -> tree levels are the label bits
    dict(N=8, s=10, l=2, a=4, n=5),    # nb = 5, log N = 3: z = 2 > L = 1 -> one encrypted tree level
    dict(N=32, s=9, l=5, a=3, n=6),    # nb = 6, log N = 5: z = 1 < L = 3 -> label bits in the chain
    dict(N=8, s=10, l=3, a=4, n=6),    # nb = 6, log N = 3: z = 3 > L = 2, l = 3: pruned label and tuple nodes
]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_encrypted_training_matches_integer_wisard(cfg):
    m = Micro(**cfg)
    H = m.train()
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    want = P.expected_model_cells(W, m.s, m.l, m.a, m.c.N)
    got = np.stack([[m.c.dec_rlwe(m.sk, H[j, d]) for d in range(m.k1)] for j in range(m.k0)])
    assert np.array_equal(got.astype(np.int64), want)
    # noise health of the trained model
    for j in range(m.k0):
        for d in range(m.k1):
            mx, _ = m.c.noise_rlwe(m.sk, H[j, d], want[j, d].astype(np.uint64))
            assert mx * 16 < m.c.delta / 2


@pytest.mark.parametrize("cfg", [CONFIGS[0], CONFIGS[3], CONFIGS[5]])
def test_encrypted_training_and_inference_coarse_gadget(cfg):
    """the same on two primes with RGSW of 2 digits of 15 bits per prime:
    decrypted cells equal integer WiSARD's counts with the noise margin of
    the default gadget's test, and PD-act predictions equal Alg. 2's"""
    m = Micro(**cfg, nq=2, gadget=(15, 2))
    assert m.c.D == 4 and m.xr.shape[-1] == m.c.rgsw_words
    H = m.train()
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    want = P.expected_model_cells(W, m.s, m.l, m.a, m.c.N)
    got = np.stack([[m.c.dec_rlwe(m.sk, H[j, d]) for d in range(m.k1)] for j in range(m.k0)])
    assert np.array_equal(got.astype(np.int64), want)
    for j in range(m.k0):
        for d in range(m.k1):
            mx, _ = m.c.noise_rlwe(m.sk, H[j, d], want[j, d].astype(np.uint64))
            assert mx * 16 < m.c.delta / 2
    Xt, _ = synth.prototype_bits(50, 3, m.s, m.l, flip=0.3)
    for t in range(3):
        xr = m.c.enc_rgsw_bits(m.sk, Xt[t], 500 + t, 0)
        cells = np.array([[m.c.dec_lwe(m.sk, m.c.infer_one(m.s, m.l, m.a, m.pi, H, lambda k: xr[k], j, c))
                           for j in range(m.k0)] for c in range(m.l)], np.int64)
        assert np.array_equal(cells, P.ram_scores(W, Xt[t], m.a, m.pi))
        assert P.pd_act_predict(cells, "log") == P.predict(W, Xt[t], m.a, m.pi, "log")


@pytest.mark.parametrize("cfg", CONFIGS)
def test_encrypted_inference_pd_act(cfg):
    m = Micro(**cfg)
    H = m.train()
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    Xt, _ = synth.prototype_bits(cfg.get("seed", 0) + 50, 3, m.s, m.l, flip=0.3)
    for t in range(3):
        xr = m.c.enc_rgsw_bits(m.sk, Xt[t], 500 + t, 0)
        cells = np.zeros((m.l, m.k0), np.int64)
        sums = []
        for c in range(m.l):
            acc = None
            for j in range(m.k0):
                lwe = m.c.infer_one(m.s, m.l, m.a, m.pi, H, lambda k: xr[k], j, c)
                cells[c, j] = m.c.dec_lwe(m.sk, lwe)
                acc = lwe if acc is None else m.c.lwe_add(acc, lwe)
            sums.append(m.c.dec_lwe(m.sk, acc))
        want = P.ram_scores(W, Xt[t], m.a, m.pi)
        assert np.array_equal(cells, want)
        assert sums == list(want.sum(axis=1) % m.c.p)
        for kind in ("bin", "log", "blog"):
            assert P.pd_act_predict(cells, kind) == P.predict(W, Xt[t], m.a, m.pi, kind)


PACKED = [
    dict(N=256, s=5, l=200, a=2, n=5),  # L = 8 = log2 N: z = 2 = a, every chain bit a label bit
    dict(N=16, s=14, l=3, a=4, n=6),   # z = 2 tuple bits in the tree, chain: 2 tuple + 2 label bits
    dict(N=8, s=10, l=2, a=4, n=5),    # z = 2, a ragged last tuple of 2 bits (z = 0 there)
    dict(N=32, s=9, l=5, a=3, n=6),    # z = 1, label bits on top of a 3-bit tuple
    dict(N=8, s=10, l=3, a=4, n=6),    # z = 3: 3 of the 4 tuple bits in the tree
    dict(N=16, s=7, l=1, a=7, n=4),    # l = 1: no label bits at all
]


@pytest.mark.parametrize("cfg", PACKED)
def test_class_packed_training_matches_integer_wisard(cfg):
    """Class-packed layout: every cell of the plaintext Integer WiSARD (Alg. 4)
    at row (addr + 2^a_j c) mod 2^z, coefficient (addr + 2^a_j c) >> z."""
    m = Micro(**cfg, layout=1)
    assert m.k1 == 1 << max(0, m.L + m.a - (m.c.N.bit_length() - 1))
    H = m.train()
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    want = P.expected_model_cells(W, m.s, m.l, m.a, m.c.N, layout=1)
    got = np.stack([[m.c.dec_rlwe(m.sk, H[j, d]) for d in range(m.k1)] for j in range(m.k0)])
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("cfg", PACKED)
def test_class_packed_inference_scores(cfg):
    """One VP per RAM gives the cell of every class: the extracted LWEs decrypt
    to the plaintext RAM scores of Alg. 2, and PD-act picks the same class."""
    m = Micro(**cfg, layout=1)
    H = m.train()
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    Xt, _ = synth.prototype_bits(51, 3, m.s, m.l, flip=0.3)
    for t in range(3):
        xr = m.c.enc_rgsw_bits(m.sk, Xt[t], 600 + t, 0)
        cells = np.zeros((m.l, m.k0), np.int64)
        for j in range(m.k0):
            lw = m.c.infer_packed(m.s, m.l, m.a, m.pi, H, lambda k: xr[k], j)
            for c in range(m.l):
                cells[c, j] = m.c.dec_lwe(m.sk, lw[c])
        want = P.ram_scores(W, Xt[t], m.a, m.pi)
        assert np.array_equal(cells, want)
        for kind in ("bin", "log", "blog"):
            assert P.pd_act_predict(cells, kind) == P.predict(W, Xt[t], m.a, m.pi, kind)


RAM_PACKED = [
    dict(N=16, s=9, l=2, a=2, n=5),    # 2^(L+a) = 8: two RAMs per row; ragged last tuple, a half-empty last row
    dict(N=32, s=12, l=3, a=2, n=6),   # 2^(L+a) = 16: two RAMs per row, l = 3 leaves a class block empty
    dict(N=64, s=10, l=1, a=3, n=4),   # l = 1: 2^a = 8, eight RAMs per row
]


@pytest.mark.parametrize("cfg", RAM_PACKED)
def test_several_rams_per_row(cfg):
    """Layout 2: packing the class-packed rows of r = N / 2^(L+a) RAMs into
    one RLWE puts every Alg. 4 count at offset (j mod r) 2^(L+a) of row
    j / r, and the VP of each RAM over its block gives the Alg. 2 scores."""
    m = Micro(**cfg, layout=1)
    H1 = m.train()
    r = m.c.rams_per_row(m.l, m.a)
    assert r == m.c.N >> (m.L + m.a) and r >= 2
    rows = m.c.model_rows(m.s, m.l, m.a, 2)
    assert rows == -(-m.k0 // r)
    H2 = m.c.pack_rams(m.s, m.l, m.a, H1)
    W = P.train_integer(m.X, m.y, m.l, m.a, m.pi)
    want = P.expected_model_cells(W, m.s, m.l, m.a, m.c.N, layout=2)
    got = np.stack([[m.c.dec_rlwe(m.sk, H2[R, 0])] for R in range(rows)])
    assert np.array_equal(got.astype(np.int64), want)
    Xt, _ = synth.prototype_bits(52, 2, m.s, m.l, flip=0.3)
    for t in range(2):
        xr = m.c.enc_rgsw_bits(m.sk, Xt[t], 700 + t, 0)
        cells = np.zeros((m.l, m.k0), np.int64)
        for j in range(m.k0):
            lw = m.c.infer_packed(m.s, m.l, m.a, m.pi, H2, lambda k: xr[k], j, layout=2)
            for c in range(m.l):
                cells[c, j] = m.c.dec_lwe(m.sk, lw[c])
        assert np.array_equal(cells, P.ram_scores(W, Xt[t], m.a, m.pi))


def test_class_packed_needs_label_bits_within_the_ring():
    """with L > log2 N the tree would hold label bits, which one VP cannot
    serve for every class: the oracle refuses the layout"""
    c = O.Ctx(32, 1, 64)
    assert c.k1(5, 200, 2, 0) == 32  # layout 0 holds it (z = 5 < L = 8: all leaves)
    for layout in (1, 2):
        with pytest.raises(ValueError):
            c.k1(5, 200, 2, layout)


def test_extract_lwe_any_index():
    """ExtractLWE(c, i) decrypts to coefficient i of c's phase for every i,
    the phase taken by the negacyclic product of the decryption."""
    c = O.Ctx(16, 2, 64)
    sk = c.keygen(7)
    msg = (np.arange(16, dtype=np.uint64) * 5 + 3) % 64
    ct = c.enc_rlwe(sk, msg, 8, 0)
    for i in range(16):
        assert c.dec_lwe(sk, c.extract_lwe(ct, i)) == int(msg[i])
    assert np.array_equal(c.extract_lwe(ct, 0), c.extract_lwe0(ct))


def test_model_additivity_and_order():
    """H(A u B) = H(A) + H(B) and any sample order gives the same bits (Sec. 3.7.2)."""
    m = Micro(N=16, s=14, l=3, a=4, n=6)
    H = m.train()
    HA = m.train(range(0, 3))
    HB = m.train(range(3, 6))
    q = m.c.primes[0]
    assert np.array_equal(H, ((HA.astype(np.uint64) + HB) % q).astype(np.uint32))
    assert np.array_equal(H, m.c.rlwe_add(HA, HB))  # the oracle's merge
    assert np.array_equal(H, m.train([5, 2, 0, 4, 1, 3]))


def test_class_counter():
    m = Micro(N=16, s=14, l=3, a=4, n=6)
    cnt = np.zeros((2, 1, 16), np.uint32)
    m.c.class_count(m.l, lambda i, u: m.yr[i, u], m.n, cnt)
    dec = m.c.dec_rlwe(m.sk, cnt)
    assert dec[:3].tolist() == [int((m.y == c).sum()) for c in range(3)]
    assert not dec[3:].any()


def test_checkpoint_roundtrip_host(tmp_path):
    """save_checkpoint / load_checkpoint keep the words and the metadata (host tensors)."""
    import torch

    from paper_2403_20190_amd import client as CL
    rng = np.random.default_rng(1)
    H = torch.from_numpy(rng.integers(0, 2**31, (3, 2, 2, 1, 16)).astype(np.int32))
    C = torch.from_numpy(rng.integers(0, 2**31, (2, 1, 16)).astype(np.int32))
    CL.save_checkpoint(tmp_path / "c.npz", H, C, N=16, trained=7)
    H2, C2, meta = CL.load_checkpoint(tmp_path / "c.npz", device="cpu")
    assert torch.equal(H, H2) and torch.equal(C, C2) and meta == {"N": 16, "trained": 7}
