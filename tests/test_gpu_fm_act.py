"""GPU parity of FM-act (Sec. 3.5.3; Alg. 7's FM-act branch): every cell of a
trained model activated by bootstraps and packed back into its row.

* Bit for bit against the oracle on a small model (N = 1024, one prime,
  p = 8: 2 RAMs of 4 cells, 6 bootstraps per cell in sequence take the
  oracle about a minute), out of place and in place.
* At the Wisconsin-shaped parameter set (N = 2048, two primes, p = 512,
  a = 8: 512 cells per row) with the log activation, by decryption: every
  coefficient of the activated model is log(W) of the cell the layout puts
  there (0 past the cells), and inference on it with class sums and
  EncryptedArgMax gives Alg. 2 with the log activation, computed in the
  clear; the same with b-log on class-packed models (layouts 1 and 2)."""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as P
from gpu_helpers import Pair, host_u32, host_u64, zeros_u32, zeros_u64

pytestmark = pytest.mark.gpu


def hw():
    from paper_2403_20190_amd import hwisard as HW
    return HW


def test_fm_act_bit_exact_with_oracle():
    N, T = 1024, 2
    rng = np.random.default_rng(31)
    X = rng.integers(0, 2, (6, 2)).astype(np.uint8)
    y = np.array([0, 1, 0, 0, 1, 1])
    pair = Pair(N, 1, 8, 2, 2, 1, X, y, seed=19)
    ctx, orc = pair.ctx, pair.orc
    H = zeros_u32(pair.k0, pair.k1, 2, 1, N)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    Ho = pair.oracle_train(range(pair.k0))
    assert np.array_equal(host_u32(H), Ho)  # the model FM-act starts from
    bsk = zeros_u32(ctx.pbs_key_words(N))
    ctx.pbs_keygen(pair.sk, 42, N, bsk)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 9, key)
    out = zeros_u32(*H.shape)
    ctx.fm_act(pair.shape, bsk, N, key, H, "ge", T, 3, out)
    inplace = H.clone()
    ctx.fm_act(pair.shape, bsk, N, key, inplace, "ge", T, 3, inplace)
    got = host_u32(out)
    assert np.array_equal(host_u32(inplace), got)
    bsk_o = orc.pbs_keygen(pair.sk_o, 42, N)
    K_o = orc.pks_keygen(pair.sk_o, 9)
    want = B.fm_act(orc, bsk_o, N, K_o, Ho, B.fm_cells(N, 2, 1), T, 8)
    assert np.array_equal(got, want)
    W = P.train_integer(pair.X, pair.y, 2, 1, pair.pi)
    cells = P.expected_model_cells(W, 2, 2, 1, N)
    assert cells.max() >= T and (cells[..., :4] < T).any()
    dec = [[B.decode(orc, pair.sk_o, orc.extract_lwe(want[j, r], k), 8) for k in range(8)]
           for j in range(pair.k0) for r in range(pair.k1)]
    assert dec == [[int(v >= T) for v in cells[j, r, :8]] for j in range(pair.k0) for r in range(pair.k1)]


def test_fm_act_rejects_bad_arguments():
    HW = hw()
    N = 1024
    pair = Pair(N, 1, 8, 2, 2, 1, np.zeros((1, 2), np.uint8), np.zeros(1), seed=3)
    ctx = pair.ctx
    H = zeros_u32(pair.k0, pair.k1, 2, 1, N)
    bsk = zeros_u32(ctx.pbs_key_words(N))  # full size: nothing here may read past a buffer
    key = zeros_u32(ctx.pks_key_words)
    for kind, T, lp in (("ge", 0, 3), ("ge", 9, 3), ("ge", 2, 0), ("ge", 2, 61), ("blog", 0, 3)):
        with pytest.raises(HW.HwError):
            ctx.fm_act(pair.shape, bsk, N, key, H, kind, T, lp, H)
    big = zeros_u32(2 * pair.k0, pair.k1, 2, 1, N)
    with pytest.raises(HW.HwError):  # a partial overlap of model and output
        ctx.fm_act(pair.shape, bsk, N, key, big[:pair.k0], "ge", 2, 3, big[1:1 + pair.k0])


def test_fm_act_wisconsin_shape_by_decryption():
    """log activation, the one the paper's parameter table gives the
    Wisconsin model (Sec. 2.4.2)"""
    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import synth
    HW = hw()
    N, s, a, l, lp = 2048, 16, 8, 2, 6  # class sums of log cells <= 2 x 9 < 2^6 / 2
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)[:, :s]
    pair = Pair(N, 2, 512, s, l, a, bits[:60], yw[:60], seed=23)
    ctx = pair.ctx
    H = zeros_u32(pair.k0, pair.k1, 2, 2, N)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    bsk = zeros_u32(ctx.pbs_key_words(N))
    ctx.pbs_keygen(pair.sk, 44, N, bsk)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 45, key)
    act = zeros_u32(*H.shape)
    ctx.fm_act(pair.shape, bsk, N, key, H, "log", 0, lp, act)
    W = P.train_integer(pair.X, pair.y, l, a, pair.pi)
    cells = P.expected_model_cells(W, s, l, a, N)
    assert B.fm_cells(N, l, a) == 512 and cells[..., 512:].max() == 0
    assert len(set(P.act_log(cells).ravel())) >= 4  # several log levels occur
    cp = HW.Context(N, 2, 1 << lp)
    dec = zeros_u64(pair.k0 * pair.k1, N)
    cp.decrypt_rlwe(pair.sk, act, pair.k0 * pair.k1, dec)
    assert np.array_equal(host_u64(dec).reshape(cells.shape).astype(np.int64), P.act_log(cells))
    # Alg. 7, FM-act branch: VP on the activated model, class sums, EncryptedArgMax
    tb = bits[[70, 71, 72, 73, 74, 112, 175, 192]]
    nt = len(tb)
    xt = pair.encrypt_dev(tb, seed_x=67)
    sc = zeros_u32(nt, l, pair.k0, ctx.lwe_words)
    ctx.infer(pair.shape, act, xt, nt, sc, None)
    sums = zeros_u32(nt, l, ctx.lwe_words)
    ctx.class_sums(sc, nt, l, pair.k0, sums)
    ds = zeros_u64(nt * l)
    cp.decrypt_lwe(pair.sk, sums, nt * l, ds)
    want_sums = [P.activate(P.ram_scores(W, tb[i], a, pair.pi), "log").sum(axis=1) for i in range(nt)]
    assert np.array_equal(host_u64(ds).reshape(nt, l).astype(np.int64), np.array(want_sums))
    idx = zeros_u32(nt, ctx.lwe_words)
    ctx.encrypted_argmax(bsk, N, sums, nt, l, lp, idx)
    c4 = HW.Context(N, 2, 4)
    di = zeros_u64(nt)
    c4.decrypt_lwe(pair.sk, idx, nt, di)
    want = [P.predict(W, tb[i], a, pair.pi, "log") for i in range(nt)]
    assert len(set(want)) == 2
    assert list(host_u64(di)) == want


@pytest.mark.parametrize("layout", [1, 2])
def test_fm_act_class_packed_layouts_by_decryption(layout):
    """FM-act of class-packed models (layout 1: one row per RAM holding every
    class; layout 2: four such RAMs per row, whose 2048 coefficients are all
    cells) with b-log, cap 2 (Sec. 2.4.2), at the Wisconsin-shaped
    parameters: every coefficient of the activated rows decrypts to b-log of
    the cell the layout puts there, and inference on the activated model,
    class sums and EncryptedArgMax give Alg. 2 with b-log."""
    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import synth
    HW = hw()
    N, s, a, l, cap, lp = 2048, 32, 8, 2, 2, 5  # class sums <= 4 RAMs x 2 < 2^5 / 2
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)[:, :s]
    pair = Pair(N, 2, 512, s, l, a, bits[:60], yw[:60], seed=29, layout=layout)
    ctx = pair.ctx
    rows, _ = ctx.model_rows(pair.shape)
    H = zeros_u32(rows, pair.k1, 2, 2, N)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    bsk = zeros_u32(ctx.pbs_key_words(N))
    ctx.pbs_keygen(pair.sk, 46, N, bsk)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 47, key)
    act = zeros_u32(*H.shape)
    ctx.fm_act(pair.shape, bsk, N, key, H, "blog", cap, lp, act)
    W = P.train_integer(pair.X, pair.y, l, a, pair.pi)
    cells = P.expected_model_cells(W, s, l, a, N, layout=layout)
    assert cells.shape == (rows, pair.k1, N) and B.fm_cells(N, l, a, layout) * rows * pair.k1 == 2048
    assert set(P.act_blog(cells, cap).ravel()) == {0, 1, 2}
    cp = HW.Context(N, 2, 1 << lp)
    dec = zeros_u64(rows * pair.k1, N)
    cp.decrypt_rlwe(pair.sk, act, rows * pair.k1, dec)
    assert np.array_equal(host_u64(dec).reshape(cells.shape).astype(np.int64), P.act_blog(cells, cap))
    tb = bits[[60, 61, 62, 63, 72, 74, 81, 91]]  # Alg. 2 with b-log predicts both classes among these
    nt = len(tb)
    xt = pair.encrypt_dev(tb, seed_x=68)
    sc = zeros_u32(nt, l, pair.k0, ctx.lwe_words)
    ctx.infer(pair.shape, act, xt, nt, sc, None)
    sums = zeros_u32(nt, l, ctx.lwe_words)
    ctx.class_sums(sc, nt, l, pair.k0, sums)
    idx = zeros_u32(nt, ctx.lwe_words)
    ctx.encrypted_argmax(bsk, N, sums, nt, l, lp, idx)
    di = zeros_u64(nt)
    HW.Context(N, 2, 4).decrypt_lwe(pair.sk, idx, nt, di)
    want = [P.predict(W, tb[i], a, pair.pi, "blog", 0, cap) for i in range(nt)]
    assert sorted(set(want)) == [0, 1]
    assert list(host_u64(di)) == want
