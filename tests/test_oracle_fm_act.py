"""Pins of the oracle's FM-act (oracle.pbs.fm_act; Sec. 3.5.3) against the
plaintext Integer WiSARD, on a 128-coefficient ring (one prime, p = 16) so
that every bootstrap runs over the whole key as it does at full size:

* every coefficient of every activated model row decrypts to [W >= T] of the
  cell the layout puts there (expected_model_cells of the plaintext
  training, Alg. 4), and to 0 past the cells;
* inference on the activated model (VP, Alg. 7's FM-act branch) sums to the
  bin-activated scores of Alg. 2, and EncryptedArgMax of the sums decrypts
  to Alg. 2's prediction with that activation.
"""
import numpy as np
import pytest

import oracle as O
from oracle import pbs as B
from oracle import plain as P

N, P_MOD, P_OUT = 128, 16, 16
S_BITS, L_CLS, A_BITS, N_TRAIN, T_THR = 8, 2, 2, 10, 2


@pytest.fixture(scope="module")
def model():
    ctx = O.Ctx(N, 1, P_MOD)
    sk = ctx.keygen(5)
    rng = np.random.default_rng(22)  # predictions of both classes and a tie among the test samples
    X = rng.integers(0, 2, (N_TRAIN + 3, S_BITS)).astype(np.uint8)
    y = rng.integers(0, L_CLS, N_TRAIN + 3)
    pi = O.permutation(3, S_BITS)
    xs, ys = {}, {}
    O._parallel(lambda ik: xs.__setitem__(ik, ctx.enc_rgsw(sk, int(X[ik[0]][ik[1]]), 11, ik[0] * S_BITS + ik[1])),
                [(i, k) for i in range(N_TRAIN + 3) for k in range(S_BITS)])
    O._parallel(lambda i: ys.__setitem__(i, ctx.enc_rgsw(sk, int(y[i]), 12, i)), range(N_TRAIN))
    k0 = -(-S_BITS // A_BITS)
    k1 = ctx.k1(S_BITS, L_CLS, A_BITS)
    H = np.zeros((k0, k1, 2, 1, N), np.uint32)
    ctx.train(S_BITS, L_CLS, A_BITS, pi, lambda i, k: xs[(i, k)], lambda i, u: ys[i], N_TRAIN, H)
    W = P.train_integer(X[:N_TRAIN], y[:N_TRAIN], L_CLS, A_BITS, pi)
    bsk = ctx.pbs_keygen(sk, 77, N)
    Kp = ctx.pks_keygen(sk, 9)
    cells = B.fm_cells(N, L_CLS, A_BITS)
    Hf = B.fm_act(ctx, bsk, N, Kp, H, cells, T_THR, P_OUT)
    return dict(ctx=ctx, sk=sk, X=X, pi=pi, xs=xs, H=H, W=W, bsk=bsk, cells=cells, Hf=Hf)


def test_cells_of_the_geometry():
    assert B.fm_cells(128, 2, 2) == 8            # 1 label bit + 2 tuple bits
    assert B.fm_cells(2048, 2, 8) == 512          # Wisconsin-shaped RAM: 2^9 cells in one row
    assert B.fm_cells(2048, 10, 12) == 2048       # MNIST-shaped: 16 index bits, 11 select the coefficient
    assert B.fm_cells(2048, 2, 4, layout=2) == 2048


def test_every_activated_cell_decrypts_to_the_threshold_of_the_plain_cell(model):
    m = model
    ctx, sk = m["ctx"], m["sk"]
    want = P.expected_model_cells(m["W"], S_BITS, L_CLS, A_BITS, N)
    assert want.shape[:2] == m["H"].shape[:2]
    assert want.max() >= T_THR and (want[..., : m["cells"]] < T_THR).any()  # both sides of the threshold occur
    for j in range(want.shape[0]):
        for r in range(want.shape[1]):
            orig = [B.decode(ctx, sk, ctx.extract_lwe(m["H"][j, r], k), P_MOD) for k in range(m["cells"])]
            assert orig == list(want[j, r, : m["cells"]])  # the model FM-act starts from
            got = [B.decode(ctx, sk, ctx.extract_lwe(m["Hf"][j, r], k), P_OUT) for k in range(N)]
            assert got == [int(v >= T_THR) for v in want[j, r]], (j, r)


def test_inference_on_the_activated_model_is_alg2_with_bin(model):
    m = model
    ctx, sk, W, pi = m["ctx"], m["sk"], m["W"], m["pi"]
    k0 = m["H"].shape[0]
    preds = []
    for i in range(N_TRAIN, N_TRAIN + 3):
        sums = []
        for c in range(L_CLS):
            acc = None
            for j in range(k0):
                v = ctx.infer_one(S_BITS, L_CLS, A_BITS, pi, m["Hf"], lambda k: m["xs"][(i, k)], j, c)
                acc = v if acc is None else ctx.lwe_add(acc, v)
            sums.append(acc)
        want_scores = P.activate(P.ram_scores(W, m["X"][i], A_BITS, pi), "bin", T_THR - 1).sum(axis=1)
        assert [B.decode(ctx, sk, u, P_OUT) for u in sums] == list(want_scores), i
        preds.append((sums, P.predict(W, m["X"][i], A_BITS, pi, "bin", T_THR - 1)))
    got = [None] * len(preds)
    O._parallel(lambda t: got.__setitem__(t, B.argmax(ctx, m["bsk"], N, preds[t][0], P_OUT)), range(len(preds)))
    assert [B.decode(ctx, sk, g, 4) for g in got] == [w for _, w in preds]
    assert sorted(set(w for _, w in preds)) == [0, 1]
