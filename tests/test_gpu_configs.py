"""GPU parity at the parameter sets the benchmark runs: the HAM-shaped class
counter and PackingKeySwitching at N = 4096 with three primes, the serving
engine at the served parameter set (N = 2048, two primes, p = 2^16) with a
Wisconsin-shaped and an MNIST-shaped model, and a batch that mixes N = 2048
and N = 4096 training and inference jobs (hw_batch_run), each against the
oracle, the single-job path and the plaintext Integer WiSARD."""
import numpy as np
import pytest

import oracle as O
from oracle import plain as P
from gpu_helpers import Pair, dev, host_u32, host_u64, label_bits_np, zeros_u32, zeros_u64
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu


def client():
    from paper_2403_20190_amd import client as CL
    return CL


# --------------------------------------------------------------------------
# HAM-shaped balancing counter (Sec. 3.7.1) at N = 4096, three primes
# --------------------------------------------------------------------------

def test_ham_class_counter_bit_exact():
    CL = client()
    Xtr, ytr, _, _ = synth.ham_like(3, n_train=20, n_test=1)
    idx = [0, 11, 19]  # several classes
    bits = CL.thermometer(CL.quantize_u8(Xtr[idx], 2), 2)
    pair = Pair(4096, 3, 16384, 4704, 7, 12, bits, ytr[idx], seed=9)
    # only the counter and one RAM are compared with the oracle; train all RAMs as the benchmark does
    xr = pair.encrypt_dev()
    yr = pair.encrypt_labels_dev()
    H = zeros_u32(pair.k0, pair.k1, 2, 3, 4096)
    cnt = zeros_u32(2, 3, 4096)
    pair.ctx.train(pair.shape, xr, yr, pair.n, H, cnt)
    cnt_o = np.zeros((2, 3, 4096), np.uint32)
    pair.orc.class_count(pair.l, pair.yo, pair.n, cnt_o)
    assert np.array_equal(host_u32(cnt), cnt_o)
    # decrypted counter: coefficient c holds the number of samples of class c
    dec = zeros_u64(1, 4096)
    pair.ctx.decrypt_rlwe(pair.sk, cnt, 1, dec)
    want = np.zeros(4096, np.int64)
    for c in pair.y:
        want[int(c)] += 1
    assert np.array_equal(host_u64(dec)[0].astype(np.int64), want)
    Ho = pair.oracle_train([200])
    assert np.array_equal(host_u32(H)[200], Ho[200])


# --------------------------------------------------------------------------
# PackingKeySwitching at the HAM parameter set
# --------------------------------------------------------------------------

def test_pks_ham_params_bit_exact_and_2744_scores():
    from paper_2403_20190_amd import hwisard as HW
    N, nq, p = 4096, 3, 16384
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(23, sk)
    sk_o = orc.keygen(23)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(sk, 98, key)
    K_o = orc.pks_keygen(sk_o, 98)
    exp = zeros_u32(ctx.pks_key_words)
    ctx.pks_key_export(key, exp)
    assert np.array_equal(host_u32(exp).reshape(K_o.shape), K_o)
    del exp
    # small k against the oracle's packing, bit for bit
    k = 9
    rng = np.random.default_rng(4096 + k)
    lwes = np.zeros((1, k, nq, N + 1), np.uint32)
    for g, q in enumerate(orc.primes):
        lwes[:, :, g, :] = rng.integers(0, q, (1, k, N + 1))
    out = zeros_u32(1, 2, nq, N)
    ctx.pack_lwe(key, dev(lwes), k, 1, out)
    assert np.array_equal(host_u32(out)[0], orc.pack_lwe(K_o, lwes[0]))
    # the HAM-shaped output: 2744 = 7 x 392 LWE scores of one sample in one RLWE.
    # LWE ciphertexts of known messages: ExtractLWE at every index of RLWE encryptions.
    k = 7 * 392
    msg = rng.integers(0, p, (1, N)).astype(np.uint64)
    rl = zeros_u32(1, 2, nq, N)
    ctx.encrypt_rlwe(sk, dev(msg), 1, 31, 0, rl)
    rlh = host_u32(rl)[0]
    lw = np.stack([orc.extract_lwe(rlh, i) for i in range(k)]).reshape(1, k, nq, N + 1)
    packed = zeros_u32(1, 2, nq, N)
    ctx.pack_lwe(key, dev(lw), k, 1, packed)
    dec = zeros_u64(1, N)
    ctx.decrypt_rlwe(sk, packed, 1, dec)
    d = host_u64(dec)[0]
    assert np.array_equal(d[:k], msg[0, :k])
    assert not d[k:].any()


# --------------------------------------------------------------------------
# serving engine at the served parameter set
# --------------------------------------------------------------------------

@pytest.mark.parametrize("gadget", [(6, 5), (15, 2)])
def test_engine_served_params_wisconsin_and_mnist(gadget):
    """with the default RGSW gadget and with 2 digits of 15 bits per prime"""
    import torch
    from paper_2403_20190_amd import hwisard as HW
    CL = client()
    N, nq, p = 2048, 2, 1 << 16
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits_w = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)
    assert np.array_equal(bits_w, P.encode(P.quantize_minmax(Xw, 16, lo, hi), 16))
    Xm, ym, _, _ = synth.mnist_like(1, per_class_train=1, per_class_test=1)
    bits_m = CL.thermometer(CL.quantize_u8(Xm, 3), 3)
    shapes = [dict(bits=bits_w, y=yw, l=2, a=8, seed=71), dict(bits=bits_m, y=ym, l=10, a=12, seed=72)]
    sk = torch.zeros(N, dtype=torch.int32, device="cuda")
    ctx = HW.Context(N, nq, p, log_base=gadget[0], digits=gadget[1])
    ctx.keygen(81, sk)
    eng = HW.Engine(N, nq, p, sk, slots=3, chunk=2, max_s=2352, max_cells=2048, arena_bytes=24 << 30,
                    log_base=gadget[0], digits=gadget[1])
    models, jobs = [], []
    for S in shapes:
        sh = HW.shape(S["bits"].shape[1], S["l"], S["a"], S["seed"])
        k0, k1, _ = ctx.dims(sh)
        H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device="cuda")
        models.append((sh, H, k0, k1))
        jobs.append(eng.add_job(sh, H))
    # (shape, kind, sample indices, enc_seed)
    reqs = [(0, "train", [0, 1, 2, 300, 301], 11), (1, "train", [0, 5, 9], 12), (0, "infer", [3, 302], 13),
            (1, "infer", [7], 14), (0, "train", [4], 15), (1, "infer", [2], 16)]
    rids, cells = [], []
    for shp, kind, idx, seed in reqs:
        S = shapes[shp]
        k0 = models[shp][2]
        c = np.zeros((len(idx), S["l"], k0), np.uint64) if kind == "infer" else None
        rids.append(eng.submit(jobs[shp], kind, S["bits"][idx], seed,
                               labels=CL.label_bits(S["y"][idx], S["l"]) if kind == "train" else None, cells=c))
        cells.append(c)
    for r in rids:
        assert eng.wait(r)[0] == HW.REQ_DONE
    assert eng.stats()["peak_inflight"] >= 2
    eng.close()
    # the direct path on the same ciphertexts, request by request, and Alg. 2 on the decrypted cells
    orc = O.Ctx(N, nq, p, log_base=gadget[0], digits=gadget[1])
    sk_o = orc.keygen(81)
    for shp, S in enumerate(shapes):
        sh, Hm, k0, k1 = models[shp]
        s, l, a = S["bits"].shape[1], S["l"], S["a"]
        L = O.ceil_log2(l)
        pi = O.permutation(S["seed"], s)
        H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device="cuda")
        W = np.zeros((l, k0, 1 << a), np.int64)
        trained = []
        for k, (rs, kind, idx, seed) in enumerate(reqs):
            if rs != shp:
                continue
            sx, sy = O.request_seeds(seed)
            X = S["bits"][idx]
            xr = zeros_u32(len(idx) * s, ctx.rgsw_words)
            ctx.encrypt_rgsw_bits(sk, dev(X.reshape(-1)), sx, 0, xr)
            if kind == "train":
                yr = zeros_u32(len(idx) * L, ctx.rgsw_words)
                ctx.encrypt_rgsw_bits(sk, dev(label_bits_np(S["y"][idx], L).reshape(-1)), sy, 0, yr)
                ctx.train(sh, xr, yr, len(idx), H, None)
                W += P.train_integer(X, S["y"][idx], l, a, pi)
                trained.append((X, S["y"][idx], sx, sy))
            else:
                for i in range(len(idx)):
                    assert np.array_equal(cells[k][i].astype(np.int64), P.ram_scores(W, X[i], a, pi)), (k, i)
        Hg = host_u32(H)
        assert np.array_equal(host_u32(Hm), Hg)
        # one RAM of the engine's model against the oracle, over every training request
        j = k0 - 1
        Ho = np.zeros((k0, k1, 2, nq, N), np.uint32)
        for X, y, sx, sy in trained:
            xo = {}
            yo = {}
            need = [(i, int(pi[j * a + t])) for i in range(len(X)) for t in range(min(a, s - j * a))]
            O._parallel(lambda ik: xo.__setitem__(ik, orc.enc_rgsw(sk_o, int(X[ik[0]][ik[1]]), sx,
                                                                    ik[0] * s + ik[1])), need)
            for i in range(len(X)):
                for u in range(L):
                    yo[(i, u)] = orc.enc_rgsw(sk_o, (int(y[i]) >> u) & 1, sy, i * L + u)
            orc.train(s, l, a, pi, lambda i, kk: xo[(i, kk)], lambda i, u: yo[(i, u)], len(X), Ho, rams=[j])
        assert np.array_equal(Hg[j], Ho[j])


# --------------------------------------------------------------------------
# hw_batch_run: training and inference jobs over two parameter sets
# --------------------------------------------------------------------------

def test_batch_run_mixed_rings_and_kinds():
    from paper_2403_20190_amd import hwisard as HW
    G = (6, 5)
    specs = [  # (N, nq, p, s, l, a, n, layout, counter, RGSW gadget)
        (2048, 2, 1024, 60, 3, 11, 3, 0, True, G),    # z = 2 = L: the tree holds the label bits
        (2048, 2, 1024, 40, 4, 8, 2, 1, False, G),
        (4096, 3, 16384, 50, 7, 12, 2, 0, True, G),   # z = 3 = L, ragged last tuple (2 bits)
        (4096, 3, 16384, 30, 2, 13, 2, 1, False, G),  # class-packed, z = 2 tree levels over tuple bits
        (2048, 2, 1024, 36, 3, 12, 2, 0, True, (15, 2)),  # a third context: 2 digits of 15 bits
    ]
    ctxs = {}
    pairs = []
    for k, (N, nq, p, s, l, a, n, layout, cnt, g) in enumerate(specs):
        X, y = synth.prototype_bits(40 + k, n + 1, s, l, flip=0.2)
        pair = Pair(N, nq, p, s, l, a, X[:n], y[:n], seed=40 + k, layout=layout, gadget=g)
        if (N, nq, g) in ctxs:  # one context and key per parameter set
            first = ctxs[(N, nq, g)]
            pair.ctx, pair.sk, pair.sk_o = first.ctx, first.sk, first.sk_o
        else:
            ctxs[(N, nq, g)] = pair
        pairs.append((pair, cnt, X[n:], g))
    order = list(ctxs)
    cl = [ctxs[k].ctx for k in order]
    jobs, bufs = [], []
    for pair, cnt, Xt, g in pairs:
        ci = order.index((pair.N, pair.nq, g))
        xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C = zeros_u32(2, pair.nq, pair.N) if cnt else None
        xt = pair.encrypt_dev(Xt, seed_x=555)
        sc = zeros_u32(1, pair.l, pair.k0, pair.ctx.lwe_words)
        sums = zeros_u32(1, pair.l, pair.ctx.lwe_words)
        jobs.append(dict(ctx=ci, kind="train", shape=pair.shape, x=xr, y=yr, n=pair.n, model=H, cnt=C))
        # an inference job on the model the same batch trains: it sees that training
        jobs.append(dict(ctx=ci, kind="infer", shape=pair.shape, x=xt, n=1, model=H, scores=sc, sums=sums))
        bufs.append((xr, yr, H, C, xt, sc, sums))
    HW.batch_run(cl, jobs)
    for (pair, cnt, Xt, _), (xr, yr, H, C, xt, sc, sums) in zip(pairs, bufs):
        H1 = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C1 = zeros_u32(2, pair.nq, pair.N) if cnt else None
        pair.ctx.train(pair.shape, xr, yr, pair.n, H1, C1)
        assert np.array_equal(host_u32(H), host_u32(H1))
        if cnt:
            assert np.array_equal(host_u32(C), host_u32(C1))
        sc1 = zeros_u32(1, pair.l, pair.k0, pair.ctx.lwe_words)
        s1 = zeros_u32(1, pair.l, pair.ctx.lwe_words)
        pair.ctx.infer(pair.shape, H1, xt, 1, sc1, s1)
        assert np.array_equal(host_u32(sc), host_u32(sc1))
        assert np.array_equal(host_u32(sums), host_u32(s1))
        # one RAM against the oracle (training and the inference on it)
        j = pair.k0 - 1
        Ho = pair.oracle_train([j])
        assert np.array_equal(host_u32(H)[j], Ho[j])
        got = host_u32(sc).reshape(1, pair.l, pair.k0, pair.nq, pair.N + 1)
        if pair.layout == 0:
            want = pair.orc.infer_one(pair.s, pair.l, pair.a, pair.pi, Ho,
                                      lambda k: pair.xo(0, k, Xt, 555, "t"), j, pair.l - 1)
            assert np.array_equal(got[0, pair.l - 1, j], want)
        else:
            want = pair.orc.infer_packed(pair.s, pair.l, pair.a, pair.pi, Ho,
                                         lambda k: pair.xo(0, k, Xt, 555, "t"), j, pair.layout)
            for c in range(pair.l):
                assert np.array_equal(got[0, c, j], want[c]), c
        # every cell by decryption: Alg. 2 on the plaintext model
        W = P.train_integer(pair.X, pair.y, pair.l, pair.a, pair.pi)
        dec = zeros_u64(pair.l * pair.k0)
        pair.ctx.decrypt_lwe(pair.sk, sc, pair.l * pair.k0, dec)
        cells = host_u64(dec).reshape(pair.l, pair.k0).astype(np.int64)
        assert np.array_equal(cells, P.ram_scores(W, Xt[0], pair.a, pair.pi))


def test_batch_run_inference_pieces_and_layout2():
    """Many samples per inference job (several pieces per item), all three
    layouts, equal to the single-job inference bit for bit."""
    from paper_2403_20190_amd import hwisard as HW
    N, nq, p = 1024, 1, 64
    ctx = HW.Context(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(5, sk)
    jobs, refs = [], []
    for k, (s, l, a, layout, n) in enumerate([(48, 3, 8, 0, 37), (40, 3, 7, 1, 23), (60, 2, 7, 2, 19),
                                              (20, 1, 6, 0, 5), (30, 2, 8, 0, 0)]):
        sh = HW.shape(s, l, a, 60 + k, layout)
        rows, _ = ctx.model_rows(sh)
        k0, k1, _ = ctx.dims(sh)
        # a model with known contents: train a few samples first
        Xtr, ytr = synth.prototype_bits(70 + k, 4, s, l, flip=0.2)
        L = O.ceil_log2(l)
        xr = zeros_u32(4 * s, ctx.rgsw_words)
        ctx.encrypt_rgsw_bits(sk, dev(Xtr.reshape(-1)), 3, 0, xr)
        yr = zeros_u32(max(1, 4 * L), ctx.rgsw_words)
        if L:
            ctx.encrypt_rgsw_bits(sk, dev(label_bits_np(ytr, L).reshape(-1)), 4, 0, yr)
        H = zeros_u32(rows, k1, 2, nq, N)
        ctx.train(sh, xr, yr, 4, H, None)
        X, _ = synth.prototype_bits(80 + k, max(n, 1), s, l, flip=0.3)
        xt = zeros_u32(max(1, n * s), ctx.rgsw_words)
        if n:
            ctx.encrypt_rgsw_bits(sk, dev(X[:n].reshape(-1)), 6 + k, 0, xt)
        sc = zeros_u32(max(1, n), l, k0, ctx.lwe_words)
        jobs.append(dict(kind="infer", shape=sh, x=xt, n=n, model=H, scores=sc))
        refs.append((sh, H, xt, n, sc, l, k0))
    HW.batch_run([ctx], jobs)
    for sh, H, xt, n, sc, l, k0 in refs:
        if n == 0:
            assert not host_u32(sc).any()
            continue
        sc1 = zeros_u32(n, l, k0, ctx.lwe_words)
        ctx.infer(sh, H, xt, n, sc1, None)
        assert np.array_equal(host_u32(sc), host_u32(sc1))


def test_batch_run_argument_checks():
    from paper_2403_20190_amd import hwisard as HW
    ctx = HW.Context(1024, 1, 64)
    sh = HW.shape(16, 2, 8, 1)
    H = zeros_u32(2, 1, 2, 1, 1024)
    x = zeros_u32(16, ctx.rgsw_words)
    sc = zeros_u32(1, 2, 2, ctx.lwe_words)
    with pytest.raises(HW.HwError):  # context index out of range
        HW.batch_run([ctx], [dict(ctx=1, kind="infer", shape=sh, x=x, n=1, model=H, scores=sc)])
    with pytest.raises(HW.HwError):  # inference scores written over a model trained in the batch
        HW.batch_run([ctx], [dict(kind="train", shape=sh, x=x, y=x, n=1, model=H),
                             dict(kind="infer", shape=sh, x=x, n=1, model=H, scores=H)])
    with pytest.raises(HW.HwError):  # two training jobs on one model
        HW.batch_run([ctx], [dict(kind="train", shape=sh, x=x, y=x, n=1, model=H),
                             dict(kind="train", shape=sh, x=x, y=x, n=1, model=H)])
    with pytest.raises(HW.HwError):  # null scores
        HW.batch_run([ctx], [dict(kind="infer", shape=sh, x=x, n=1, model=H, scores=None)])
    assert not host_u32(H).any()
