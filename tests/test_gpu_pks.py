"""GPU parity of PackingKeySwitching (Sec. 2.5.1; the packed PD-act scores
of Alg. 7): key rows bit-exact with the oracle's (canonical export), packed
RLWE bit-exact with the oracle's packing for ragged k and several groups,
and packed inference scores decrypting to the per-RAM scores."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import dev, host_u32, host_u64, zeros_u32, zeros_u64

pytestmark = pytest.mark.gpu


def _setup(N, nq, p):
    from paper_2403_20190_amd import hwisard as HW
    ctx, orc = HW.Context(N, nq, p), O.Ctx(N, nq, p)
    sk = zeros_u32(N)
    ctx.keygen(21, sk)
    sk_o = orc.keygen(21)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(sk, 99, key)
    return HW, ctx, orc, sk, sk_o, key


@pytest.mark.parametrize("N,nq,p,k,count", [(1024, 1, 64, 1000, 3), (1024, 1, 64, 1024, 1), (1024, 1, 64, 1, 2),
                                             (2048, 2, 1024, 1960, 1)])
def test_key_and_packing_bit_exact(N, nq, p, k, count):
    HW, ctx, orc, sk, sk_o, key = _setup(N, nq, p)
    K_o = orc.pks_keygen(sk_o, 99)
    exp = zeros_u32(ctx.pks_key_words)
    ctx.pks_key_export(key, exp)
    assert np.array_equal(host_u32(exp).reshape(K_o.shape), K_o)
    rng = np.random.default_rng(N + k)
    lwes = np.zeros((count, k, nq, N + 1), np.uint32)
    for g, q in enumerate(orc.primes):
        lwes[:, :, g, :] = rng.integers(0, q, (count, k, N + 1))
    out = zeros_u32(count, 2, nq, N)
    ctx.pack_lwe(key, dev(lwes), k, count, out)
    got = host_u32(out)
    for c in range(count if N == 1024 else 1):
        assert np.array_equal(got[c], orc.pack_lwe(K_o, lwes[c])), c


def test_packed_inference_scores_decrypt_to_ram_scores():
    """Tiny configuration: the l x k0 PD-act scores of each test sample packed
    into one RLWE decrypt to the same cells as the individual LWE scores."""
    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import synth
    from gpu_helpers import Pair
    Xtr, ytr, Xte, _ = synth.tiny(0)
    bits = CL.thermometer(CL.quantize_u8(Xtr, 2), 2)
    pair = Pair(1024, 1, 64, 128, 2, 8, bits, ytr, seed=1)
    ctx = pair.ctx
    H = zeros_u32(pair.k0, pair.k1, 2, 1, 1024)
    ctx.train(pair.shape, pair.encrypt_dev(), pair.encrypt_labels_dev(), pair.n, H, None)
    tb = CL.thermometer(CL.quantize_u8(Xte, 2), 2)
    n = len(tb)
    xr = pair.encrypt_dev(tb, seed_x=55)
    scores = zeros_u32(n, pair.l, pair.k0, ctx.lwe_words)
    ctx.infer(pair.shape, H, xr, n, scores, None)
    key = zeros_u32(ctx.pks_key_words)
    ctx.pks_keygen(pair.sk, 5, key)
    k = pair.l * pair.k0
    packed = zeros_u32(n, 2, 1, 1024)
    ctx.pack_lwe(key, scores, k, n, packed)
    cells = zeros_u64(n * k)
    ctx.decrypt_lwe(pair.sk, scores, n * k, cells)
    dec = zeros_u64(n, 1024)
    ctx.decrypt_rlwe(pair.sk, packed, n, dec)
    d = host_u64(dec)
    assert np.array_equal(d[:, :k], host_u64(cells).reshape(n, k))
    assert not d[:, k:].any()


def test_pack_argument_checks():
    HW, ctx, orc, sk, sk_o, key = _setup(1024, 1, 64)
    lwe = zeros_u32(2, ctx.lwe_words)
    out = zeros_u32(1, 2, 1, 1024)
    with pytest.raises(HW.HwError):
        ctx.pack_lwe(key, lwe, 0, 1, out)
    with pytest.raises(HW.HwError):
        ctx.pack_lwe(key, lwe, 1025, 1, out)
    ctx.pack_lwe(key, lwe, 2, 0, out)  # no groups: nothing happens
