"""Model merge (Sec. 3.7.2: Integer WiSARD models trained apart are merged by
adding their RAMs) and checkpoint/resume on the GPU: hw_rlwe_add against the
oracle's merge, models trained on two halves and merged equal to training on
the union bit for bit, and training resumed from a checkpoint equal to
training in one go."""
import numpy as np
import pytest

from gpu_helpers import Pair, dev, host_u32, zeros_u32
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2), (4096, 3)])
def test_rlwe_add_matches_oracle(N, nq):
    import oracle as O
    from paper_2403_20190_amd import hwisard as HW
    ctx, orc = HW.Context(N, nq, 64), O.Ctx(N, nq, 64)
    rng = np.random.default_rng(N + nq)
    count = 7
    x = np.stack([np.stack([np.stack([rng.integers(0, q, N) for q in orc.primes]) for _ in range(2)])
                  for _ in range(count)]).astype(np.uint32)
    y = np.stack([np.stack([np.stack([rng.integers(0, q, N) for q in orc.primes]) for _ in range(2)])
                  for _ in range(count)]).astype(np.uint32)
    X, Y = dev(x), dev(y)
    ctx.rlwe_add(X, Y, count)
    assert np.array_equal(host_u32(X), orc.rlwe_add(x, y))
    assert np.array_equal(host_u32(Y), y)
    ctx.rlwe_add(Y, Y, count)  # in place: doubling
    assert np.array_equal(host_u32(Y), orc.rlwe_add(y, y))
    with pytest.raises(HW.HwError):
        ctx.rlwe_add(X[0, 0, 0, 1:], Y, 1)  # not 16-byte aligned


def _pair():
    X, y = synth.prototype_bits(31, 6, 40, 5, flip=0.2)
    return Pair(2048, 2, 64, 40, 5, 12, X, y, seed=31)


def test_merge_of_halves_equals_training_on_all():
    pair = _pair()
    ctx = pair.ctx
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
    C = zeros_u32(2, pair.nq, pair.N)
    ctx.train(pair.shape, xr, yr, pair.n, H, C)
    halves = []
    for lo, hi in ((0, 3), (3, 6)):  # two entities, each with its own samples
        Hh = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        Ch = zeros_u32(2, pair.nq, pair.N)
        ctx.train(pair.shape, xr[lo * pair.s:hi * pair.s], yr[lo * pair.L:hi * pair.L], hi - lo, Hh, Ch)
        halves.append((Hh, Ch))
    (HA, CA), (HB, CB) = halves
    ctx.rlwe_add(HA, HB, pair.k0 * pair.k1)
    ctx.rlwe_add(CA, CB, 1)
    assert np.array_equal(host_u32(HA), host_u32(H))
    assert np.array_equal(host_u32(CA), host_u32(C))
    assert np.array_equal(host_u32(H), pair.oracle_train(range(pair.k0)))


def test_checkpoint_resume(tmp_path):
    from paper_2403_20190_amd import client as CL
    pair = _pair()
    ctx = pair.ctx
    xr, yr = pair.encrypt_dev(), pair.encrypt_labels_dev()
    H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
    ctx.train(pair.shape, xr, yr, pair.n, H, None)
    first = 2
    H1 = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
    ctx.train(pair.shape, xr, yr, first, H1, None)
    path = tmp_path / "ckpt.npz"
    CL.save_checkpoint(path, H1, N=pair.N, nq=pair.nq, s=pair.s, l=pair.l, a=pair.a,
                       perm_seed=pair.seed_perm, trained=first)
    H2, cnt, meta = CL.load_checkpoint(path)
    assert cnt is None and meta["trained"] == first and meta["perm_seed"] == pair.seed_perm
    rest = pair.n - meta["trained"]
    ctx.train(pair.shape, xr[first * pair.s:], yr[first * pair.L:], rest, H2, None)
    assert np.array_equal(host_u32(H2), host_u32(H))
