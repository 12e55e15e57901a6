"""GPU parity of batched training (one persistent launch over many uneven
jobs): every job's model and class counter equal, bit for bit, the per-job
call and the oracle; the cut of RAMs into pieces of samples does not change
any bit; captured batch plans replay the same result."""
import os

import numpy as np
import pytest

import oracle as O
from gpu_helpers import Pair, dev, host_u32, zeros_u32
from paper_2403_20190_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [  # (s, l, a, n, counter)
    (40, 4, 10, 3, True),
    (23, 3, 11, 2, False),   # ragged last tuple, encrypted tree level (z = 3 > L = 2)
    (64, 2, 8, 4, True),
    (17, 1, 6, 2, False),    # l = 1: no label bits
    (30, 5, 7, 0, False),    # empty job
    (96, 10, 12, 1, True),   # z = 6
]


def make_jobs(ctx_args, seed0=20):
    pairs = []
    for k, (s, l, a, n, cnt) in enumerate(SHAPES):
        X, y = synth.prototype_bits(seed0 + k, max(n, 1), s, l, flip=0.2)
        pairs.append((Pair(X=X[:n], y=y[:n], s=s, l=l, a=a, seed=seed0 + k, **ctx_args), cnt))
    return pairs


def run_batch(ctx, pairs):
    bufs = []
    jobs = []
    for pair, cnt in pairs:
        xr = pair.encrypt_dev() if pair.n else zeros_u32(1, ctx.rgsw_words)
        yr = pair.encrypt_labels_dev() if pair.n else None
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C = zeros_u32(2, pair.nq, pair.N) if cnt else None
        bufs.append((xr, yr, H, C))
        jobs.append((pair.shape, xr, yr, pair.n, H, C))
    ctx.batch_train(jobs)
    return bufs


def test_batch_equals_single_job_and_oracle():
    pairs = make_jobs(dict(N=1024, nq=2, p=64))
    # every Pair made its own context with the same parameters; use the first for the batch
    ctx = pairs[0][0].ctx
    for pair, _ in pairs:
        pair.ctx, pair.sk = ctx, pairs[0][0].sk  # one key for all jobs of the batch
        pair.sk_o = pairs[0][0].sk_o
    bufs = run_batch(ctx, pairs)
    for (pair, cnt), (xr, yr, H, C) in zip(pairs, bufs):
        if pair.n == 0:
            assert not host_u32(H).any()
            continue
        H1 = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        C1 = zeros_u32(2, pair.nq, pair.N) if cnt else None
        ctx.train(pair.shape, xr, yr, pair.n, H1, C1)
        assert np.array_equal(host_u32(H), host_u32(H1)), pair.s
        if cnt:
            assert np.array_equal(host_u32(C), host_u32(C1))
    # one job against the oracle directly
    pair, _ = pairs[1]
    Ho = pair.oracle_train(range(pair.k0))
    assert np.array_equal(host_u32(bufs[1][2]), Ho)


def test_batch_pieces_do_not_change_bits():
    """A workspace budget of one byte forces one piece per RAM (every model
    row accumulated in place, no reduction); the default budget cuts these
    small jobs into one-sample pieces.  Same bits either way."""
    pairs = make_jobs(dict(N=2048, nq=2, p=1024), seed0=40)
    ctx = pairs[0][0].ctx
    for pair, _ in pairs:
        pair.ctx, pair.sk, pair.sk_o = ctx, pairs[0][0].sk, pairs[0][0].sk_o
    big = run_batch(ctx, pairs)
    os.environ["HWISARD_WS_BYTES"] = "1"
    try:
        from paper_2403_20190_amd import hwisard as HW
        small = HW.Context(2048, 2, 1024)
    finally:
        del os.environ["HWISARD_WS_BYTES"]
    jobs = [(pair.shape, b[0], b[1], pair.n, zeros_u32(pair.k0, pair.k1, 2, 2, 2048),
             zeros_u32(2, 2, 2048) if cnt else None) for (pair, cnt), b in zip(pairs, big)]
    small.batch_train(jobs)
    for (pair, cnt), b, j in zip(pairs, big, jobs):
        assert np.array_equal(host_u32(b[2]), host_u32(j[4]))
        if cnt:
            assert np.array_equal(host_u32(b[3]), host_u32(j[5]))


def test_batch_argument_checks():
    from paper_2403_20190_amd import hwisard as HW
    ctx = HW.Context(1024, 1, 64)
    H = zeros_u32(4, 1, 2, 1, 1024)
    x = zeros_u32(32, ctx.rgsw_words)
    sh = HW.shape(32, 2, 8, 1)
    with pytest.raises(HW.HwError):  # two jobs writing one model
        ctx.batch_train([(sh, x, x, 1, H, None), (sh, x, x, 1, H, None)])
    with pytest.raises(HW.HwError):
        ctx.batch_train([(HW.shape(32, 2, 0, 1), x, x, 1, H, None)])
    before = host_u32(H).copy()
    ctx.batch_train([])
    assert np.array_equal(host_u32(H), before)


def _fresh_outputs(pairs, bufs):
    return [(pair.shape, b[0], b[1], pair.n, zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N),
             zeros_u32(2, pair.nq, pair.N) if cnt else None) for (pair, cnt), b in zip(pairs, bufs)]


def _same(jobs, ref):
    for j, r in zip(jobs, ref):
        if not np.array_equal(host_u32(j[4]), host_u32(r[4])):
            return False
        if j[5] is not None and not np.array_equal(host_u32(j[5]), host_u32(r[5])):
            return False
    return True


@pytest.mark.parametrize("ws_bytes", [None, "1"])
def test_batch_plan_replays_match_eager(ws_bytes):
    """A batch plan (queue computed once, launches captured into a HIP graph)
    replayed three times, with eager work and synchronisations between the
    replays, equals the eager batched call every time; a replay without
    clearing the models adds the batch again; replays read the inputs as they
    are at replay time.  ws_bytes="1" forces one piece per RAM."""
    import torch
    from paper_2403_20190_amd import hwisard as HW
    if ws_bytes:
        os.environ["HWISARD_WS_BYTES"] = ws_bytes
    try:
        ctx = HW.Context(1024, 2, 64)
    finally:
        os.environ.pop("HWISARD_WS_BYTES", None)
    pairs = make_jobs(dict(N=1024, nq=2, p=64), seed0=60)
    for pair, _ in pairs:
        pair.ctx, pair.sk, pair.sk_o = ctx, pairs[0][0].sk, pairs[0][0].sk_o
    bufs = run_batch(ctx, pairs)
    ref = [(None, None, None, None, b[2], b[3]) for b in bufs]
    jobs = _fresh_outputs(pairs, bufs)
    plan = ctx.batch_plan(jobs)
    info = (plan.max_pieces, plan.items, plan.workspace_bytes)
    assert (plan.max_pieces == 1) if ws_bytes else (plan.max_pieces > 1), info
    assert plan.items > 0 and plan.external_products > 0
    for rep in range(3):
        for j in jobs:
            j[4].zero_()
            if j[5] is not None:
                j[5].zero_()
        plan.launch()
        torch.cuda.synchronize()
        assert _same(jobs, ref), rep
        # unrelated eager work on the same context between replays
        pair = pairs[2][0]
        H = zeros_u32(pair.k0, pair.k1, 2, pair.nq, pair.N)
        ctx.train(pair.shape, bufs[2][0], bufs[2][1], pair.n, H, None)
        torch.cuda.synchronize()
    # a second replay on top of the first adds the batch again (mod q)
    plan.launch()
    torch.cuda.synchronize()
    primes = pairs[0][0].orc.primes
    for j, r in zip(jobs, ref):
        twice = host_u32(r[4]).astype(np.uint64) * 2
        for i, q in enumerate(primes):
            twice[:, :, :, i, :] %= q
        assert np.array_equal(host_u32(j[4]), twice.astype(np.uint32))
    # new input bits encrypted into job 0's buffer: the replay sees them
    pair = pairs[0][0]
    X2, _ = synth.prototype_bits(99, pair.n, pair.s, pair.l, flip=0.3)
    ctx.encrypt_rgsw_bits(pair.sk, dev(np.ascontiguousarray(X2, np.uint8).reshape(-1)), pair.seed_x + 5, 0,
                          bufs[0][0])
    for j in jobs:
        j[4].zero_()
        if j[5] is not None:
            j[5].zero_()
    plan.launch()
    eager = _fresh_outputs(pairs, bufs)
    ctx.batch_train(eager)
    torch.cuda.synchronize()
    assert _same(jobs, eager)
    assert not np.array_equal(host_u32(jobs[0][4]), host_u32(ref[0][4]))
    plan.close()
