#!/usr/bin/env python3
"""Benchmark of the encrypted WiSARD hot path on one MI355X.

Workload (default): MNIST-shaped synthetic data -- 28x28 uint8 images, 10
balanced classes, 3-level thermometer code (s = 2352 bits), tuple size 12
(196 RAMs), 1000 training + 1000 test samples, RLWE N = 2048 with two 30-bit
primes, plaintext modulus 1024.  `--workload ham`, `wisconsin` and `tiny`
select the other shapes (see WORKLOADS).

A step is one encrypted training pass over the 1000 training samples: the
client-side RGSW encryption of every input and label bit (on the device, from
thermometer bits resident in HBM) followed by homomorphic training (Alg. 6)
into a zeroed model, chunk by chunk.  `value` = training samples per second of
that whole step.  After the timed steps the same run measures, untimed by the
step clock: kernel-level times (HIP events on the launch stream), encrypted
inference of the 1000 test samples with PD-act decoding, a batched NTT, the
oracle on the host cores (cpu_baseline) and the roofline of the dominant
kernel.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fractions
PEAK_HBM_GBS = 8000.0
CU, LANES, CLOCK_GHZ = 256, 64, 2.4
PEAK_INT32_TOPS = CU * LANES * CLOCK_GHZ / 1000.0  # 39.32 T 32-bit lane ops/s

WORKLOADS = {
    "mnist": dict(name="mnist-shaped 28x28x1, 10 classes, therm 3, tuple 12, 1000 train + 1000 test, N=2048 x 2 primes",
                  N=2048, nq=2, p=1024, l=10, a=12, T=3, n_train=1000, n_test=1000, chunk=50, balance=False),
    "ham": dict(name="ham10000-shaped 28x28x3, 7 skewed classes, therm 2, tuple 12, 10000 train + 1000 test, N=4096 x 3 primes",
                N=4096, nq=3, p=16384, l=7, a=12, T=2, n_train=10000, n_test=1000, chunk=10, balance=True, cpu_rams=49),
    "wisconsin": dict(name="wisconsin-shaped 30 float features, 2 classes 357/212, therm 16 (480 bits), tuple 8, "
                           "400 train + 169 test, N=2048 x 2 primes",
                      N=2048, nq=2, p=512, l=2, a=8, T=16, n_train=400, n_test=169, chunk=100, balance=False,
                      cpu_samples=12, otf=16, fm=4, act=("log", 0), boot_n=1024),
    "tiny": dict(name="tiny 8x8, 2 classes, therm 2, tuple 8, 32 train + 16 test, N=1024 x 1 prime",
                 N=1024, nq=1, p=64, l=2, a=8, T=2, n_train=32, n_test=16, chunk=32, balance=False),
}


KERNEL_SOURCES = ["hw_device.h", "hw_kernels.hip", "hw_internal.h"]


def kernel_code_sha256() -> str:
    """sha256 of the training kernel's sources (KERNEL_SOURCES, in that
    order) with comments removed and whitespace runs collapsed: it changes
    when their code does, not when a comment does"""
    import hashlib
    import re
    sha = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2403_20190_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        sha.update(" ".join(text.split()).encode())
        sha.update(b"\0")
    return sha.hexdigest()


def measured_traffic(schedule: str | None):
    """HBM bytes (read + write) per training call (k_train, plus the
    k_train_level launches when the tree levels are staged) measured with
    rocprofv3 FETCH_SIZE / WRITE_SIZE (profiles/k_train_mnist_pmc.md) for the
    schedule in use, or None when the kernel code changed since
    (kernel_code_sha256 no longer matches)."""
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", "k_train_mnist_pmc.md")).read()
    except OSError:
        return None
    kind = "staged" if schedule and "staged" in schedule else "fused"
    t = re.search(r"traffic_bytes_per_launch_%s:\s*(\d+)" % kind, text)
    h = re.search(r"kernel_code_sha256:\s*([0-9a-f]{64})", text)
    if not t or not h:
        return None
    return int(t.group(1)) if kernel_code_sha256() == h.group(1) else None


class Progress:
    """A line on stderr about every 20 s of a long loop.  The loops enqueue
    work asynchronously, so a line first waits for the device (a few ms of
    idle time per line)."""

    def __init__(self, what: str, total: int, every: float = 20.0):
        self.what, self.total, self.every = what, total, every
        self.last = time.perf_counter()

    def __call__(self, done: int):
        now = time.perf_counter()
        if now - self.last >= self.every:
            import torch
            torch.cuda.synchronize()
            print("bench: %s %d / %d" % (self.what, done, self.total), file=sys.stderr, flush=True)
            self.last = time.perf_counter()


def ops_per_xp(N: int, nq: int) -> float:
    """Algorithmic 32-bit integer operations of one external product.

    Model: a forward (Cooley-Tukey, Harvey lazy) butterfly = 9 ops (Shoup
    product 4, lazy correction 2, add 1, sub 2); an inverse (Gentleman-Sande)
    butterfly = 9 ops; the 1/N scaling 6 ops per coefficient; a
    multiply-accumulate term = 2 ops (32x32->64 product, 64-bit add); a
    balanced digit = 6 ops (extract 3, lift 2, shift 1).  Per product: 10 nq^2
    forward and 2 nq inverse NTTs of (N/2) log2 N butterflies, 20 nq^2 N MAC
    terms, 10 nq^2 N digit coefficients."""
    logN = N.bit_length() - 1
    bf = (N // 2) * logN
    return (9.0 * bf * (10 * nq * nq + 2 * nq) + 6.0 * N * 2 * nq + 2.0 * 20 * nq * nq * N
            + 6.0 * 10 * nq * nq * N)


def ops_first_xp(N: int, nq: int) -> float:
    """Algorithmic ops of the first external product of an IVP chain, whose
    input (0, Delta (X - 1)) has a zero a side and two-coefficient digit
    polynomials: no forward NTT; per output prime and side, 5 nq gadget rows
    x N coefficients x two multiply-accumulates (2 ops each), 15 ops of
    reduction and the evaluation product per coefficient; 2 nq inverse
    NTTs."""
    logN = N.bit_length() - 1
    return (9.0 * (N // 2) * logN + 6.0 * N) * 2 * nq + 4.0 * 5 * nq * nq * 2 * N + 15.0 * 2 * nq * N


def train_ops(N: int, nq: int, xp: float, ivps: float) -> float:
    """ops of a training launch with `xp` external products over `ivps` IVP
    chains (each chain's first product is the cheaper one above)"""
    return (xp - ivps) * ops_per_xp(N, nq) + ivps * ops_first_xp(N, nq)


def ops_per_enc_row(N: int, nq: int) -> float:
    """Algorithmic int32 ops of one RGSW row (an RLWE encryption of 0 plus the
    gadget term), drawn as k_enc_rgsw draws it: Philox4x32-10 blocks for the
    uniform a (nq N / 4: one 32-bit word per residue; the rare rejected word's
    fallback draw is not counted) and for the Gaussian e (N / 2, one 64-bit
    word per sample), 80 ops a block (10 rounds of two 32x32->64 products at
    2 ops and 4 XORs; the key schedule is scalar); 6 ops to reduce a word mod
    q and test it; 12 per CDT sample (the guide lookup, two steps of a
    64-bit compare and a select, the sign; the six-step search of the top
    bucket, 2.4e-4 of the draws, is not counted); the forward NTT of e under each prime
    (9 ops a butterfly); 16 per coefficient and prime for the lift of e and
    b = a s + e + gadget (a Shoup product with the transformed key)."""
    logN = N.bit_length() - 1
    return (80.0 * (nq * N / 4 + N / 2) + 6.0 * nq * N + 12.0 * N + 9.0 * nq * (N // 2) * logN
            + 16.0 * nq * N)


def modmul_per_xp(N: int, nq: int, dig: int = 5) -> float:
    """Modular multiplications of one external product:
    (2 l nq^2 + 2 nq) (N/2) log2 N + 4 l nq^2 N with l = dig digits per prime."""
    logN = N.bit_length() - 1
    return (2 * dig * nq * nq + 2 * nq) * (N // 2) * logN + 4 * dig * nq * nq * N


def rgsw_bytes(N: int, nq: int, dig: int = 5) -> int:
    """2D rows (D = dig nq) x 2 polynomials x nq residues x N words"""
    return 2 * dig * nq * 2 * nq * N * 4


def device_peaks(dev) -> dict:
    """The device's peak rates measured on this GPU (hw_microbench): a stream
    triad over three 1 GiB arrays (GB/s) and the lane-instruction rate of the
    32-bit VALU instructions of the modular arithmetic (T/s)."""
    from paper_2403_20190_amd import hwisard as HW
    out = {"triad_gbs": round(HW.microbench("triad", 1 << 30, dev.index or 0)[0] / 1e9, 1)}
    for k in ("v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32"):
        out[k + "_tops"] = round(HW.microbench(k, 0, dev.index or 0)[0] / 1e12, 2)
    return out


# A modular multiplication by a precomputed operand (Shoup) issues three
# 32-bit multiplies: mul_hi for the quotient estimate, mul_lo for the product
# and one multiply-add (v_mad_u64_u32) with the modulus.
MUL_PER_MODMUL = 3


def xp_roofline(kernel: str, N: int, nq: int, xp: float, ms: float, launches: int, peaks: dict | None,
                ops: float | None = None, dig: int = 5) -> dict:
    """Roofline of a kernel made of external products, in per-product units:
    each product streams one RGSW ciphertext (16 l nq^2 N bytes, l = dig
    digits per prime, 5 unless stated) and performs (2 l nq^2 + 2 nq)(N/2) log2 N + 4 l nq^2 N modular
    multiplications.  `achieved` = those bytes / time against HBM and those
    multiplies (MUL_PER_MODMUL int32 multiplies each) / time against the
    VALU; `bound` is the resource with the larger fraction.  `ops` (the
    builder's op model of the instructions, optional) is reported beside."""
    if not ms or not launches:
        return {"kernel": kernel, "bound": None}
    sec = ms / 1000.0
    per_launch = xp / launches
    gbs = xp * rgsw_bytes(N, nq, dig) / sec / 1e9
    mm_s = xp * modmul_per_xp(N, nq, dig) / sec
    mul_t = mm_s * MUL_PER_MODMUL / 1e12
    hbm = {"achieved_gbs": round(gbs, 1), "peak_gbs": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4)}
    valu = {"modmul_per_s": round(mm_s, 1), "int32_mul_per_modmul": MUL_PER_MODMUL,
            "achieved_tops": round(mul_t, 3), "peak_tops": round(PEAK_INT32_TOPS, 2),
            "frac": round(mul_t / PEAK_INT32_TOPS, 4)}
    if peaks:
        hbm["measured_peak_gbs"] = peaks["triad_gbs"]
        hbm["frac_of_measured"] = round(gbs / peaks["triad_gbs"], 4)
        mp = min(peaks["v_mul_lo_u32_tops"], peaks["v_mul_hi_u32_tops"])
        valu["measured_peak_tops"] = mp
        valu["frac_of_measured"] = round(mul_t / mp, 4)
    bound = "hbm" if hbm["frac"] >= valu["frac"] else "alu"
    r = {"bound": bound, "kernel": kernel}
    if bound == "hbm":
        r.update(achieved=hbm["achieved_gbs"], peak=PEAK_HBM_GBS, unit="GB/s", frac=hbm["frac"])
    else:
        r.update(achieved=valu["achieved_tops"], peak=round(PEAK_INT32_TOPS, 2), unit="TOPS(int32 mul)",
                 frac=valu["frac"])
    r.update(unit_of_work="external product", bytes_per_unit=rgsw_bytes(N, nq, dig),
             modmul_per_unit=modmul_per_xp(N, nq, dig), units_per_launch=per_launch, launches=launches,
             avg_launch_ms=round(ms / launches, 3), hbm=hbm, valu=valu)
    if ops is not None:
        r["op_model"] = {"int32_ops_per_launch": ops / launches, "achieved_tops": round(ops / sec / 1e12, 3),
                         "frac": round(ops / sec / 1e12 / PEAK_INT32_TOPS, 4)}
    return r


def gen_data(wl: str, W: dict):
    from paper_2403_20190_amd import synth
    if wl == "wisconsin":
        X, y = synth.wisconsin_like(4)
        n = W["n_train"]
        return X[:n], y[:n], X[n:], y[n:]
    if wl == "mnist":
        return synth.mnist_like(1, per_class_train=W["n_train"] // 10, per_class_test=W["n_test"] // 10)
    if wl == "ham":
        return synth.ham_like(3, n_train=W["n_train"], n_test=W["n_test"])
    return synth.tiny(0, W["n_train"], W["n_test"])


def levels_of(mod, W: dict, X, ref):
    """quantisation levels of X with `mod`'s quantiser (the client's or the
    oracle's plain one): uint8 images by value, float features by min-max
    over the reference data"""
    if W.get("minmax"):
        return mod.quantize_minmax(X, W["T"], ref.min(axis=0), ref.max(axis=0))
    return mod.quantize_u8(X, W["T"])


def host_info():
    """host cores the oracle may use and the CPU model"""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity": affinity, "cpu_model": model}


# The paper's own CPU timings of encrypted training and evaluation (Table 7,
# desktop i7-12700K at 5.0 GHz with AVX-512, TFHE torus parameters with one or
# two digits), quoted as context: other parameters, other hardware.
PAPER_CPU_CONTEXT = {
    "mnist": "MNIST_T (1000 train samples, a = 12): training 12m16s on 1 thread, 1m33s on 8 threads "
             "(10.8 samples/s); evaluation of the test set 2h11m / 19m40s (paper Table 7, i7-12700K)",
    "ham": "HAM10000_S (1002 train samples, a = 12): training 54m13s on 1 thread, 6m50s on 8 threads "
           "(paper Table 7, i7-12700K)",
    "wisconsin": "Wisconsin (about 455 train samples, a = 10): training 11 s on 1 thread, 1436 ms on 8 threads "
                 "(paper Table 7, i7-12700K)",
    "tiny": None,
}


def cpu_baseline(wl: str, W: dict, Xtr, ytr, Xte, seeds: dict, ctx, sh, sk_dev, dev, ref=None):
    """The oracle, as it is, on a bounded sample of the workload, timed on the
    host's cores (at most 16 threads: the host share of one GPU), and checked
    bit for bit against the GPU on the same sample:

    * all threads: client encryption of the first m training samples and IVP
      training of them over every RAM (`cpu_rams` RAMs when set) -> samples/s;
      the oracle's model is compared with the GPU's model of the same samples;
    * one thread: the same for one sample over 4 RAMs (the RGSW those RAMs
      read), extrapolated linearly to all input bits and RAMs -> samples/s;
    * all threads: inference of the first test sample on the m-sample model
      over 8 RAMs x every label, extrapolated to all RAMs; the LWE scores are
      compared with the GPU's scores of the same sample."""
    import numpy as np
    import torch

    import oracle as O
    from oracle import plain as P
    from paper_2403_20190_amd import client as CL
    N, nq, p, l, a, T = W["N"], W["nq"], W["p"], W["l"], W["a"], W["T"]
    m = W.get("cpu_samples", 1)
    info = host_info()
    threads = max(1, min(16, info["affinity"]))
    orc = O.Ctx(N, nq, p, log_base=ctx.log_base, digits=ctx.digits)  # the gadget of the GPU run it checks
    bits = P.encode(levels_of(P, W, Xtr[:m], ref), T)
    tbits = P.encode(levels_of(P, W, Xte[:1], ref), T)
    s = bits.shape[1]
    L = O.ceil_log2(l)
    sk = orc.keygen(seeds["key"])
    pi = O.permutation(seeds["perm"], s)
    k0, k1 = -(-s // a), orc.k1(s, l, a)
    rams = list(range(min(k0, W.get("cpu_rams") or k0)))

    def tuple_bits(js):
        return sorted({int(pi[j * a + u]) for j in js for u in range(min(a, s - j * a))})

    # --- all threads: encryption + training of m samples ---------------------------
    t0 = time.perf_counter()
    xr, yr = {}, {}
    need = tuple_bits(rams)
    O._parallel(lambda ik: xr.__setitem__(ik, orc.enc_rgsw(sk, int(bits[ik[0], ik[1]]), seeds["x"],
                                                                 ik[0] * s + ik[1])),
                [(i, k) for i in range(m) for k in need], threads)
    O._parallel(lambda iu: yr.__setitem__(iu, orc.enc_rgsw(sk, (int(ytr[iu[0]]) >> iu[1]) & 1, seeds["y"],
                                                                 iu[0] * L + iu[1])),
                [(i, u) for i in range(m) for u in range(L)], threads)
    t_enc_all = time.perf_counter() - t0
    H = np.zeros((k0, k1, 2, nq, N), np.uint32)
    t0 = time.perf_counter()
    orc.train(s, l, a, pi, lambda i, k: xr[(i, k)], lambda i, u: yr[(i, u)], m, H, rams=rams, threads=threads)
    t_tr_all = time.perf_counter() - t0
    dt_all = t_enc_all + t_tr_all
    # seconds per sample over every input bit and RAM (linear in both)
    per_sample_all = (t_enc_all * (s + L) / (len(need) + L) + t_tr_all * k0 / len(rams)) / m
    # --- one thread: one sample, 4 RAMs, extrapolated ----------------------------------
    r1 = rams[:4]
    need1 = tuple_bits(r1)
    t0 = time.perf_counter()
    x1 = {k: orc.enc_rgsw(sk, int(bits[0, k]), seeds["x"], k) for k in need1}
    y1 = {u: orc.enc_rgsw(sk, (int(ytr[0]) >> u) & 1, seeds["y"], u) for u in range(L)}
    t_enc1 = time.perf_counter() - t0
    H1 = np.zeros((k0, k1, 2, nq, N), np.uint32)
    t0 = time.perf_counter()
    orc.train(s, l, a, pi, lambda i, k: x1[k], lambda i, u: y1[u], 1, H1, rams=r1, threads=1)
    t_tr1 = time.perf_counter() - t0
    sec_1thr = t_enc1 * (s + L) / (len(need1) + L) + t_tr1 * k0 / len(r1)
    # --- all threads: inference of one test sample, 8 RAMs x every label ---------------
    ri = rams[:8]
    needi = tuple_bits(ri)
    t0 = time.perf_counter()
    xt = {}
    O._parallel(lambda k: xt.__setitem__(k, orc.enc_rgsw(sk, int(tbits[0, k]), seeds["xt"], k)), needi, threads)
    t_enci = time.perf_counter() - t0
    out_o = {}
    t0 = time.perf_counter()
    O._parallel(lambda jc: out_o.__setitem__(jc, orc.infer_one(s, l, a, pi, H, lambda k: xt[k], jc[0], jc[1])),
                [(j, c) for j in ri for c in range(l)], threads)
    t_inf = time.perf_counter() - t0
    sec_inf = t_enci * s / len(needi) + t_inf * k0 / len(ri)
    # --- the GPU on the same samples ----------------------------------------------------
    xb = torch.from_numpy(CL.thermometer(levels_of(CL, W, Xtr[:m], ref), T)).to(dev)
    yb = torch.from_numpy(CL.label_bits(ytr[:m], l)).to(dev)
    gx = torch.empty(m * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    gy = torch.empty(max(1, m * L), ctx.rgsw_words, dtype=torch.int32, device=dev)
    ctx.encrypt_rgsw_bits(sk_dev, xb.reshape(-1), seeds["x"], 0, gx)
    if L:
        ctx.encrypt_rgsw_bits(sk_dev, yb.reshape(-1), seeds["y"], 0, gy)
    Hg = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev)
    ctx.train(sh, gx, gy, m, Hg, None)
    del gx, gy
    tx = torch.from_numpy(CL.thermometer(levels_of(CL, W, Xte[:1], ref), T)).to(dev)
    gt = torch.empty(s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    ctx.encrypt_rgsw_bits(sk_dev, tx.reshape(-1), seeds["xt"], 0, gt)
    sc = torch.empty(1, l, k0, ctx.lwe_words, dtype=torch.int32, device=dev)
    ctx.infer(sh, Hg, gt, 1, sc, None)
    torch.cuda.synchronize()
    Hh = Hg.cpu().numpy().view(np.uint32)
    sch = sc.cpu().numpy().view(np.uint32).reshape(l, k0, nq, N + 1)
    del Hg, gt, sc
    train_equal = bool(np.array_equal(Hh[rams], H[rams]))
    infer_equal = all(np.array_equal(sch[c, j], out_o[(j, c)]) for j in ri for c in range(l))
    return dict(
        value=round(1.0 / per_sample_all, 5), unit="samples/s", cores=threads, kind="oracle",
        sample="%d training sample(s): oracle encryption of the RGSW of %d input bits + %d label bits and IVP "
               "training of %d of %d RAMs, %.1f s on %d threads%s" % (
                   m, len(need), L, len(rams), k0, dt_all, threads,
                   "" if len(rams) == k0 else " (extrapolated to all RAMs)"),
        one_thread_samples_per_s=round(1.0 / sec_1thr, 6),
        one_thread_sample="1 sample, RGSW of %d input bits + %d label bits, 4 RAMs: %.1f s encryption + %.1f s "
                          "training on 1 thread, extrapolated to %d bits and %d RAMs" % (
                              len(need1), L, t_enc1, t_tr1, s + L, k0),
        infer_samples_per_s=round(1.0 / sec_inf, 5),
        infer_sample="1 test sample, %d RAMs x %d labels: %.1f s encryption + %.1f s VP on %d threads, "
                     "extrapolated to %d RAMs" % (len(ri), l, t_enci, t_inf, threads, k0),
        bit_exact={"train_model_rams": train_equal, "infer_scores": infer_equal},
        host=info, paper_context=PAPER_CPU_CONTEXT.get(wl))


def side_workload(args):
    """--workload batched / served: one JSON line"""
    import torch
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    if args.workload == "batched":
        r = batched_full(dev, args.batched_ring, args.batched_window_gib, args.batched_per_job, args.batched_jobs,
                         oracle_rams=0 if args.no_cpu_baseline else args.batched_oracle_rams)
        line = {"metric": "batched encrypted train samples/s (training kernels)", "value": r["batched_samples_per_s"],
                "unit": "samples/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u32", "data": "synthetic",
                "config": {"workload": "256 uneven training jobs (n U{32..2000}, s U{128..2352}, a U{8..12}, "
                                       "l U{2..10}), ring %d" % args.batched_ring}, "batched": r}
    else:
        r = served_full(dev, args.served_requests, args.served_max_size, args.served_loads or [],
                        args.served_sat_rps, args.served_one_at_a_time, tuple(args.served_orders),
                        gadget=(6, 5) if args.gadget == "6x5" else (15, 2))
        line = {"metric": "served p50/p99 latency and throughput", "unit": "ms", "n_gpus": 1, "dtype": "u32",
                "data": "synthetic", "config": {"workload": "Poisson train/infer requests, half Wisconsin- half "
                                                            "MNIST-shaped, N=2048 x 2 primes, p=2^16"}, "served": r}
    line["wall_s"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mnist", choices=sorted(WORKLOADS) + ["batched", "served"],
                    help="batched / served: the batched and served configurations at their stated sizes "
                         "(separate runs, one JSON line each; see --batched-* / --served-*)")
    ap.add_argument("--batched-ring", type=int, default=2048, choices=[2048, 4096])
    ap.add_argument("--batched-jobs", type=int, nargs=2, default=None, metavar=("FIRST", "END"),
                    help="only jobs [FIRST, END) of the ring's jobs")
    ap.add_argument("--batched-window-gib", type=float, default=160.0)
    ap.add_argument("--batched-per-job", type=int, default=2, help="samples per job per window")
    ap.add_argument("--batched-oracle-rams", type=int, default=16,
                    help="RAMs of the smallest job that the oracle trains over all its samples")
    ap.add_argument("--served-loads", type=float, nargs="*", default=None,
                    help="loads (fractions of the saturated request rate) for --workload served")
    ap.add_argument("--served-sat-rps", type=float, default=None,
                    help="saturated request rate from an earlier run (skips the saturated run)")
    ap.add_argument("--served-orders", nargs="+", default=["fifo"], choices=["fifo", "shortest"],
                    help="engine orders to run each load with (the saturated run uses the first)")
    ap.add_argument("--served-one-at-a-time", action="store_true",
                    help="also replay the requests one job at a time")
    ap.add_argument("--n-train", type=int, default=None, help="override the number of training samples")
    ap.add_argument("--chunk", type=int, default=None, help="samples encrypted and trained per call")
    ap.add_argument("--no-extras", action="store_true", help="only the timed steps (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--overlap", action="store_true",
                    help="encrypt chunk k+1 on a second stream while chunk k trains (default: one stream; "
                         "measured slower, as either kernel alone keeps the GPU busy)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the device peak probes")
    ap.add_argument("--force", action="append", default=[], metavar="KERNEL=VARIANT",
                    help="force a schedule variant of a tuned kernel (hw_tune_set), e.g. train=3")
    ap.add_argument("--calib-copy", type=int, default=0, help="also run a plain device copy of this many MiB")
    ap.add_argument("--batched-scale", type=float, nargs="*", default=[1.0 / 64, 1.0 / 512],
                    help="job sizes of the 256-job batched workload are scaled by these factors")
    ap.add_argument("--fm-full", action="store_true",
                    help="wisconsin: FM-act of the whole model, then inference on it (minutes)")
    ap.add_argument("--gadget", default="6x5", choices=["6x5", "15x2"],
                    help="RGSW gadget of the timed step (or of the served engine with --workload served): 5 "
                         "digits of 6 bits per prime (default) or 2 of 15 bits (rings of two or more primes); "
                         "the extras then skip the gadget leg")
    ap.add_argument("--no-gadget-leg", action="store_true",
                    help="skip the step and inference with RGSW of 2 digits of 15 bits per prime")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--served-max-size", type=int, default=50,
                    help="request sizes are U{1..max}; the served workload's 1..500 scaled down")
    ap.add_argument("--served-load", type=float, default=0.7, help="offered load as a fraction of saturation")
    args = ap.parse_args()
    if args.workload in ("batched", "served"):
        if args.gpus != 1:
            print("bench.py: one GPU only.", file=sys.stderr)
            sys.exit(2)
        return side_workload(args)
    if args.gpus != 1:
        print("bench.py: one GPU only; the path shards by sample or by RAM across GPUs, which is not run here. "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW

    W = dict(WORKLOADS[args.workload])
    if args.n_train:
        W["n_train"] = args.n_train
    if args.chunk:
        W["chunk"] = args.chunk
    torch.cuda.set_device(0)
    N, nq, p, l, a, T = W["N"], W["nq"], W["p"], W["l"], W["a"], W["T"]
    seeds = dict(key=11, x=12, y=13, perm=14, xt=15)
    Xtr, ytr, Xte, yte = gen_data(args.workload, W)
    W["minmax"] = args.workload == "wisconsin"
    ref = np.concatenate([Xtr, Xte])  # min-max range of the float features
    W["ref"] = ref
    Xtr, ytr = Xtr[:W["n_train"]], ytr[:W["n_train"]]
    n = len(Xtr)
    bits_tr = CL.thermometer(levels_of(CL, W, Xtr, ref), T)
    s = bits_tr.shape[1]
    L = CL.ceil_log2(l)
    lab_tr = CL.label_bits(ytr, l)
    lb, dig = (6, 5) if args.gadget == "6x5" else (15, 2)
    ctx = HW.Context(N, nq, p, log_base=lb, digits=dig)
    for f in args.force:
        kname, var = f.split("=")
        ctx.tune_set(kname, int(var))
    sh = HW.shape(s, l, a, seeds["perm"])
    k0, k1, model_bytes = ctx.dims(sh)
    dev = torch.device("cuda:0")
    # inputs resident in HBM before timing: thermometer bits, label bits, key
    xb = torch.from_numpy(bits_tr).to(dev)
    yb = torch.from_numpy(lab_tr).to(dev)
    sk = torch.zeros(N, dtype=torch.int32, device=dev)
    ctx.keygen(seeds["key"], sk)
    chunk = W["chunk"]
    # with --overlap, two chunk buffers: the client encrypts chunk k+1 on its
    # own stream while the server trains chunk k (both at the default priority)
    nbuf = 2 if args.overlap else 1
    xr = [torch.empty(chunk * s, ctx.rgsw_words, dtype=torch.int32, device=dev) for _ in range(nbuf)]
    yr = [torch.empty(max(1, chunk * L), ctx.rgsw_words, dtype=torch.int32, device=dev) for _ in range(nbuf)]
    H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev)
    cnt = torch.zeros(2, nq, N, dtype=torch.int32, device=dev) if W["balance"] else None
    s_train = torch.cuda.current_stream(dev)
    s_enc = torch.cuda.Stream(device=dev) if args.overlap else s_train

    def train_step():
        H.zero_()
        if cnt is not None:
            cnt.zero_()
        prog = Progress("training samples", n)
        free = [None] * nbuf  # event: the training that last read buffer b is done
        s_enc.wait_stream(s_train)
        for idx, c0 in enumerate(range(0, n, chunk)):
            m = min(chunk, n - c0)
            b = idx % nbuf
            with torch.cuda.stream(s_enc):
                if free[b] is not None:
                    s_enc.wait_event(free[b])
                ctx.encrypt_rgsw_bits(sk, xb[c0:c0 + m].reshape(-1), seeds["x"], c0 * s, xr[b][:m * s])
                if L:
                    ctx.encrypt_rgsw_bits(sk, yb[c0:c0 + m].reshape(-1), seeds["y"], c0 * L, yr[b][:m * L])
                enc_done = torch.cuda.Event()
                enc_done.record(s_enc)
            s_train.wait_event(enc_done)
            ctx.train(sh, xr[b], yr[b], m, H, cnt)
            free[b] = torch.cuda.Event()
            free[b].record(s_train)
            prog(c0 + m)
        s_train.wait_stream(s_enc)

    print("bench: workload %s, n_train %d, chunk %d, k0 %d, k1 %d" % (args.workload, n, chunk, k0, k1),
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        train_step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        train_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = n / (ms_per_step / 1000.0)
    tr_ms, tr_launch, tr_xp = ctx.profile_read("train")
    rd_ms, _, _ = ctx.profile_read("reduce")
    # bytes the reductions read and write: per launch every live leaf of every
    # (sample, RAM) block (4 B) plus the model read and written (8 B per word)
    rd_bytes = args.steps * (n * (k0 * k1 + (1 if W["balance"] else 0)) * ctx.rlwe_words * 4
                             + -(-n // chunk) * (k0 * k1 + (1 if W["balance"] else 0)) * ctx.rlwe_words * 8)
    en_ms, en_launch, en_rows = ctx.profile_read("encrypt_rgsw")
    ctx.profile(False)
    print("bench: %.1f ms/step, %.2f samples/s" % (ms_per_step, value), file=sys.stderr, flush=True)

    if args.calib_copy:
        src = torch.empty(args.calib_copy * (1 << 20) // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    steps_xp = tr_xp / args.steps
    steps_ivps = n * (k0 + (1 if W["balance"] and L else 0))  # IVP chains per step
    steps_full = steps_xp - steps_ivps                         # external products other than the chains' first
    train_kernel_ms = tr_ms / args.steps
    opx = ops_per_xp(N, nq)
    result = {
        "metric": "encrypted train samples/s",
        "value": round(value, 3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": W["name"], "n_train": n, "s": s, "k0": k0, "k1": k1,
                   "chunk": chunk, "step": "device RGSW encryption + homomorphic training of n_train samples",
                   "gadget": "%d balanced digits of %d bits per prime" % (dig, lb)},
    }
    # IVP chains per step: every (sample, RAM) plus the class counter's (label bits only)
    ivps = args.steps * steps_ivps
    peaks = None if args.no_peaks else device_peaks(dev)
    result["roofline"] = xp_roofline("k_train", N, nq, tr_xp, tr_ms, tr_launch, peaks,
                                     ops=train_ops(N, nq, tr_xp, ivps) if dig == 5 else None, dig=dig)
    result["roofline"]["traffic"] = (measured_traffic(ctx.schedule().get("train"))
                                     if args.workload == "mnist" and chunk == 50 and dig == 5 else None)
    result["roofline"]["traffic_unit"] = ("HBM bytes per training call of the schedule in use (rocprofv3 "
                                          "FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)")
    result["roofline"]["first_xp_of_chain"] = ("one product in %d reads half its RGSW (no forward transforms)"
                                               % round(steps_xp / steps_ivps))
    result["device_peaks"] = peaks
    result["kernels"] = {
        # with encryption on its own stream the step takes less than the sum of its kernels
        "overlap": "encryption of chunk k+1 on a second stream while chunk k trains" if args.overlap else "serial",
        "kernel_sum_ms_per_step": round((tr_ms + rd_ms + en_ms) / args.steps, 2),
        "train_ms_per_step": round(train_kernel_ms, 2),
        "reduce_ms_per_step": round(rd_ms / args.steps, 2),
        # k_reduce_model reads every sample's leaf block once: bytes / time
        "reduce_hbm_frac": round(rd_bytes / (rd_ms / 1000.0) / 1e9 / PEAK_HBM_GBS, 4) if rd_ms else None,
        "encrypt_ms_per_step": round(en_ms / args.steps, 2),
        "train_only_samples_per_s": round(n / (train_kernel_ms / 1000.0), 3) if train_kernel_ms else None,
        "encrypt_only_samples_per_s": round(n / (en_ms / args.steps / 1000.0), 3) if en_ms else None,
        "encrypt_roofline": {
            "bound": "alu", "kernel": "k_enc_rgsw", "unit": "TOPS(int32)", "peak": round(PEAK_INT32_TOPS, 2),
            "achieved": round(en_rows * ops_per_enc_row(N, nq) / (en_ms / 1000.0) / 1e12, 3) if en_ms else None,
            "frac": round(en_rows * ops_per_enc_row(N, nq) / (en_ms / 1000.0) / 1e12 / PEAK_INT32_TOPS, 4)
            if en_ms else None,
            "rows": en_rows, "ops_per_row": ops_per_enc_row(N, nq)},
        "xp_per_s": round(steps_xp / (train_kernel_ms / 1000.0), 1) if train_kernel_ms else None,
        # the first product of each chain: 2 nq inverse NTTs, 2 nq N evaluation products, half the RGSW
        "ntt_per_s_in_xp": round((steps_full * (2 * dig * nq * nq + 2 * nq) + steps_ivps * 2 * nq)
                                 / (train_kernel_ms / 1000.0), 1) if train_kernel_ms else None,
        "modmul_per_s": round((steps_full * modmul_per_xp(N, nq, dig) + steps_ivps * (
            2 * nq * (N // 2) * (N.bit_length() - 1) + 2 * nq * N)) / (train_kernel_ms / 1000.0), 1)
        if train_kernel_ms else None,
        "rgsw_read_gbs": round((steps_full + steps_ivps / 2) * rgsw_bytes(N, nq, dig) / (train_kernel_ms / 1000.0) / 1e9,
                               1) if train_kernel_ms else None,
    }

    result["schedule"] = ctx.schedule()
    del xr, yr, xb, yb
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["inference"], cells0 = infer_pass(ctx, sh, H, sk, Xte, yte, W, seeds, k0, dev, peaks)
        if not args.no_gadget_leg and dig == 5:
            result["gadget_15x2"] = gadget_pass(W, bits_tr, lab_tr, Xte, seeds, s, k0, k1, dev, H, cells0,
                                                args.steps, args.warmup, peaks)
        result["class_packed"] = packed_layout_pass(ctx, W, bits_tr, lab_tr, Xte, sk, seeds, cells0, dev, peaks)
        if W.get("otf"):
            result["otf_act"] = otf_pass(ctx, sh, H, sk, Xte, W, seeds, k0, dev, cells0)
        if W.get("fm"):
            result["fm_act"] = fm_pass(ctx, sh, H, sk, Xte, W, seeds, k0, k1, dev, cells0, args.fm_full)
        result["merge"] = merge_pass(ctx, H, k0, k1)
        result["ntt"] = ntt_pass(ctx, N, nq, dev)
        result["hbm_copy_gbs"] = hbm_copy(dev)
        if not args.no_batched:
            result["batched"] = [batched_pass(sc, dev) for sc in args.batched_scale]
        if not args.no_served:
            result["served"] = served_pass(dev, args.served_requests, args.served_max_size, args.served_load)
    if not args.no_extras:
        result["schedule"] = ctx.schedule()
    if not args.no_cpu_baseline and not args.no_extras:
        result["cpu_baseline"] = cpu_baseline(args.workload, W, Xtr, ytr, Xte, seeds, ctx, sh, sk, dev, ref)
    print(json.dumps(result), flush=True)


def infer_loop(ctx, sh, H, sk, bits, W, seeds, k0, dev):
    """device encryption + inference + decryption of the test bits, chunk by
    chunk: (decrypted cells [nt][l][k0], seconds, infer kernel ms, XP, the
    last chunk's scores)"""
    import numpy as np
    import torch
    l = W["l"]
    nt, s = bits.shape
    xb = torch.from_numpy(bits).to(dev)
    chunk = max(1, W["chunk"])
    xr = torch.empty(chunk * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    scores = torch.empty(chunk, l, k0, ctx.lwe_words, dtype=torch.int32, device=dev)
    dec = torch.empty(chunk * l * k0, dtype=torch.int64, device=dev)
    cells = np.zeros((nt, l, k0), np.int64)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prog = Progress("inference samples", nt)
    for c0 in range(0, nt, chunk):
        m = min(chunk, nt - c0)
        ctx.encrypt_rgsw_bits(sk, xb[c0:c0 + m].reshape(-1), seeds["xt"], c0 * s, xr[:m * s])
        ctx.infer(sh, H, xr, m, scores, None)
        ctx.decrypt_lwe(sk, scores, m * l * k0, dec)
        cells[c0:c0 + m] = dec[:m * l * k0].cpu().numpy().reshape(m, l, k0)
        prog(c0 + m)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf_ms, inf_launch, inf_xp = ctx.profile_read("infer")
    ctx.profile(False)
    return cells, dt, inf_ms, inf_xp, scores, inf_launch


def infer_pass(ctx, sh, H, sk, Xte, yte, W, seeds, k0, dev, peaks=None):
    """Encrypted inference of the test set (device encryption + VP + PD-act)."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    T, l = W["T"], W["l"]
    bits = CL.thermometer(levels_of(CL, W, Xte[:W["n_test"]], W.get("ref")), T)
    nt = len(bits)
    chunk = max(1, W["chunk"])
    cells, dt, inf_ms, inf_xp, scores, inf_launch = infer_loop(ctx, sh, H, sk, bits, W, seeds, k0, dev)
    # PackingKeySwitching of the last chunk's scores: l k0 LWE -> one RLWE per
    # sample (when l k0 <= N), decrypting to the same cells
    packed = None
    k = l * k0
    if k <= ctx.N:
        key = torch.empty(ctx.pks_key_words, dtype=torch.int32, device=dev)
        ctx.pks_keygen(sk, seeds["key"] + 100, key)
        m = nt - (nt - 1) // chunk * chunk
        out = torch.empty(m, ctx.rlwe_words, dtype=torch.int32, device=dev)
        ctx.pack_lwe(key, scores, k, m, out)  # warm-up
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(3):
            ctx.pack_lwe(key, scores, k, m, out)
        pk_ms, _, pk_groups = ctx.profile_read("pack_lwe")
        ctx.profile(False)
        pdec = torch.empty(m, ctx.N, dtype=torch.int64, device=dev)
        ctx.decrypt_rlwe(sk, out, m, pdec)
        same = np.array_equal(pdec.cpu().numpy()[:, :k].reshape(m, l, k0), cells[nt - m:])
        packed = {"lwe_per_sample": k, "ms_per_sample": round(pk_ms / pk_groups, 3),
                  "bytes_per_sample": ctx.rlwe_words * 4, "lwe_bytes_per_sample": k * ctx.lwe_words * 4,
                  "decrypts_equal": bool(same), "key_mib": round(ctx.pks_key_words * 4 / 2**20, 1)}
        del key, out
    pred = CL.pd_act_predict(cells, "bin")
    acc = float((pred == np.asarray(yte[:nt])).mean())
    N, nq, dig = ctx.N, ctx.nq, ctx.digits
    return {
        "samples_per_s": round(nt / dt, 3),
        "infer_kernel_samples_per_s": round(nt / (inf_ms / 1000.0), 3) if inf_ms else None,
        "xp_per_s": round(inf_xp / (inf_ms / 1000.0), 1) if inf_ms else None,
        "roofline": xp_roofline("k_infer", N, nq, inf_xp, inf_ms, inf_launch, peaks,
                                ops=inf_xp * ops_per_xp(N, nq) if dig == 5 else None, dig=dig),
        "n_test": nt, "pd_act": "bin", "test_accuracy": round(acc, 4),
        "packing": packed,
    }, cells


def gadget_pass(W, bits_tr, lab_tr, Xte, seeds, s, k0, k1, dev, H0, cells0, steps: int, warmup: int,
                peaks=None):
    """The step (device RGSW encryption + homomorphic training of the n_train
    samples) and the test-set inference again, with RGSW of 2 balanced
    digits of 15 bits per prime (the digit size of the paper's HE1 TFHE
    set) instead of 5 of 6 bits, on the same ring, key and seeds: rates, the
    training call's per-product roofline in that gadget's units, and whether
    the decrypted model and scores equal the default gadget's.  Rings of two
    or more primes only (None otherwise)."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    N, nq, p, l, a, T = W["N"], W["nq"], W["p"], W["l"], W["a"], W["T"]
    if nq < 2:
        return None
    ctx = HW.Context(N, nq, p, log_base=15, digits=2)
    sh = HW.shape(s, l, a, seeds["perm"])
    sk = torch.zeros(N, dtype=torch.int32, device=dev)
    ctx.keygen(seeds["key"], sk)
    n, L, chunk = len(bits_tr), CL.ceil_log2(l), W["chunk"]
    xb = torch.from_numpy(bits_tr).to(dev)
    yb = torch.from_numpy(lab_tr).to(dev)
    xr = torch.empty(chunk * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    yr = torch.empty(max(1, chunk * L), ctx.rgsw_words, dtype=torch.int32, device=dev)
    H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev)
    cnt = torch.zeros(2, nq, N, dtype=torch.int32, device=dev) if W["balance"] else None

    def step():
        H.zero_()
        if cnt is not None:
            cnt.zero_()
        for c0 in range(0, n, chunk):
            m = min(chunk, n - c0)
            ctx.encrypt_rgsw_bits(sk, xb[c0:c0 + m].reshape(-1), seeds["x"], c0 * s, xr[:m * s])
            if L:
                ctx.encrypt_rgsw_bits(sk, yb[c0:c0 + m].reshape(-1), seeds["y"], c0 * L, yr[:m * L])
            ctx.train(sh, xr, yr, m, H, cnt)

    print("bench: the same step with RGSW of 2 digits of 15 bits", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    tr_ms, tr_launch, tr_xp = ctx.profile_read("train")
    en_ms, _, _ = ctx.profile_read("encrypt_rgsw")
    ctx.profile(False)
    del xr, yr, xb, yb
    d0 = torch.empty(k0 * k1, N, dtype=torch.int64, device=dev)
    d1 = torch.empty_like(d0)
    ctx.decrypt_rlwe(sk, H0, k0 * k1, d0)  # RLWE under the same key: either context decrypts it
    ctx.decrypt_rlwe(sk, H, k0 * k1, d1)
    same_model = bool(torch.equal(d0, d1))
    del d0, d1
    bits = CL.thermometer(levels_of(CL, W, Xte[:W["n_test"]], W.get("ref")), T)
    cells, dt, inf_ms, inf_xp, _, inf_launch = infer_loop(ctx, sh, H, sk, bits, W, seeds, k0, dev)
    nt = len(bits)
    out = {
        "gadget": "2 balanced digits of 15 bits per prime (RGSW of 2 x 2 nq rows)",
        "samples_per_s": round(n / (ms / 1000.0), 3), "ms_per_step": round(ms, 2), "steps": steps,
        "train_ms_per_step": round(tr_ms / steps, 2), "encrypt_ms_per_step": round(en_ms / steps, 2),
        "train_only_samples_per_s": round(n / (tr_ms / steps / 1000.0), 3) if tr_ms else None,
        "xp_per_s": round(tr_xp / (tr_ms / 1000.0), 1) if tr_ms else None,
        "roofline": xp_roofline("k_train", N, nq, tr_xp, tr_ms, tr_launch, peaks, dig=2),
        "model_cells_equal_default_gadget": same_model,
        "inference": {"samples_per_s": round(nt / dt, 3),
                      "infer_kernel_samples_per_s": round(nt / (inf_ms / 1000.0), 3) if inf_ms else None,
                      "xp_per_s": round(inf_xp / (inf_ms / 1000.0), 1) if inf_ms else None,
                      "scores_equal_default_gadget": bool(np.array_equal(cells, cells0))},
    }
    del H, cnt
    torch.cuda.empty_cache()
    return out


def boot_key(ctx, sk, seed: int, W: dict, dev):
    """the bootstrapping key of the workload: through a key switch to a
    binary LWE key of W["boot_n"] coefficients, or (boot_n = 0) over the
    ring key.  Returns (key for the bootstrapping calls, description,
    key generation seconds)."""
    import torch
    N = W["N"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if W.get("boot_n"):
        key = ctx.pbs_ks_keygen(sk, seed, W["boot_n"], dev)
        info = {"kind": "key switch to a binary LWE key", "n": W["boot_n"],
                "external_products_per_bootstrap": W["boot_n"],
                "bsk_gib": round(key.bsk.numel() * 4 / 2**30, 3), "ksk_mib": round(key.ksk.numel() / 2**20, 1)}
    else:
        key = torch.empty(ctx.pbs_key_words(N), dtype=torch.int32, device=dev)
        ctx.pbs_keygen(sk, seed, N, key)
        info = {"kind": "ring key (two CMUXes per coefficient)", "n": N, "external_products_per_bootstrap": 2 * N,
                "bsk_gib": round(ctx.pbs_key_words(N) * 4 / 2**30, 3)}
    torch.cuda.synchronize()
    return key, info, time.perf_counter() - t0


def act_max(kind: str, param: int, P: int) -> int:
    """largest value the activation takes on m < 2^P"""
    return 1 if kind == "ge" else (P if kind == "log" else min(param, P))


def act_bootstraps(kind: str, param: int, P: int) -> int:
    """bootstraps of one activation (hw_activate)"""
    if kind == "ge" or kind == "log" or param >= P - 1:
        return 2 * P
    return 2 * P - 1


def act_name(kind: str, param: int) -> str:
    return {"ge": "bin, thr = %d: [count >= %d]" % (param - 1, param), "log": "log: floor(log2(count + 1))",
            "blog": "b-log: min(floor(log2(count + 1)), %d)" % param}[kind]


def act_plain(CL, x, kind: str, param: int):
    """the activation in the clear (the client's functions)"""
    return CL.activate(x, *{"ge": ("bin", param - 1, 4), "log": ("log", 0, 4), "blog": ("blog", 0, param)}[kind])


def pd_predict(CL, cells, kind: str, param: int):
    """PD-act predictions with the same activation"""
    k, thr, cap = {"ge": ("bin", param - 1, 4), "log": ("log", 0, 4), "blog": ("blog", 0, param)}[kind]
    return CL.pd_act_predict(cells, k, thr, cap)


def otf_pass(ctx, sh, H, sk, Xte, W, seeds, k0, dev, cells0):
    """OTF-act (Sec. 3.5.2, Alg. 7) on the first W["otf"] test samples: every
    per-RAM score activated with the model's activation (W["act"]: the
    paper's parameter table gives the Wisconsin model log) by the
    bootstrapped circuit (hw_activate), summed per class (hw_class_sums),
    then EncryptedArgMax: only the class index is decrypted.  Compared with
    the PD-act prediction of the same samples (decrypted cells, the same
    activation, ArgMax on the client)."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    N, nq, l, T = W["N"], W["nq"], W["l"], W["T"]
    m = min(W["otf"], W["n_test"])
    bits = CL.thermometer(levels_of(CL, W, Xte[:m], W.get("ref")), T)
    s = bits.shape[1]
    xr = torch.empty(m * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    ctx.encrypt_rgsw_bits(sk, torch.from_numpy(bits).to(dev).reshape(-1), seeds["xt"], 0, xr)
    sc = torch.empty(m, l, k0, ctx.lwe_words, dtype=torch.int32, device=dev)
    ctx.infer(sh, H, xr, m, sc, None)
    del xr
    bsk, key_info, key_s = boot_key(ctx, sk, seeds["key"] + 200, W, dev)
    kind, param = W["act"]
    P = (W["p"] - 1).bit_length()
    lp = (k0 * act_max(kind, param, P)).bit_length() + 1  # class sums below p_out / 2
    act = torch.empty(m * l * k0, ctx.lwe_words, dtype=torch.int32, device=dev)
    sums = torch.empty(m, l, ctx.lwe_words, dtype=torch.int32, device=dev)
    idx = torch.empty(m, ctx.lwe_words, dtype=torch.int32, device=dev)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.activate(bsk, N, sc, m * l * k0, kind, param, lp, act)
    ctx.class_sums(act, m, l, k0, sums)
    ctx.encrypted_argmax(bsk, N, sums, m, l, lp, idx)  # n is the key's when bsk is key-switched
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a_ms = ctx.profile_read("activate")[0]
    g_ms = ctx.profile_read("argmax")[0]
    ctx.profile(False)
    L = (l - 1).bit_length()
    dc = HW.Context(N, nq, 1 << (L + 1))
    out = torch.empty(m, dtype=torch.int64, device=dev)
    dc.decrypt_lwe(sk, idx, m, out)
    got = out.cpu().numpy()
    want = pd_predict(CL, cells0[:m], kind, param)
    pbs_per_sample = l * k0 * act_bootstraps(kind, param, P) + (l * (l - 1) // 2) * lp + l * max(0, l - 2)
    del bsk, act, sums, idx, sc
    torch.cuda.empty_cache()
    xpb = key_info["external_products_per_bootstrap"]
    return {"samples": m, "activation": act_name(kind, param), "output_modulus": 1 << lp, "key": key_info,
            "bootstraps_per_sample": pbs_per_sample,
            "external_products_per_bootstrap": xpb,
            "seconds": round(dt, 3), "samples_per_s": round(m / dt, 4),
            "activate_ms_per_sample": round(a_ms / m, 2), "argmax_ms_per_sample": round(g_ms / m, 2),
            "external_products_per_s": round(m * pbs_per_sample * xpb / dt, 1), "keygen_s": round(key_s, 3),
            "predictions_equal_pd_act": bool(np.array_equal(got, want)),
            "paper_estimate": "OTF-act 3.7 min per inference at 9-bit precision on one thread (paper Table 9)"}


def fm_pass(ctx, sh, H, sk, Xte, W, seeds, k0, k1, dev, cells0, full=False):
    """FM-act (Sec. 3.5.3): the model's cells activated once with the
    model's activation (W["act"]) by bootstraps and packed back into their
    rows (hw_fm_act).  By default the first W["fm"] RAMs (every cell of their
    rows), timed, with the full model's time extrapolated from the cell
    rate; each activated cell is checked against the decrypted cell.  With
    `full`, the whole model, then inference on it for the first W["otf"]
    test samples (VP, class sums, EncryptedArgMax: Alg. 7's FM-act branch),
    compared with the PD-act prediction of the same samples."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    N, nq, l, a, T = W["N"], W["nq"], W["l"], W["a"], W["T"]
    rows = k0 if full else min(W["fm"], k0)
    shs = sh if full else HW.shape(rows * a, l, a, seeds["perm"], 0)  # the first `rows` RAMs
    src = H.view(k0 * k1, -1)[: rows * k1]
    bsk, key_info, key_s = boot_key(ctx, sk, seeds["key"] + 300, W, dev)
    key = torch.empty(ctx.pks_key_words, dtype=torch.int32, device=dev)
    ctx.pks_keygen(sk, seeds["key"] + 301, key)
    kind, param = W["act"]
    P = (W["p"] - 1).bit_length()
    lp = (k0 * act_max(kind, param, P)).bit_length() + 1  # class sums below p_out / 2
    act = torch.empty_like(src)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fm_act(shs, bsk, N, key, src, kind, param, lp, act)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = {k: ctx.profile_read(k)[0] for k in ("extract_cells", "activate", "pack_lwe")}
    ctx.profile(False)
    K = 1 << min((l - 1).bit_length() + a, N.bit_length() - 1)
    cells = rows * k1 * K
    dec0 = torch.empty(rows * k1, N, dtype=torch.int64, device=dev)
    ctx.decrypt_rlwe(sk, src, rows * k1, dec0)
    dc = HW.Context(N, nq, 1 << lp)
    dec1 = torch.empty(rows * k1, N, dtype=torch.int64, device=dev)
    dc.decrypt_rlwe(sk, act, rows * k1, dec1)
    want = act_plain(CL, dec0.cpu().numpy(), kind, param)
    want[:, K:] = 0
    nb = act_bootstraps(kind, param, P)
    xpb = key_info["external_products_per_bootstrap"]
    out = {"rams": rows, "cells": cells, "activation": act_name(kind, param), "output_modulus": 1 << lp,
           "key": key_info, "bootstraps_per_cell": nb, "external_products_per_bootstrap": xpb,
           "seconds": round(dt, 3), "cells_per_s": round(cells / dt, 2),
           "external_products_per_s": round(cells * nb * xpb / dt, 1),
           "ms": {k: round(v, 1) for k, v in ms.items()},
           "full_model_cells": k0 * k1 * K, "full_model_s": round(k0 * k1 * K / (cells / dt), 1),
           "keygen_s": round(key_s, 3), "pks_key_gib": round(ctx.pks_key_words * 4 / 2**30, 2),
           "activated_cells_equal": bool(np.array_equal(dec1.cpu().numpy(), want)),
           "paper_estimate": "FM-act 0.1 h for the Wisconsin model at 9-bit precision on 64 threads (paper Table 9)"}
    if full:
        m = min(W["otf"], W["n_test"])
        bits = CL.thermometer(levels_of(CL, W, Xte[:m], W.get("ref")), T)
        s = bits.shape[1]
        xr = torch.empty(m * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
        ctx.encrypt_rgsw_bits(sk, torch.from_numpy(bits).to(dev).reshape(-1), seeds["xt"], 0, xr)
        sc = torch.empty(m, l, k0, ctx.lwe_words, dtype=torch.int32, device=dev)
        sums = torch.empty(m, l, ctx.lwe_words, dtype=torch.int32, device=dev)
        idx = torch.empty(m, ctx.lwe_words, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.infer(sh, act.view(H.shape), xr, m, sc, None)
        ctx.class_sums(sc, m, l, k0, sums)
        ctx.encrypted_argmax(bsk, N, sums, m, l, lp, idx)
        torch.cuda.synchronize()
        di = time.perf_counter() - t0
        L = (l - 1).bit_length()
        got = torch.empty(m, dtype=torch.int64, device=dev)
        HW.Context(N, nq, 1 << (L + 1)).decrypt_lwe(sk, idx, m, got)
        out["inference"] = {"samples": m, "seconds": round(di, 3), "samples_per_s": round(m / di, 3),
                            "predictions_equal_pd_act": bool(np.array_equal(got.cpu().numpy(),
                                                                            pd_predict(CL, cells0[:m], kind, param)))}
        del xr, sc, sums, idx
    del bsk, key, act, dec0, dec1
    torch.cuda.empty_cache()
    return out


def packed_layout_pass(ctx, W, bits_tr, lab_tr, Xte, sk, seeds, cells0, dev, peaks=None):
    """The class-packed model layout (horizontal packing across
    discriminators) on the same data and key: training with the index [tuple
    bits, label bits] (every tree leaf kept), then inference by one VP per
    RAM that yields the scores of all classes.  Reports the training and
    inference kernel rates and whether the decrypted scores equal those of
    the label-pruned layout."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    N, nq, l, a, T = W["N"], W["nq"], W["l"], W["a"], W["T"]
    n, s = bits_tr.shape
    L = CL.ceil_log2(l)
    sh = HW.shape(s, l, a, seeds["perm"], HW.LAYOUT_PACKED)
    k0, k1, model_bytes = ctx.dims(sh)
    chunk = W["chunk"]
    xb = torch.from_numpy(bits_tr).to(dev)
    yb = torch.from_numpy(lab_tr).to(dev)
    xr = torch.empty(chunk * s, ctx.rgsw_words, dtype=torch.int32, device=dev)
    yr = torch.empty(max(1, chunk * L), ctx.rgsw_words, dtype=torch.int32, device=dev)
    H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev)
    ctx.profile(True)
    ctx.profile_reset()
    prog = Progress("class-packed training samples", n)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        ctx.encrypt_rgsw_bits(sk, xb[c0:c0 + m].reshape(-1), seeds["x"], c0 * s, xr[:m * s])
        if L:
            ctx.encrypt_rgsw_bits(sk, yb[c0:c0 + m].reshape(-1), seeds["y"], c0 * L, yr[:m * L])
        ctx.train(sh, xr, yr, m, H, None)
        prog(c0 + m)
    torch.cuda.synchronize()
    tr_ms, tr_launch, tr_xp = ctx.profile_read("train")
    rd_ms, _, _ = ctx.profile_read("reduce")
    ctx.profile(False)
    del xr, yr, xb, yb
    bits = CL.thermometer(levels_of(CL, W, Xte[:W["n_test"]], W.get("ref")), T)
    nt = len(bits)
    # untimed: the online tuner's first launches try every schedule of this launch shape
    infer_loop(ctx, sh, H, sk, bits[:8 * W["chunk"]], W, seeds, k0, dev)
    cells, dt, inf_ms, inf_xp, _, inf_launch = infer_loop(ctx, sh, H, sk, bits, W, seeds, k0, dev)
    # several small RAMs per row (layout 2) when a RAM fills less than half an RLWE
    ram_packed = None
    sh2 = HW.shape(s, l, a, seeds["perm"], HW.LAYOUT_RAM_PACKED)
    rows, rpr = ctx.model_rows(sh2)
    if rpr > 1:
        _, _, bytes2 = ctx.dims(sh2)
        H2 = torch.empty(rows, 1, 2, nq, N, dtype=torch.int32, device=dev)
        ctx.pack_rams(sh2, H, H2)
        cells2, dt2, inf2_ms, _, _, _ = infer_loop(ctx, sh2, H2, sk, bits, W, seeds, k0, dev)
        ram_packed = {"rams_per_row": rpr, "rows": rows, "model_mib": round(bytes2 / 2**20, 2),
                      "infer_samples_per_s": round(nt / dt2, 3),
                      "infer_kernel_samples_per_s": round(nt / (inf2_ms / 1000.0), 3) if inf2_ms else None,
                      "scores_equal_label_pruned": bool(np.array_equal(cells2, cells0))}
        del H2
    del H
    torch.cuda.empty_cache()
    return {
        "k1": k1, "model_mib": round(model_bytes / 2**20, 1),
        "train_kernel_samples_per_s": round(n / (tr_ms / 1000.0), 3) if tr_ms else None,
        "train_xp_per_sample": round(tr_xp / n, 1),
        "train_roofline": xp_roofline("k_train (class-packed)", N, nq, tr_xp, tr_ms, tr_launch, peaks,
                                      ops=train_ops(N, nq, tr_xp, n * k0) if ctx.digits == 5 else None,
                                      dig=ctx.digits),
        "reduce_ms": round(rd_ms, 2),
        "infer_samples_per_s": round(nt / dt, 3),
        "infer_kernel_samples_per_s": round(nt / (inf_ms / 1000.0), 3) if inf_ms else None,
        "infer_xp_per_sample": round(inf_xp / nt, 1),
        "infer_roofline": xp_roofline("k_infer (class-packed)", N, nq, inf_xp, inf_ms, inf_launch, peaks,
                                      ops=inf_xp * ops_per_xp(N, nq) if ctx.digits == 5 else None,
                                      dig=ctx.digits),
        "scores_equal_label_pruned": bool(np.array_equal(cells, cells0)),
        "several_rams_per_row": ram_packed,
    }


def merge_pass(ctx, H, k0, k1):
    """Model merge (hw_rlwe_add) of pairs of models of the workload's shape:
    12 bytes of HBM traffic per word (two reads, one write).  Merges rotate
    over 4 distinct pairs (about 1 GB for the MNIST shape) so that no pair is
    still in the 256 MB last-level cache when it is merged again."""
    import torch
    count = k0 * k1
    pairs = [(H.clone(), H.clone()) for _ in range(4)]
    for g, h in pairs:
        ctx.rlwe_add(g, h, count)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    for r in range(20):
        g, h = pairs[r % 4]
        ctx.rlwe_add(g, h, count)
    ms, launches, words = ctx.profile_read("rlwe_add")
    ctx.profile(False)
    gbs = words * 12 / (ms / 1000.0) / 1e9
    del pairs
    return {"model_mib": round(count * ctx.rlwe_words * 4 / 2**20, 1), "ms_per_merge": round(ms / launches, 3),
            "gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}


def ntt_pass(ctx, N, nq, dev):
    """Batched standalone NTT: 2^15 polynomials, forward then inverse."""
    import torch
    count = 1 << 15
    polys = torch.randint(0, min(ctx.primes), (count, nq, N), dtype=torch.int32, device=dev)
    ctx.ntt(polys, count, False)
    ctx.ntt(polys, count, True)
    torch.cuda.synchronize()
    for _ in range(10):  # the first launches tune the schedule (polynomials per workgroup)
        ctx.ntt(polys, count, False)
        ctx.ntt(polys, count, True)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(3):
        ctx.ntt(polys, count, False)
        ctx.ntt(polys, count, True)
    ms, launches, work = ctx.profile_read("ntt")
    ctx.profile(False)
    nt_s = work / (ms / 1000.0)
    bytes_moved = work * N * 4 * 2  # read + write per transform
    # 9 int32 ops per Harvey butterfly (the op model of ops_per_xp): 6.2
    # ops per byte moved at N = 2048, above the chip's 4.9 (39.3 T / 8 TB/s),
    # so the transform is bound by the VALU before HBM
    ops = 9.0 * (N // 2) * (N.bit_length() - 1)
    return {"polys": count * nq, "ntt_per_s": round(nt_s, 1), "gbs": round(bytes_moved / (ms / 1000.0) / 1e9, 1),
            "hbm_frac": round(bytes_moved / (ms / 1000.0) / 1e9 / PEAK_HBM_GBS, 4),
            "ops_per_ntt": ops, "valu_frac": round(nt_s * ops / 1e12 / PEAK_INT32_TOPS, 4),
            "bound": "alu" if ops / (N * 8) > PEAK_INT32_TOPS * 1e12 / (PEAK_HBM_GBS * 1e9) else "hbm"}


def batched_pass(scale: float, dev, window_bytes: int = 96 << 30):
    """256 uneven training jobs (sizes U{32..2000} x scale, s U{128..2352},
    a U{8..12}, l U{2..10}, N 2048 or 4096): batched persistent launches, and
    the replay of a batch plan (the same launches captured into a HIP graph),
    versus the same kernels one job at a time, on the same encrypted inputs.
    Jobs of one ring degree share a context (p = 4096 covers every job's
    counts); they are taken in groups whose input ciphertexts fit in
    `window_bytes` of device memory, each group one batch."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    from paper_2403_20190_amd import synth
    torch.cuda.empty_cache()
    jobs = synth.batched_jobs(2)
    groups = {}
    for j, J in enumerate(jobs):
        groups.setdefault(J["N"], []).append((j, J))
    out = {"jobs": len(jobs), "scale": scale, "samples": 0, "xp": 0.0, "batched_ms": 0.0, "single_ms": 0.0,
           "plan_ms": 0.0, "plan_max_pieces": 0, "kernel_ms": {}, "ops": 0.0, "bytes": 0.0, "modmul": 0.0,
           "bit_identical": True}
    for N, members in sorted(groups.items()):
        nq = 2 if N == 2048 else 3
        ctx = HW.Context(N, nq, 4096)
        sk = torch.zeros(N, dtype=torch.int32, device=dev)
        ctx.keygen(101, sk)
        rg = ctx.rgsw_words * 4
        window = []
        used = 0

        def run(window):
            bufs = []
            for j, J, n in window:
                X, y = synth.prototype_bits(J["seed"] % (2 ** 31), n, J["s"], J["l"])
                L = CL.ceil_log2(J["l"])
                xr = torch.empty(n * J["s"], ctx.rgsw_words, dtype=torch.int32, device=dev)
                ctx.encrypt_rgsw_bits(sk, torch.from_numpy(X.reshape(-1)).to(dev), 1000 + j, 0, xr)
                yr = None
                if L:
                    yr = torch.empty(n * L, ctx.rgsw_words, dtype=torch.int32, device=dev)
                    ctx.encrypt_rgsw_bits(sk, torch.from_numpy(CL.label_bits(y, J["l"]).reshape(-1)).to(dev),
                                          2000 + j, 0, yr)
                sh = HW.shape(J["s"], J["l"], J["a"], 3000 + j)
                k0, k1, _ = ctx.dims(sh)
                bufs.append((sh, xr, yr, n, k0, k1))
            mw = [torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev) for (_, _, _, _, k0, k1) in bufs]
            mb = [torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev) for (_, _, _, _, k0, k1) in bufs]
            ms = [torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev) for (_, _, _, _, k0, k1) in bufs]
            mp = [torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev) for (_, _, _, _, k0, k1) in bufs]
            plan = ctx.batch_plan([(sh, xr, yr, n, m, None) for (sh, xr, yr, n, _, _), m in zip(bufs, mp)])
            # untimed: a first eager batch sizes the context's workspace and lets the
            # tuner try its schedules (the one-job path then finds its workspace ready too)
            ctx.batch_train([(sh, xr, yr, n, m, None) for (sh, xr, yr, n, _, _), m in zip(bufs, mw)])
            torch.cuda.synchronize()
            del mw
            ctx.profile(True)
            ctx.profile_reset()
            torch.cuda.synchronize()
            e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
            e0.record()
            ctx.batch_train([(sh, xr, yr, n, m, None) for (sh, xr, yr, n, _, _), m in zip(bufs, mb)])
            e1.record()
            for (sh, xr, yr, n, _, _), m in zip(bufs, ms):
                ctx.train(sh, xr, yr, n, m, None)
            e2.record()
            plan.launch()
            e3.record()
            torch.cuda.synchronize()
            out["batched_ms"] += e0.elapsed_time(e1)
            out["single_ms"] += e1.elapsed_time(e2)
            out["plan_ms"] += e2.elapsed_time(e3)
            out["plan_max_pieces"] = max(out["plan_max_pieces"], plan.max_pieces)
            xpb = ctx.profile_read("train_batch")[2]
            out["xp"] += xpb
            out["ops"] += train_ops(N, nq, xpb, sum(b[3] * b[4] for b in bufs))
            out["bytes"] += xpb * rgsw_bytes(N, nq)
            out["modmul"] += xpb * modmul_per_xp(N, nq)
            for k in ("train_batch", "reduce_batch", "train", "reduce", "batch_plan"):
                out["kernel_ms"][k] = out["kernel_ms"].get(k, 0.0) + ctx.profile_read(k)[0]
            ctx.profile(False)
            plan.close()
            out["samples"] += sum(b[3] for b in bufs)
            out["bit_identical"] &= all(torch.equal(a, b) for a, b in zip(mb, ms))
            out["bit_identical"] &= all(torch.equal(a, b) for a, b in zip(mb, mp))

        for j, J in members:
            n = max(1, int(round(J["n"] * scale)))
            need = n * (J["s"] + 4) * rg
            if window and used + need > window_bytes:
                run(window)
                window, used = [], 0
            window.append((j, J, n))
            used += need
        if window:
            run(window)
        ctx.close()
        torch.cuda.empty_cache()
    out["batched_samples_per_s"] = round(out["samples"] / (out["batched_ms"] / 1000.0), 2)
    out["single_job_samples_per_s"] = round(out["samples"] / (out["single_ms"] / 1000.0), 2)
    out["batched_xp_per_s"] = round(out["xp"] / (out["batched_ms"] / 1000.0), 1)
    # k_train_batch in per-product units (each ring degree's RGSW bytes and
    # modular multiplications) over the persistent kernel's time
    tb = out["kernel_ms"].get("train_batch", 0.0)
    if tb:
        sec = tb / 1000.0
        hf = out["bytes"] / sec / 1e9 / PEAK_HBM_GBS
        vf = out["modmul"] * MUL_PER_MODMUL / sec / 1e12 / PEAK_INT32_TOPS
        out["roofline"] = {"kernel": "k_train_batch", "bound": "hbm" if hf >= vf else "alu",
                           "hbm_gbs": round(out["bytes"] / sec / 1e9, 1), "hbm_frac": round(hf, 4),
                           "modmul_per_s": round(out["modmul"] / sec, 1), "valu_frac": round(vf, 4),
                           "op_model_frac": round(out["ops"] / sec / 1e12 / PEAK_INT32_TOPS, 4)}
    del out["ops"], out["bytes"], out["modmul"]
    out["speedup"] = round(out["single_ms"] / out["batched_ms"], 3)
    out["plan_speedup"] = round(out["single_ms"] / out["plan_ms"], 3)
    out["batched_ms"] = round(out["batched_ms"], 1)
    out["single_ms"] = round(out["single_ms"], 1)
    out["plan_ms"] = round(out["plan_ms"], 1)
    out["kernel_ms"] = {k: round(v, 1) for k, v in out["kernel_ms"].items()}
    return out


def served_setup(dev, n_req: int, max_size: int, seed: int = 5, gadget=(6, 5)):
    """The served workload: one parameter set (N=2048, two primes, p=2^16;
    RGSW gadget (log_base, digits)) and key; half Wisconsin-shaped (30 features, 2 classes 357/212, min-max +
    16-level thermometer = 480 bits, tuple 8), half MNIST-shaped models, 4
    resident models of each shape pre-trained with 64 samples; n_req
    requests, half train and half infer, sizes U{1..max_size}.  Returns
    (ctx, make_engine, reqs)."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    from paper_2403_20190_amd import synth
    N, nq, p = 2048, 2, 1 << 16
    torch.cuda.empty_cache()
    ctx = HW.Context(N, nq, p, log_base=gadget[0], digits=gadget[1])
    sk = torch.zeros(N, dtype=torch.int32, device=dev)
    ctx.keygen(202, sk)
    Xw, yw = synth.wisconsin_like(4)
    lo, hi = Xw.min(axis=0), Xw.max(axis=0)
    bits_w = CL.thermometer(CL.quantize_minmax(Xw, 16, lo, hi), 16)
    Xm, ym, _, _ = synth.mnist_like(1, per_class_train=60, per_class_test=1)
    bits_m = CL.thermometer(CL.quantize_u8(Xm, 3), 3)
    shapes = {"wisconsin": (bits_w, yw, 2, 8), "mnist": (bits_m, ym, 10, 12)}
    g = np.random.Generator(np.random.PCG64(seed))
    pre = {}  # the pre-training samples of each model, drawn once
    for name, (bits, y, l, a) in shapes.items():
        for r in range(4):
            pre[(name, r)] = g.integers(0, len(bits), 64)

    def make_engine(order="fifo"):
        eng = HW.Engine(N, nq, p, sk, slots=4, chunk=8, max_s=2352, max_cells=2048, arena_bytes=64 << 30, order=order,
                        log_base=gadget[0], digits=gadget[1])
        jobs = []
        for name, (bits, y, l, a) in shapes.items():
            for r in range(4):
                sh = HW.shape(bits.shape[1], l, a, 7000 + 10 * len(jobs))
                k0, k1, _ = ctx.dims(sh)
                H = torch.zeros(k0, k1, 2, nq, N, dtype=torch.int32, device=dev)
                j = eng.add_job(sh, H)
                idx = pre[(name, r)]
                rid = eng.submit(j, "train", bits[idx], 8000 + j, labels=CL.label_bits(y[idx], l))
                eng.wait(rid)
                jobs.append((j, name, H, k0))
        return eng, jobs

    reqs = []
    for k in range(n_req):
        name = "wisconsin" if g.random() < 0.5 else "mnist"
        bits, y, l, a = shapes[name]
        size = int(g.integers(1, max_size + 1))
        idx = g.integers(0, len(bits), size)
        reqs.append(dict(shape=name, kind="train" if g.random() < 0.5 else "infer", job=int(g.integers(0, 4)),
                         bits=bits[idx], labels=CL.label_bits(y[idx], l), l=l, size=size, seed=9000 + 7 * k))
    return ctx, make_engine, reqs


def served_play(make_engine, reqs, arrivals, one_at_a_time: bool = False):
    """Submit the requests at their arrival times (s from the start) to a
    fresh engine; (latencies ms, span s, engine stats).  one_at_a_time: each
    request is submitted only after the previous one finished (the plain
    one-job-at-a-time path; latencies are then service times)."""
    import numpy as np
    eng, jobs = make_engine()
    by = {}
    for j, name, H, k0 in jobs:
        by.setdefault(name, []).append((j, k0))
    t0 = time.perf_counter()
    ids, lat = [], []
    for i, (r, t_arr) in enumerate(zip(reqs, arrivals)):
        dt = t0 + t_arr - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        j, k0 = by[r["shape"]][r["job"]]
        cells = np.zeros((r["size"], r["l"], k0), np.uint64) if r["kind"] == "infer" else None
        rid = eng.submit(j, r["kind"], r["bits"], r["seed"], labels=r["labels"] if r["kind"] == "train" else None,
                         cells=cells)
        if one_at_a_time:
            lat.append(eng.wait(rid)[1])
        else:
            ids.append(rid)
        if i % 16 == 15:
            print("bench: served %d / %d submitted" % (i + 1, len(reqs)), file=sys.stderr, flush=True)
    last = time.perf_counter()
    for k, i in enumerate(ids):
        lat.append(eng.wait(i)[1])
        if time.perf_counter() - last > 10.0:
            print("bench: served %d / %d done" % (k + 1, len(ids)), file=sys.stderr, flush=True)
            last = time.perf_counter()
    span = time.perf_counter() - t0
    st = eng.stats()
    eng.close()
    return np.array(lat), span, st


def lindley(service_ms, arrivals_s):
    """Latencies (ms) of a single FIFO server with the given service times
    under the given arrivals: W_{k+1} = max(0, W_k + S_k - (A_{k+1} - A_k))."""
    import numpy as np
    S = np.asarray(service_ms, float)
    A = np.asarray(arrivals_s, float) * 1000.0
    W = np.zeros_like(S)
    for k in range(1, len(S)):
        W[k] = max(0.0, W[k - 1] + S[k - 1] - (A[k] - A[k - 1]))
    return W + S


def served_pass(dev, n_req: int, max_size: int, load: float):
    """Continuous batching of Poisson-arrival train/infer requests (the
    default run's scaled-down served mix): all requests at once
    (saturation), then Poisson arrivals at `load` x the saturated rate."""
    import numpy as np

    from paper_2403_20190_amd import synth
    ctx, make_engine, reqs = served_setup(dev, n_req, max_size)
    lat0, span0, st0 = served_play(make_engine, reqs, [0.0] * n_req)
    sat_rps = n_req / span0
    qps = load * sat_rps
    arr = synth.poisson_arrivals(6, qps, n_req)
    lat1, span1, st1 = served_play(make_engine, reqs, list(arr - arr[0]))
    samples = sum(r["size"] for r in reqs)
    ctx.close()
    return {
        "requests": n_req, "sizes": "U{1..%d}" % max_size, "samples": samples,
        "saturated_req_per_s": round(sat_rps, 3), "saturated_samples_per_s": round(samples / span0, 2),
        "offered_qps": round(qps, 3), "load": load,
        "p50_ms": round(float(np.percentile(lat1, 50)), 2), "p99_ms": round(float(np.percentile(lat1, 99)), 2),
        "throughput_samples_per_s": round(samples / span1, 2),
        "saturated_p50_ms": round(float(np.percentile(lat0, 50)), 2),
        "saturated_p99_ms": round(float(np.percentile(lat0, 99)), 2),
        "peak_inflight_chunks": st1["peak_inflight"], "peak_arena_gib": round(st1["peak_arena_bytes"] / 2**30, 2),
    }


def served_full(dev, n_req: int, max_size: int, loads, sat_rps: float | None, sequential: bool,
                orders=("fifo",), gadget=(6, 5)) -> dict:
    """The served configuration at its stated size: 400 requests of U{1..500}
    samples.  Runs whichever parts are asked for (each can be its own
    process, so that one run stays within a time limit): the saturated run
    (all requests at t = 0), which sets the request rate the loads scale;
    Poisson arrivals at each load x that rate (p50/p99 latency, throughput);
    and the same request list one job at a time (service times, from which
    the one-job-at-a-time latencies under the same arrivals follow by the
    single-server recursion).  Each load runs once per engine order in
    `orders` ("fifo", "shortest"), the saturated run with the first."""
    import numpy as np

    from paper_2403_20190_amd import synth
    ctx, make_engine, reqs = served_setup(dev, n_req, max_size, gadget=gadget)
    samples = sum(r["size"] for r in reqs)
    out = {"requests": n_req, "sizes": "U{1..%d}" % max_size, "samples": samples,
           "gadget": "%d digits of %d bits per prime" % (gadget[1], gadget[0]),
           "mix": {"train": sum(r["kind"] == "train" for r in reqs), "mnist": sum(r["shape"] == "mnist" for r in reqs)}}

    def pct(x):
        return {"p50_ms": round(float(np.percentile(x, 50)), 1), "p99_ms": round(float(np.percentile(x, 99)), 1)}

    if sat_rps is None:
        lat0, span0, st0 = served_play(lambda: make_engine(orders[0]), reqs, [0.0] * n_req)
        sat_rps = n_req / span0
        out["saturated"] = dict(req_per_s=round(sat_rps, 4), samples_per_s=round(samples / span0, 2),
                                span_s=round(span0, 1), peak_inflight_chunks=st0["peak_inflight"], **pct(lat0))
    out["saturated_req_per_s"] = round(sat_rps, 4)
    if sequential:
        svc, span1, _ = served_play(make_engine, reqs, [0.0] * n_req, one_at_a_time=True)
        # the same Poisson arrivals as the loaded runs, served one request at a time
        q = []
        for load in (0.25, 0.5, 0.75, 0.9):
            arr = synth.poisson_arrivals(6, load * sat_rps, n_req)
            q.append(dict(load=load, **pct(lindley(svc, arr - arr[0]))))
        out["one_at_a_time"] = dict(samples_per_s=round(samples / span1, 2), span_s=round(span1, 1),
                                    service=pct(svc), poisson=q)
    out["loads"] = []
    for load in loads:
        qps = load * sat_rps
        arr = synth.poisson_arrivals(6, qps, n_req)
        arr = list(arr - arr[0])
        for order in orders:
            lat, span, st = served_play(lambda: make_engine(order), reqs, arr)
            out["loads"].append(dict(load=load, order=order, offered_qps=round(qps, 4),
                                     throughput_samples_per_s=round(samples / span, 2),
                                     span_s=round(span, 1), peak_inflight_chunks=st["peak_inflight"],
                                     peak_arena_gib=round(st["peak_arena_bytes"] / 2**30, 2), **pct(lat)))
    ctx.close()
    return out


def batched_oracle_leg(st, ring: int, nq: int, nrams: int) -> dict:
    """The oracle on the job of the mix with the fewest external products per
    RAM over all its samples: the RGSW of every sample's bits for its first
    RAMs (as many as host threads, at most `nrams`; the oracle trains RAMs in
    parallel) and its label bits (the same seeds and ciphertext indices as
    the device), then those RAMs trained over all of the job's samples; the
    rows are compared bit for bit with the persistent batch's model, and the
    oracle's rate is given per external product and extrapolated to the job
    and the mix."""
    import numpy as np

    import oracle as O
    S = min(st, key=lambda S: S["J"]["n"] * job_xp_per_ram(S["J"], ring))
    J, j = S["J"], S["j"]
    n, s_, l, a, L = J["n"], J["s"], J["l"], J["a"], S["L"]
    info = host_info()
    threads = max(1, min(16, info["affinity"]))
    orc = O.Ctx(ring, nq, 4096)
    sk = orc.keygen(101)
    pi = O.permutation(3000 + j, s_)
    k0 = -(-s_ // a)
    rams = list(range(min(nrams, threads, k0)))
    X, y = S["X"], S["y"]
    xs, ys = {}, {}
    need = [(i, int(pi[r * a + t])) for r in rams for i in range(n) for t in range(min(a, s_ - r * a))]
    t0 = time.perf_counter()
    O._parallel(lambda ik: xs.__setitem__(ik, orc.enc_rgsw(sk, int(X[ik[0], ik[1]]), 1000 + j, ik[0] * s_ + ik[1])),
                need, threads)
    O._parallel(lambda iu: ys.__setitem__(iu, orc.enc_rgsw(sk, (int(y[iu[0]]) >> iu[1]) & 1, 2000 + j,
                                                           iu[0] * L + iu[1])),
                [(i, u) for i in range(n) for u in range(L)], threads)
    t_enc = time.perf_counter() - t0
    H = np.zeros((k0, orc.k1(s_, l, a), 2, nq, ring), np.uint32)
    t0 = time.perf_counter()
    orc.train(s_, l, a, pi, lambda i, k: xs[(i, k)], lambda i, u: ys[(i, u)], n, H, rams=rams, threads=threads)
    t_train = time.perf_counter() - t0
    got = S["mb"].cpu().numpy().view(np.uint32)
    xp = n * len(rams) * job_xp_per_ram(J, ring)
    rate = xp / t_train
    mix_xp = sum(S2["J"]["n"] * job_xp_per_sample(S2["J"], ring) for S2 in st)
    return {"value": round(rate, 2), "unit": "external products/s (training)", "cores": threads, "kind": "oracle",
            "sample": "job %d (n %d, s %d, a %d, l %d): RGSW of the bits of RAMs %s and of "
                      "the labels for all %d samples (%.1f s), then those RAMs trained over all samples (%.1f s)"
                      % (j, n, s_, a, l, rams, n, t_enc, t_train),
            "job_s_extrapolated": round(n * job_xp_per_sample(J, ring) / rate, 1),
            "mix_train_s_extrapolated": round(mix_xp / rate, 1),
            "bit_exact_with_batch": bool(np.array_equal(got[rams], H[rams])), "host": info}


def job_xp_per_ram(J, ring: int) -> int:
    """training external products per (sample, full RAM): the rotation chain
    and the live CDEMUX splits of the label-pruned tree"""
    L = (J["l"] - 1).bit_length()
    logN = ring.bit_length() - 1
    nb = L + J["a"]
    nr = min(nb, logN)
    z = nb - nr
    live = (lambda u: z < L or (u & ((1 << L) - 1)) < J["l"])
    splits = sum(1 for lev in range(z) for u in range(1 << lev) if live(u) and live(u + (1 << lev)))
    return nr + splits


def job_xp_per_sample(J, ring: int) -> int:
    return -(-J["s"] // J["a"]) * job_xp_per_ram(J, ring)


def batched_full(dev, ring: int, window_gib: float, per_job: int, jobs_range=None, chunk: int = 50,
                 oracle_rams: int = 0) -> dict:
    """The batched configuration at its stated size: the 256 jobs of
    synth.batched_jobs (n U{32..2000}, s U{128..2352}, a U{8..12}, l
    U{2..10}), those of ring degree `ring` (two primes at 2048, three at
    4096, p = 4096 >= every job's count).  Their input ciphertexts (up to
    several TB) are streamed: each window takes the next `per_job` samples of
    as many unfinished jobs as fit `window_gib` GiB of encrypted inputs,
    encrypts them on the device, then trains them once as one batch
    (hw_batch_train: one persistent launch over the window's jobs) and once
    job by job (hw_wisard_train_encrypted), into two model sets that must end
    bit-identical.  Times are HIP events around the two training passes;
    encryption is timed apart.  Then the plain one-job-at-a-time path: each
    job alone, its samples encrypted and trained in chunks of `chunk` (as
    many as fit the window), into a third model set that must equal the
    others."""
    import numpy as np
    import torch

    from paper_2403_20190_amd import client as CL
    from paper_2403_20190_amd import hwisard as HW
    from paper_2403_20190_amd import synth
    torch.cuda.empty_cache()
    nq = 2 if ring == 2048 else 3
    alljobs = [(j, J) for j, J in enumerate(synth.batched_jobs(2)) if J["N"] == ring]
    if jobs_range:
        alljobs = alljobs[jobs_range[0]:jobs_range[1]]
    ctx = HW.Context(ring, nq, 4096)
    sk = torch.zeros(ring, dtype=torch.int32, device=dev)
    ctx.keygen(101, sk)
    rg = ctx.rgsw_words * 4
    st = []
    for j, J in alljobs:
        X, y = synth.prototype_bits(J["seed"] % (2 ** 31), J["n"], J["s"], J["l"])
        sh = HW.shape(J["s"], J["l"], J["a"], 3000 + j)
        k0, k1, _ = ctx.dims(sh)
        st.append(dict(j=j, J=J, X=X, y=y, L=CL.ceil_log2(J["l"]), sh=sh, done=0,
                       mb=torch.zeros(k0, k1, 2, nq, ring, dtype=torch.int32, device=dev),
                       ms=torch.zeros(k0, k1, 2, nq, ring, dtype=torch.int32, device=dev)))
    out = {"ring": ring, "jobs": len(st), "samples": int(sum(S["J"]["n"] for S in st)), "windows": 0,
           "batched_ms": 0.0, "single_ms": 0.0, "encrypt_ms": 0.0, "xp": 0.0, "bytes": 0.0, "modmul": 0.0}
    ctx.profile(True)
    ctx.profile_reset()
    prog = Progress("batched samples", out["samples"])
    trained = 0
    while any(S["done"] < S["J"]["n"] for S in st):
        win, used = [], 0
        for S in st:
            m = min(per_job, S["J"]["n"] - S["done"])
            if m <= 0:
                continue
            need = m * (S["J"]["s"] + S["L"]) * rg
            if win and used + need > window_gib * 2**30:
                continue
            win.append((S, m))
            used += need
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record()
        bufs = []
        for S, m in win:
            J, c0 = S["J"], S["done"]
            xr = torch.empty(m * J["s"], ctx.rgsw_words, dtype=torch.int32, device=dev)
            ctx.encrypt_rgsw_bits(sk, torch.from_numpy(S["X"][c0:c0 + m].reshape(-1)).to(dev), 1000 + S["j"],
                                  c0 * J["s"], xr)
            yr = None
            if S["L"]:
                yr = torch.empty(m * S["L"], ctx.rgsw_words, dtype=torch.int32, device=dev)
                ctx.encrypt_rgsw_bits(sk, torch.from_numpy(CL.label_bits(S["y"][c0:c0 + m], J["l"]).reshape(-1))
                                      .to(dev), 2000 + S["j"], c0 * S["L"], yr)
            bufs.append((S, m, xr, yr))
        e1.record()
        ctx.batch_train([(S["sh"], xr, yr, m, S["mb"], None) for S, m, xr, yr in bufs])
        e2.record()
        for S, m, xr, yr in bufs:
            ctx.train(S["sh"], xr, yr, m, S["ms"], None)
        e3.record()
        torch.cuda.synchronize()
        out["encrypt_ms"] += e0.elapsed_time(e1)
        out["batched_ms"] += e1.elapsed_time(e2)
        out["single_ms"] += e2.elapsed_time(e3)
        out["windows"] += 1
        for S, m, _, _ in bufs:
            S["done"] += m
            trained += m
        del bufs
        prog(trained)
    xpb = ctx.profile_read("train_batch")[2]
    out["xp"] = xpb
    out["kernel_ms"] = {k: round(ctx.profile_read(k)[0], 1) for k in ("train_batch", "reduce_batch", "train", "reduce",
                                                                      "encrypt_rgsw")}
    ctx.profile(False)
    out["bit_identical"] = all(torch.equal(S["mb"], S["ms"]) for S in st)
    if oracle_rams:
        out["cpu_baseline"] = batched_oracle_leg(st, ring, nq, oracle_rams)
    # the plain one-job-at-a-time path: job after job, each in chunks that fill the GPU
    for S in st:
        S["ms"].zero_()
    jt = 0.0
    prog = Progress("one-job-at-a-time samples", out["samples"])
    done = 0
    for S in st:
        J = S["J"]
        cmax = max(1, min(chunk, int(window_gib * 2**30 // ((J["s"] + S["L"]) * rg))))
        for c0 in range(0, J["n"], cmax):
            m = min(cmax, J["n"] - c0)
            xr = torch.empty(m * J["s"], ctx.rgsw_words, dtype=torch.int32, device=dev)
            ctx.encrypt_rgsw_bits(sk, torch.from_numpy(S["X"][c0:c0 + m].reshape(-1)).to(dev), 1000 + S["j"],
                                  c0 * J["s"], xr)
            yr = None
            if S["L"]:
                yr = torch.empty(m * S["L"], ctx.rgsw_words, dtype=torch.int32, device=dev)
                ctx.encrypt_rgsw_bits(sk, torch.from_numpy(CL.label_bits(S["y"][c0:c0 + m], J["l"]).reshape(-1))
                                      .to(dev), 2000 + S["j"], c0 * S["L"], yr)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.train(S["sh"], xr, yr, m, S["ms"], None)
            e1.record()
            torch.cuda.synchronize()
            jt += e0.elapsed_time(e1)
            del xr, yr
            done += m
            prog(done)
    out["job_by_job_ms"] = round(jt, 1)
    out["job_by_job_chunk"] = chunk
    out["job_by_job_samples_per_s"] = round(out["samples"] / (jt / 1000.0), 2)
    out["speedup_vs_job_by_job"] = round(jt / out["batched_ms"], 4)
    out["bit_identical"] &= all(torch.equal(S["mb"], S["ms"]) for S in st)
    out["schedule"] = ctx.schedule()
    ctx.close()
    sec_b, sec_s = out["batched_ms"] / 1000.0, out["single_ms"] / 1000.0
    out["batched_samples_per_s"] = round(out["samples"] / sec_b, 2)
    out["single_job_samples_per_s"] = round(out["samples"] / sec_s, 2)
    out["speedup"] = round(sec_s / sec_b, 4)
    tb = out["kernel_ms"]["train_batch"] / 1000.0
    hf = xpb * rgsw_bytes(ring, nq) / tb / 1e9 / PEAK_HBM_GBS if tb else 0.0
    vf = xpb * modmul_per_xp(ring, nq) * MUL_PER_MODMUL / tb / 1e12 / PEAK_INT32_TOPS if tb else 0.0
    out["roofline"] = {"kernel": "k_train_batch", "bound": "hbm" if hf >= vf else "alu",
                       "hbm_gbs": round(xpb * rgsw_bytes(ring, nq) / tb / 1e9, 1) if tb else None,
                       "hbm_frac": round(hf, 4), "valu_frac": round(vf, 4)}
    for k in ("batched_ms", "single_ms", "encrypt_ms"):
        out[k] = round(out[k], 1)
    del out["bytes"], out["modmul"]
    return out


def hbm_copy(dev):
    import torch
    n = (4 << 30) // 4
    a = torch.ones(n, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    return round(2 * n * 4 / (ms / 1000.0) / 1e9, 1)


if __name__ == "__main__":
    main()
