"""Bootstrapped activation (Activate) and EncryptedArgMax on LWE ciphertexts.

TEST INFRASTRUCTURE, like the rest of ``oracle``: only ``tests/`` and
``bench.py``'s ``cpu_baseline`` leg use it.

The paper treats the programmable bootstrapping as a black box that
evaluates two functions over LWE ciphertexts (Sec. 2.5.3): Activate (f over
each ciphertext) and EncryptedArgMax (the index of the largest of several);
OTF-act applies Activate to the inference scores, adds them per class and
returns EncryptedArgMax of the sums (Sec. 3.5.2, Alg. 7).  This module
evaluates them with bootstraps whose test polynomial is a constant V, each
of which decides one sign: V when the switched phase lies in [0, N), -V
otherwise (``Ctx.pbs``).  A sign needs a margin of N/8 positions or more
against the modulus-switch error, where a single bootstrap of a 9-bit count
would need N/1024.  The steps, with integer constants (Q the ciphertext
modulus, p the plaintext modulus, P = log2 p, Delta_p = floor(Q / p)):

bits(x, p): the bits of the message m in [0, p) of x (phase ~ Delta_p m),
least significant first.  V_b = floor(Delta_p / 2).  For k = 0 .. P-1:
    y   = 2^(P-1-k) x + floor(Q/4)       (bit k of m decides the top bit)
    o   = PBS(y, V_b)                    (V_b if the bit is 0, -V_b if 1)
    E_k = V_b - o                        (phase ~ 2 V_b bit_k)
    x   = x - 2^k E_k                    (bit k removed: m -> m - 2^k bit_k)

activate_ge(x, T, p_out): an LWE of [m >= T] (phase ~ 2 V_o [m >= T],
V_o = floor(Delta_{p_out} / 2)), 1 <= T <= p: the carry out of m + (p - T),
t = p - T, carry c_0 = 0, V_c = floor(Q/16), for k = 0 .. P-1:
    z = 2^(P-3) E_k + c_k - (V_c if bit k of t is 1 else 3 V_c)
    c_{k+1} = PBS(z, V) + V,  V = V_o for k = P-1, V_c before
(with b_k + c_k in {0, 1, 2} at scale ~Q/8, subtracting Q/16 decides
b_k OR c_k, subtracting 3Q/16 decides b_k AND c_k).

activate_log(x, p_out, cap): the logarithmic activations of Sec. 2.4.2,
log(m) = floor(log2(m + 1)) and b-log(m) = min(log(m), cap), as LWE with
phase ~ 2 V_o f(m), p_out >= 8.  With m' = m + 1 mod p (x plus Delta_p on
the body; m' = 0 only for m = p - 1) and o_i = [m' >= 2^i] = OR of bits
i..P-1 of m', log(m) = sum_{i=1}^{P-1} o_i + P (1 - o_0) and, for cap < P,
b-log(m) = sum_{i=1}^{cap} o_i + cap (1 - o_0).  Steps: E = bits(x', p);
chain value c = 2^(P-3) E_{P-1} (scale ~Q/8); for i = P-2 down to 0,
z_i = 2^(P-3) E_i + c - V_c (the OR decision, as in the carry circuit),
w_i = PBS(z_i, V_o) + V_o (o_i at the output scale) and, while i >= 1,
c = 2^(log2 p_out - 3) w_i (o_i back at the chain scale ~Q/8).  o_(P-1),
when the sum needs it, is PBS(2^(P-3) E_{P-1} - V_c, V_o) + V_o.  2P
bootstraps for log, 2P - 1 for b-log with cap < P - 1.

fm_act(H, K, T, p_out): FM-act (Sec. 3.5.3), the activation applied once to
every cell of a trained model: for every model row (one RLWE), the LWE of
each of its coefficients 0..K-1 (ExtractLWE), activate_ge of it, and the K
results packed back into one RLWE at the same coefficients
(PackingKeySwitching, Sec. 2.5.1); coefficients from K on decrypt to 0.  K
(fm_cells) covers every cell a RAM's index can address: with nb = ceil(log2
l) + a index bits, cell m sits at coefficient m >> z, z = nb - min(nb, log2
N), so K = 2^min(nb, log2 N); rows holding several RAMs fill all N.

argmax(u, p_in): the index of the largest of l class scores s_c in
[0, p_in/2) (phase ~ 2 V_i s_c, V_i = floor(Delta_{p_in} / 2)), ties to the
lowest index: for c < c', D = s_c - s_c' + p_in/2 lies in [0, p_in) and its
top bit is [s_c >= s_c']; G(c, c') = 2^(P-3) E_{P-1}(D) (scale ~Q/8),
G(c', c) = S8 - G(c, c') with S8 = 2^(P-3) 2 V_i.  W_c = the AND over c' != c
of G(c, c') (chains of PBS(a + b - 3 V_c, V) + V, the last with
V = V_x = floor(floor(Q / 2^(L+1)) / 2), L = ceil(log2 l); for l = 2,
W_c = 2 G(c, c')); index = sum_c c W_c (phase ~ 2 V_x index).
"""
from __future__ import annotations

import numpy as np


def log2_exact(p: int) -> int:
    P = p.bit_length() - 1
    if p != 1 << P:
        raise ValueError("%d is not a power of two" % p)
    return P


def lin(ctx, terms, const: int = 0) -> np.ndarray:
    """sum of alpha * x over (alpha, x) terms, plus `const` on the body, mod each q_i"""
    out = np.zeros((ctx.nq, ctx.N + 1), np.uint64)
    for i, q in enumerate(ctx.primes):
        acc = np.zeros(ctx.N + 1, np.uint64)
        for alpha, x in terms:
            acc = (acc + (int(alpha) % q) * np.asarray(x, np.uint64)[i] % q) % q
        acc[ctx.N] = (int(acc[ctx.N]) + const) % q
        out[i] = acc
    return out.astype(np.uint32)


def trivial(ctx, value: int) -> np.ndarray:
    return lin(ctx, [], value)


def encrypt_short(ctx, s, m: int, n: int, p: int, rng) -> np.ndarray:
    """An LWE encryption of m (phase Delta_p m + e, |e| <= 8) under the first n
    coefficients of the ring key s, mask zero past them: seeded test input."""
    delta = ctx.Q // p
    e = int(rng.integers(-8, 9))
    out = np.zeros((ctx.nq, ctx.N + 1), np.uint32)
    for i, q in enumerate(ctx.primes):  # independent residues: a uniform mask mod Q (CRT)
        out[i, :n] = rng.integers(0, q, n)
    for i, q in enumerate(ctx.primes):
        dot = sum(int(out[i, k]) * (int(s[k]) % q) for k in range(n))
        out[i, ctx.N] = (dot + delta * m + e) % q
    return out


def phase(ctx, s, lwe) -> int:
    """b - <a, s> in [0, Q), by the CRT of the residues"""
    Q = ctx.Q
    out = 0
    for i, q in enumerate(ctx.primes):
        a = np.asarray(lwe, np.int64)[i]
        r = (int(a[ctx.N]) - sum(int(a[k]) * int(s[k]) for k in range(ctx.N))) % q
        Mi = Q // q
        out += r * Mi * pow(Mi, -1, q)
    return out % Q


def decode(ctx, s, lwe, p: int) -> int:
    """round(phase p / Q) mod p"""
    return ((phase(ctx, s, lwe) * p + ctx.Q // 2) // ctx.Q) % p


def bits(ctx, bsk, n: int, x, p: int) -> list:
    P = log2_exact(p)
    Q = ctx.Q
    vb = (Q // p) // 2
    E = []
    for k in range(P):
        y = lin(ctx, [(1 << (P - 1 - k), x)], Q // 4)
        o = ctx.pbs(bsk, y, n, vb)
        e = lin(ctx, [(-1, o)], vb)
        E.append(e)
        x = lin(ctx, [(1, x), (-(1 << k), e)])
    return E


def activate_ge(ctx, bsk, n: int, x, T: int, p_out: int) -> np.ndarray:
    p = ctx.p
    P = log2_exact(p)
    if P < 3 or not 1 <= T <= p:
        raise ValueError("needs p >= 8 and 1 <= T <= p")
    Q = ctx.Q
    E = bits(ctx, bsk, n, x, p)
    t = p - T
    vc = Q // 16
    vo = (Q // p_out) // 2
    carry = trivial(ctx, 0)
    for k in range(P):
        z = lin(ctx, [(1 << (P - 3), E[k]), (1, carry)], -(vc if (t >> k) & 1 else 3 * vc))
        V = vo if k == P - 1 else vc
        carry = lin(ctx, [(1, ctx.pbs(bsk, z, n, V))], V)
    return carry


def activate_log(ctx, bsk, n: int, x, p_out: int, cap: int | None = None) -> np.ndarray:
    p = ctx.p
    P = log2_exact(p)
    lo = log2_exact(p_out)
    if P < 3 or lo < 3 or (cap is not None and cap < 1):
        raise ValueError("needs p >= 8, p_out >= 8 and cap >= 1")
    top = P - 1 if cap is None or cap >= P else cap  # outputs o_1 .. o_top
    kc = P if cap is None or cap >= P else cap
    Q = ctx.Q
    vc = Q // 16
    vo = (Q // p_out) // 2
    sh = 1 << (P - 3)
    E = bits(ctx, bsk, n, lin(ctx, [(1, x)], Q // p), p)
    chain = lin(ctx, [(sh, E[P - 1])])
    terms = []
    if top == P - 1:
        z = lin(ctx, [(sh, E[P - 1])], -vc)
        terms.append((1, lin(ctx, [(1, ctx.pbs(bsk, z, n, vo))], vo)))
    for i in range(P - 2, -1, -1):
        z = lin(ctx, [(sh, E[i]), (1, chain)], -vc)
        w = lin(ctx, [(1, ctx.pbs(bsk, z, n, vo))], vo)
        if i == 0:
            terms.append((-kc, w))
        elif i <= top:
            terms.append((1, w))
        if i >= 1:
            chain = lin(ctx, [(1 << (lo - 3), w)])
    return lin(ctx, terms, kc * 2 * vo)


def argmax(ctx, bsk, n: int, u, p_in: int) -> np.ndarray:
    l = len(u)
    P = log2_exact(p_in)
    if l < 2 or P < 3:
        raise ValueError("needs l >= 2 and p_in >= 8")
    Q = ctx.Q
    L = (l - 1).bit_length()
    vi = (Q // p_in) // 2
    vc = Q // 16
    vx = (Q // (1 << (L + 1))) // 2
    s8 = (1 << (P - 3)) * 2 * vi
    G = {}
    for c in range(l):
        for c2 in range(c + 1, l):
            d = lin(ctx, [(1, u[c]), (-1, u[c2])], (p_in // 2) * 2 * vi)
            msb = bits(ctx, bsk, n, d, p_in)[P - 1]
            G[(c, c2)] = lin(ctx, [(1 << (P - 3), msb)])
            G[(c2, c)] = lin(ctx, [(-1, G[(c, c2)])], s8)
    W = []
    for c in range(l):
        others = [c2 for c2 in range(l) if c2 != c]
        if l == 2:
            W.append(lin(ctx, [(2, G[(c, others[0])])]))
            continue
        acc = G[(c, others[0])]
        for j, c2 in enumerate(others[1:]):
            V = vx if j == len(others) - 2 else vc
            z = lin(ctx, [(1, acc), (1, G[(c, c2)])], -3 * vc)
            acc = lin(ctx, [(1, ctx.pbs(bsk, z, n, V))], V)
        W.append(acc)
    return lin(ctx, [(c, W[c]) for c in range(1, l)])


def fm_cells(N: int, l: int, a: int, layout: int = 0) -> int:
    """coefficients of a model row that hold cells: 2^min(ceil(log2 l) + a,
    log2 N), or N when a row holds several RAMs (layout 2)"""
    logN = N.bit_length() - 1
    nb = (l - 1).bit_length() + a
    return N if layout == 2 else 1 << min(nb, logN)


def fm_act(ctx, bsk, n: int, K_pks, H, cells: int, T: int, p_out: int) -> np.ndarray:
    """FM-act of a model H (RLWE rows of any leading shape, [..][2][nq][N]):
    each row's coefficients 0..cells-1 extracted, activated with [m >= T]
    (activate_ge, output modulus p_out) and packed back into one RLWE"""
    from . import _parallel
    H = np.ascontiguousarray(H, np.uint32)
    rows = H.reshape(-1, 2, ctx.nq, ctx.N)
    jobs = [(r, i) for r in range(len(rows)) for i in range(cells)]
    act = {}

    def one(ri):
        r, i = ri
        act[ri] = activate_ge(ctx, bsk, n, ctx.extract_lwe(rows[r], i), T, p_out)

    _parallel(one, jobs)
    out = np.zeros_like(rows)
    for r in range(len(rows)):
        out[r] = ctx.pack_lwe(K_pks, np.stack([act[(r, i)] for i in range(cells)]))
    return out.reshape(H.shape)
