"""CPU oracle for the encrypted WiSARD hot path (Homomorphic WiSARDs, arXiv 2403.20190).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package.  The product package
never imports it, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, exact integer arithmetic); this
module is a ctypes wrapper around it that marshals numpy arrays.  The
plaintext WiSARD (Def. 1, Alg. 1/2/4) and the client-side decode and PD-act
live in :mod:`oracle.plain`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

u32p = C.POINTER(C.c_uint32)
u64p = C.POINTER(C.c_uint64)
i32p = C.POINTER(C.c_int32)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            sig = {
                "orc_is_prime": (C.c_int, [C.c_uint64]),
                "orc_find_primes": (C.c_int, [C.c_uint32, C.c_uint32, u32p]),
                "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
                "orc_w64": (C.c_uint64, [C.c_uint64, C.c_uint32, C.c_uint64]),
                "orc_w32": (C.c_uint32, [C.c_uint64, C.c_uint32, C.c_uint64]),
                "orc_uniform_mod": (C.c_uint64, [C.c_uint64, C.c_uint64, C.c_uint64]),
                "orc_cdt_table": (None, [C.c_double, u64p]),
                "orc_cdt_sample": (C.c_int64, [u64p, C.c_uint64]),
                "orc_ctx_new": (C.c_void_p, [C.c_uint32, C.c_uint32, u32p, C.c_uint32, C.c_uint32, C.c_uint64, C.c_double]),
                "orc_ctx_free": (None, [C.c_void_p]),
                "orc_ctx_info": (None, [C.c_void_p, u32p, u64p, u64p, u64p]),
                "orc_ctx_cdt": (None, [C.c_void_p, u64p]),
                "orc_negmul_schoolbook": (None, [C.c_uint32, C.c_uint64, u64p, u64p, u64p]),
                "orc_negmul": (None, [C.c_void_p, C.c_uint32, u64p, u64p, u64p]),
                "orc_rlwe_rotate": (None, [C.c_void_p, u32p, C.c_int64, u32p]),
                "orc_keygen": (None, [C.c_void_p, C.c_uint64, i32p]),
                "orc_enc_rlwe_row": (None, [C.c_void_p, i32p, u64p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, u32p]),
                "orc_enc_rlwe": (None, [C.c_void_p, i32p, u64p, C.c_uint64, C.c_uint64, u32p]),
                "orc_enc_rgsw": (None, [C.c_void_p, i32p, C.c_uint32, C.c_uint64, C.c_uint64, u32p]),
                "orc_trivial_rgsw": (None, [C.c_void_p, C.c_uint32, u32p]),
                "orc_dec_rlwe": (None, [C.c_void_p, i32p, u32p, u64p]),
                "orc_noise_rlwe": (C.c_double, [C.c_void_p, i32p, u32p, u64p, C.POINTER(C.c_double)]),
                "orc_dec_lwe": (None, [C.c_void_p, i32p, u32p, u64p]),
                "orc_decompose": (None, [C.c_void_p, u32p, i32p]),
                "orc_extprod": (None, [C.c_void_p, u32p, u32p, u32p]),
                "orc_cmux": (None, [C.c_void_p, u32p, u32p, u32p, u32p]),
                "orc_blind_rotate": (None, [C.c_void_p, u32p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_uint32, u32p]),
                "orc_cdemux": (None, [C.c_void_p, u32p, u32p, u32p, u32p]),
                "orc_ivp": (None, [C.c_void_p, C.POINTER(C.c_void_p), C.c_uint32, u32p, u32p]),
                "orc_ivp_pruned": (None, [C.c_void_p, C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32, u32p, u32p]),
                "orc_leaf_row": (C.c_int32, [C.c_uint32, C.c_uint32, C.c_uint32]),
                "orc_rlwe_add_n": (None, [C.c_void_p, u32p, u32p, C.c_uint64, u32p]),
                "orc_pks_keygen": (None, [C.c_void_p, i32p, C.c_uint64, C.c_uint32, C.c_uint32, u32p]),
                "orc_pks_partial": (None, [C.c_void_p, u32p, u32p, C.c_uint32, C.c_uint32, C.c_uint32, u32p]),
                "orc_pks_finish": (None, [C.c_void_p, u32p, C.c_uint32, u32p, u32p]),
                "orc_extract_lwe0": (None, [C.c_void_p, u32p, u32p]),
                "orc_modswitch": (None, [C.c_void_p, u32p, C.c_uint32, C.POINTER(C.c_int64)]),
                "orc_pbs": (None, [C.c_void_p, C.POINTER(C.c_void_p), u32p, C.c_uint32, u64p, u32p]),
                "orc_vp": (None, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_uint8), C.c_uint32, u32p, u32p]),
                "orc_permutation": (None, [C.c_uint64, C.c_uint32, u32p]),
                "orc_k1": (C.c_uint32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32]),
                "orc_k1_layout": (C.c_uint32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
                "orc_train": (None, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, u32p, C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                     u32p]),
                "orc_infer_packed": (None, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, u32p, u32p,
                                            C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32, u32p]),
                "orc_rams_per_row": (C.c_uint32, [C.c_void_p, C.c_uint32, C.c_uint32]),
                "orc_model_rows": (C.c_uint32, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
                "orc_pack_rams": (None, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, u32p, u32p]),
                "orc_extract_lwe": (None, [C.c_void_p, u32p, C.c_uint32, u32p]),
                "orc_vp_rlwe": (None, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_uint8), C.c_uint32, u32p,
                                       u32p]),
                "orc_class_count": (None, [C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p), C.c_uint64, u32p]),
                "orc_infer_one": (None, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, u32p, u32p,
                                         C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32, u32p]),
                "orc_lwe_add": (None, [C.c_void_p, u32p, u32p, u32p]),
                "orc_rlwe_words": (C.c_uint64, [C.c_void_p]),
                "orc_rgsw_words": (C.c_uint64, [C.c_void_p]),
                "orc_logN": (C.c_uint32, [C.c_void_p]),
                "orc_lwe_keygen": (None, [C.c_uint64, C.c_uint32, C.POINTER(C.c_uint8)]),
                "orc_ksk_gen": (None, [C.c_void_p, i32p, C.POINTER(C.c_uint8), C.c_uint32, C.c_uint64, C.c_uint32,
                                       C.c_uint32, u32p]),
                "orc_key_switch": (None, [C.c_void_p, u32p, C.c_uint32, u32p, u32p]),
                "orc_pbs_ks": (None, [C.c_void_p, C.POINTER(C.c_void_p), u32p, C.c_uint32, u32p, u64p, u32p]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _p(a: np.ndarray, t):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(t)


def _ptr_array(arrs):
    """Array of void* to the given numpy arrays (None -> NULL)."""
    out = (C.c_void_p * max(1, len(arrs)))()
    for i, a in enumerate(arrs):
        out[i] = None if a is None else a.ctypes.data
    return out


# ---------------------------------------------------------------------------
# free functions
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(n))


def find_primes(N: int, nq: int) -> list[int]:
    out = np.zeros(nq, np.uint32)
    if lib().orc_find_primes(N, nq, _p(out, u32p)) != 0:
        raise ValueError("not enough primes")
    return [int(x) for x in out]


def philox4x32_10(ctr, key) -> list[int]:
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c, u32p), _p(k, u32p), _p(o, u32p))
    return [int(x) for x in o]


def leaf_row(d: int, z: int, l: int) -> int:
    """model row of tree leaf d (z tree bits, l classes), -1 for no class < l"""
    return int(lib().orc_leaf_row(d, z, l))


def w64(seed: int, domain: int, index: int) -> int:
    return int(lib().orc_w64(seed, domain, index))


# domain of the serving engine's per-request seed derivation
DOM_REQ = 6


def request_seeds(enc_seed: int) -> tuple[int, int]:
    """Encryption seeds (inputs, labels) that a serving request with seed
    enc_seed uses: the 64-bit draws 0 and 1 of stream (enc_seed, DOM_REQ).
    Deriving both by the generator, not by seed arithmetic, keys every
    request's input and label streams apart (Sec. 2.5: each RLWE sample takes
    fresh randomness)."""
    return w64(enc_seed, DOM_REQ, 0), w64(enc_seed, DOM_REQ, 1)


def w32(seed: int, domain: int, index: int) -> int:
    return int(lib().orc_w32(seed, domain, index))


def uniform_mod(seed: int, x: int, q: int) -> int:
    """uniform residue mod q of encryption draw x (32-bit word with rejection,
    64-bit fallback draw)"""
    return int(lib().orc_uniform_mod(seed, x, q))


def cdt_table(sigma: float = 3.2) -> np.ndarray:
    T = np.zeros(42, np.uint64)
    lib().orc_cdt_table(sigma, _p(T, u64p))
    return T


def cdt_sample(T: np.ndarray, w: int) -> int:
    return int(lib().orc_cdt_sample(_p(T, u64p), w))


def negmul_schoolbook(q: int, a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, np.uint64)
    b = np.ascontiguousarray(b, np.uint64)
    out = np.zeros_like(a)
    lib().orc_negmul_schoolbook(len(a), q, _p(a, u64p), _p(b, u64p), _p(out, u64p))
    return out


def permutation(seed: int, s: int) -> np.ndarray:
    pi = np.zeros(max(1, s), np.uint32)
    lib().orc_permutation(seed, s, _p(pi, u32p))
    return pi[:s]


def ceil_log2(l: int) -> int:
    L = 0
    while (1 << L) < l:
        L += 1
    return L


# ---------------------------------------------------------------------------
# parameter context
# ---------------------------------------------------------------------------

class Ctx:
    """One RLWE parameter set: ring degree N, nq primes, gadget base 2^log_base
    with `digits` digits per prime, plaintext modulus p, Gaussian sigma."""

    def __init__(self, N: int, nq: int, p: int, primes=None, log_base: int = 6, digits: int = 5,
                 sigma: float = 3.2):
        pr = np.zeros(4, np.uint32)
        if primes:
            pr[: len(primes)] = primes
        h = lib().orc_ctx_new(N, nq, _p(pr, u32p), log_base, digits, p, sigma)
        if not h:
            raise ValueError("invalid oracle parameters")
        self.h = C.c_void_p(h)
        self.N, self.nq, self.p = N, nq, p
        self.log_base, self.digits, self.sigma = log_base, digits, sigma
        self.D = digits * nq
        self.logN = int(lib().orc_logN(self.h))
        prim = np.zeros(4, np.uint32)
        dm = np.zeros(4, np.uint64)
        qw = np.zeros(2, np.uint64)
        dw = np.zeros(2, np.uint64)
        lib().orc_ctx_info(self.h, _p(prim, u32p), _p(dm, u64p), _p(qw, u64p), _p(dw, u64p))
        self.primes = [int(x) for x in prim[:nq]]
        self.delta_mod = [int(x) for x in dm[:nq]]
        self.Q = int(qw[0]) | (int(qw[1]) << 64)
        self.delta = int(dw[0]) | (int(dw[1]) << 64)
        self.rlwe_words = int(lib().orc_rlwe_words(self.h))
        self.rgsw_words = int(lib().orc_rgsw_words(self.h))
        self.lwe_words = nq * (N + 1)

    def __del__(self):
        try:
            lib().orc_ctx_free(self.h)
        except Exception:
            pass

    # -- shapes ------------------------------------------------------------
    def rlwe(self, count=None):
        shape = (2, self.nq, self.N) if count is None else (count, 2, self.nq, self.N)
        return np.zeros(shape, np.uint32)

    def cdt(self) -> np.ndarray:
        T = np.zeros(42, np.uint64)
        lib().orc_ctx_cdt(self.h, _p(T, u64p))
        return T

    # -- ring ----------------------------------------------------------------
    def negmul(self, i: int, a, b) -> np.ndarray:
        a = np.ascontiguousarray(a, np.uint64)
        b = np.ascontiguousarray(b, np.uint64)
        out = np.zeros(self.N, np.uint64)
        lib().orc_negmul(self.h, i, _p(a, u64p), _p(b, u64p), _p(out, u64p))
        return out

    def rotate(self, ct, e: int) -> np.ndarray:
        ct = np.ascontiguousarray(ct, np.uint32)
        out = np.zeros_like(ct)
        lib().orc_rlwe_rotate(self.h, _p(ct, u32p), e, _p(out, u32p))
        return out

    # -- keys and encryption -------------------------------------------------
    def keygen(self, seed: int) -> np.ndarray:
        s = np.zeros(self.N, np.int32)
        lib().orc_keygen(self.h, seed, _p(s, i32p))
        return s

    def enc_rlwe(self, s, mu, seed: int, ct: int) -> np.ndarray:
        out = self.rlwe()
        mu_p = None
        if mu is not None:
            mu = np.ascontiguousarray(mu, np.uint64)
            mu_p = _p(mu, u64p)
        lib().orc_enc_rlwe(self.h, _p(s, i32p), mu_p, seed, ct, _p(out, u32p))
        return out

    def enc_rgsw(self, s, m: int, seed: int, ct: int) -> np.ndarray:
        out = np.zeros((2 * self.D, 2, self.nq, self.N), np.uint32)
        lib().orc_enc_rgsw(self.h, _p(s, i32p), int(m), seed, ct, _p(out, u32p))
        return out

    def enc_rgsw_bits(self, s, bits, seed: int, ct0: int) -> np.ndarray:
        bits = np.asarray(bits).reshape(-1)
        out = np.zeros((len(bits), 2 * self.D, 2, self.nq, self.N), np.uint32)

        def one(k):
            lib().orc_enc_rgsw(self.h, _p(s, i32p), int(bits[k]), seed, ct0 + k, _p(out[k], u32p))

        _parallel(one, range(len(bits)))
        return out

    def trivial_rgsw(self, m: int) -> np.ndarray:
        out = np.zeros((2 * self.D, 2, self.nq, self.N), np.uint32)
        lib().orc_trivial_rgsw(self.h, int(m), _p(out, u32p))
        return out

    def trivial_rlwe(self, mu_const: int = 1) -> np.ndarray:
        """(0, Delta*mu) with mu a constant polynomial: the IVP input of Alg. 6."""
        out = self.rlwe()
        for i, q in enumerate(self.primes):
            out[1, i, 0] = (self.delta_mod[i] * mu_const) % q
        return out

    def dec_rlwe(self, s, ct) -> np.ndarray:
        ct = np.ascontiguousarray(ct, np.uint32)
        mu = np.zeros(self.N, np.uint64)
        lib().orc_dec_rlwe(self.h, _p(s, i32p), _p(ct, u32p), _p(mu, u64p))
        return mu

    def noise_rlwe(self, s, ct, mu) -> tuple[float, np.ndarray]:
        ct = np.ascontiguousarray(ct, np.uint32)
        mu = np.ascontiguousarray(mu, np.uint64)
        nz = np.zeros(self.N, np.float64)
        mx = lib().orc_noise_rlwe(self.h, _p(s, i32p), _p(ct, u32p), _p(mu, u64p),
                                  nz.ctypes.data_as(C.POINTER(C.c_double)))
        return float(mx), nz

    def dec_lwe(self, s, lwe) -> int:
        lwe = np.ascontiguousarray(lwe, np.uint32)
        mu = np.zeros(1, np.uint64)
        lib().orc_dec_lwe(self.h, _p(s, i32p), _p(lwe, u32p), _p(mu, u64p))
        return int(mu[0])

    # -- external product and friends ----------------------------------------
    def decompose(self, poly) -> np.ndarray:
        poly = np.ascontiguousarray(poly, np.uint32)
        out = np.zeros((self.D, self.N), np.int32)
        lib().orc_decompose(self.h, _p(poly, u32p), _p(out, i32p))
        return out

    def extprod(self, rgsw, ct) -> np.ndarray:
        rgsw = np.ascontiguousarray(rgsw, np.uint32)
        ct = np.ascontiguousarray(ct, np.uint32)
        out = self.rlwe()
        lib().orc_extprod(self.h, _p(rgsw, u32p), _p(ct, u32p), _p(out, u32p))
        return out

    def cmux(self, rgsw, d1, d0) -> np.ndarray:
        out = self.rlwe()
        args = [np.ascontiguousarray(x, np.uint32) for x in (rgsw, d1, d0)]
        lib().orc_cmux(self.h, *[_p(x, u32p) for x in args], _p(out, u32p))
        return out

    def blind_rotate(self, ct, rgsws, exps) -> np.ndarray:
        ct = np.ascontiguousarray(ct, np.uint32)
        rg = [np.ascontiguousarray(r, np.uint32) for r in rgsws]
        e = (C.c_int64 * max(1, len(exps)))(*[int(x) for x in exps])
        out = self.rlwe()
        lib().orc_blind_rotate(self.h, _p(ct, u32p), _ptr_array(rg), e, len(rg), _p(out, u32p))
        return out

    def cdemux(self, rgsw, ct):
        rgsw = np.ascontiguousarray(rgsw, np.uint32)
        ct = np.ascontiguousarray(ct, np.uint32)
        o0, o1 = self.rlwe(), self.rlwe()
        lib().orc_cdemux(self.h, _p(rgsw, u32p), _p(ct, u32p), _p(o0, u32p), _p(o1, u32p))
        return o0, o1

    def ivp(self, rgsws, ct) -> np.ndarray:
        rg = [np.ascontiguousarray(r, np.uint32) for r in rgsws]
        nb = len(rg)
        nr = min(nb, self.logN)
        out = self.rlwe(1 << (nb - nr))
        ct = np.ascontiguousarray(ct, np.uint32)
        lib().orc_ivp(self.h, _ptr_array(rg), nb, _p(ct, u32p), _p(out, u32p))
        return out

    def ivp_pruned(self, rgsws, l, ct) -> np.ndarray:
        """IVP over [label bits, tuple bits] creating only the tree nodes that
        lead to a class below l; the other leaves are returned as zeros."""
        rg = [np.ascontiguousarray(r, np.uint32) for r in rgsws]
        nb = len(rg)
        nr = min(nb, self.logN)
        out = self.rlwe(1 << (nb - nr))
        ct = np.ascontiguousarray(ct, np.uint32)
        lib().orc_ivp_pruned(self.h, _ptr_array(rg), nb, l, _p(ct, u32p), _p(out, u32p))
        return out

    def vp(self, rgsws, clear, lut) -> np.ndarray:
        """rgsws[u] is an RGSW or None (then clear[u] is the cleartext bit)."""
        rg = [None if r is None else np.ascontiguousarray(r, np.uint32) for r in rgsws]
        cl = (C.c_uint8 * max(1, len(rg)))(*[int(x) for x in clear])
        lut = np.ascontiguousarray(lut, np.uint32)
        out = np.zeros((self.nq, self.N + 1), np.uint32)
        lib().orc_vp(self.h, _ptr_array(rg), cl, len(rg), _p(lut, u32p), _p(out, u32p))
        return out

    def vp_rlwe(self, rgsws, clear, lut) -> np.ndarray:
        """the VP accumulator before ExtractLWE"""
        rg = [None if r is None else np.ascontiguousarray(r, np.uint32) for r in rgsws]
        cl = (C.c_uint8 * max(1, len(rg)))(*[int(x) for x in clear])
        lut = np.ascontiguousarray(lut, np.uint32)
        out = self.rlwe()
        lib().orc_vp_rlwe(self.h, _ptr_array(rg), cl, len(rg), _p(lut, u32p), _p(out, u32p))
        return out

    def extract_lwe(self, ct, idx: int) -> np.ndarray:
        ct = np.ascontiguousarray(ct, np.uint32)
        out = np.zeros((self.nq, self.N + 1), np.uint32)
        lib().orc_extract_lwe(self.h, _p(ct, u32p), idx, _p(out, u32p))
        return out

    def extract_lwe0(self, ct) -> np.ndarray:
        ct = np.ascontiguousarray(ct, np.uint32)
        out = np.zeros((self.nq, self.N + 1), np.uint32)
        lib().orc_extract_lwe0(self.h, _p(ct, u32p), _p(out, u32p))
        return out

    # -- programmable bootstrapping (Sec. 2.5.3; circuits in oracle.pbs) --------
    def modswitch(self, lwe, n: int) -> np.ndarray:
        """round(2N x / Q) mod 2N of the first n mask coefficients and the body"""
        lwe = np.ascontiguousarray(lwe, np.uint32)
        out = np.zeros(n + 1, np.int64)
        lib().orc_modswitch(self.h, _p(lwe, u32p), n, out.ctypes.data_as(C.POINTER(C.c_int64)))
        return out

    def pbs_keygen(self, s, seed: int, n: int) -> list:
        """bootstrapping key for the first n key coefficients: RGSW([s_k = 1])
        and RGSW([s_k = -1]) as ciphertexts 2k and 2k + 1 of stream `seed`"""
        bits = []
        for k in range(n):
            bits += [1 if int(s[k]) == 1 else 0, 1 if int(s[k]) == -1 else 0]
        out = [None] * (2 * n)
        _parallel(lambda t: out.__setitem__(t, self.enc_rgsw(s, bits[t], seed, t)), range(2 * n))
        return out

    def pbs_ks_keygen(self, s, seed: int, n: int) -> "KsKey":
        """bootstrapping key through a key switch: the binary LWE key s1 of n
        coefficients (stream seed, domain LWE_KEY), the key-switching key from
        s to s1 (modulus 2^32, domains KSK_A and KSK_E of seed) and
        bsk[i] = RGSW(s1_i) under s as ciphertext i of stream `seed`"""
        s = np.ascontiguousarray(s, np.int32)
        s1 = np.zeros(n, np.uint8)
        lib().orc_lwe_keygen(seed, n, s1.ctypes.data_as(C.POINTER(C.c_uint8)))
        ksk = np.zeros((self.N * KS_DIGITS, n + 1), np.uint32)
        ranges = [(k0, min(self.N, k0 + 32)) for k0 in range(0, self.N, 32)]
        _parallel(lambda r: lib().orc_ksk_gen(self.h, _p(s, i32p), s1.ctypes.data_as(C.POINTER(C.c_uint8)), n, seed,
                                              r[0], r[1], _p(ksk, u32p)), ranges)
        g = self.bsk_ctx()
        bsk = [None] * n
        _parallel(lambda i: bsk.__setitem__(i, g.enc_rgsw(s, int(s1[i]), seed, i)), range(n))
        return KsKey(n, s1, ksk, bsk, g)

    def gadget_ctx(self, log_base: int, digits: int) -> "Ctx":
        """the same ring, primes, p and sigma with another gadget (this
        context when it already has that one): RLWE and LWE ciphertexts are
        the same under both, RGSW and PackingKeySwitching keys follow it"""
        if (log_base, digits) == (self.log_base, self.digits):
            return self
        cache = self.__dict__.setdefault("_gadget_ctx", {})
        if (log_base, digits) not in cache:
            cache[(log_base, digits)] = Ctx(self.N, self.nq, self.p, primes=list(self.primes), log_base=log_base,
                                            digits=digits, sigma=self.sigma)
        return cache[(log_base, digits)]

    def bsk_ctx(self) -> "Ctx":
        """the same ring with the key-switched bootstrapping key's gadget:
        BSK_DIGITS balanced digits of BSK_LOG_BASE bits per prime when Q has
        two or more primes; the training gadget (this context) on a one-prime
        ring, whose 30-bit modulus leaves no room for the coarser digits'
        noise"""
        return self if self.nq < 2 else self.gadget_ctx(BSK_LOG_BASE, BSK_DIGITS)

    def pks_ctx(self) -> "Ctx":
        """the context of PackingKeySwitching: its decomposition has
        parameters of its own (the paper's TFHE parameter table lists them
        beside the RGSW gadget), here 5 balanced digits of 6 bits per prime
        whatever this context's RGSW gadget"""
        return self.gadget_ctx(PKS_LOG_BASE, PKS_DIGITS)

    def key_switch(self, key: "KsKey", lwe) -> np.ndarray:
        """the LWE (ring key, modulus Q) switched to key.s1 at modulus 2^32: [n + 1] uint32"""
        lwe = np.ascontiguousarray(lwe, np.uint32)
        out = np.zeros(key.n + 1, np.uint32)
        lib().orc_key_switch(self.h, _p(key.ksk, u32p), key.n, _p(lwe, u32p), _p(out, u32p))
        return out

    def pbs(self, bsk, lwe, n: int, V: int) -> np.ndarray:
        """programmable bootstrap with the constant test polynomial V: an LWE of
        V when the switched phase lies in [0, N), of -V otherwise.  bsk: the
        ring-key bootstrapping key (list of 2n RGSW; blind rotation over the
        first n ring-key coefficients) or a KsKey (key switch, then blind
        rotation over the binary key; n is then the key's)"""
        if isinstance(bsk, KsKey):
            lwe = np.ascontiguousarray(lwe, np.uint32)
            rg = [np.ascontiguousarray(r, np.uint32) for r in bsk.bsk]
            v = np.array([V % q for q in self.primes], np.uint64)
            out = np.zeros((self.nq, self.N + 1), np.uint32)
            lib().orc_pbs_ks(bsk.gctx.h, _ptr_array(rg), _p(bsk.ksk, u32p), bsk.n, _p(lwe, u32p), _p(v, u64p),
                             _p(out, u32p))
            return out
        lwe = np.ascontiguousarray(lwe, np.uint32)
        rg = [np.ascontiguousarray(r, np.uint32) for r in bsk[: 2 * n]]
        v = np.array([V % q for q in self.primes], np.uint64)
        out = np.zeros((self.nq, self.N + 1), np.uint32)
        lib().orc_pbs(self.h, _ptr_array(rg), _p(lwe, u32p), n, _p(v, u64p), _p(out, u32p))
        return out

    def rlwe_add(self, x, y) -> np.ndarray:
        """x + y over RLWE arrays of any leading shape (model merge, Sec. 3.7.2)"""
        x = np.ascontiguousarray(x, np.uint32)
        y = np.ascontiguousarray(y, np.uint32)
        assert x.shape == y.shape and x.size % (2 * self.nq * self.N) == 0
        out = np.zeros_like(x)
        lib().orc_rlwe_add_n(self.h, _p(x, u32p), _p(y, u32p), x.size // (2 * self.nq * self.N), _p(out, u32p))
        return out

    # -- PackingKeySwitching ----------------------------------------------
    def pks_keygen(self, s, seed: int, threads=None) -> np.ndarray:
        """K[j][r] = RLWE_s(s_j G_r) for j < N, r < D: [N][D][2][nq][N]
        (rows are independent; ranges of j go to threads), D = 5 nq: the
        gadget of pks_ctx()"""
        if self.pks_ctx() is not self:
            return self.pks_ctx().pks_keygen(s, seed, threads)
        s = np.ascontiguousarray(s, np.int32)
        K = np.zeros((self.N, self.D, 2, self.nq, self.N), np.uint32)
        ranges = [(j0, min(self.N, j0 + 64)) for j0 in range(0, self.N, 64)]
        _parallel(lambda r: lib().orc_pks_keygen(self.h, _p(s, i32p), seed, r[0], r[1], _p(K, u32p)), ranges,
                  threads)
        return K

    def pack_lwe(self, K, lwes, threads=None) -> np.ndarray:
        """one RLWE whose phase is sum_i phase(lwes[i]) X^i (k = len(lwes) <= N);
        the sum over key coordinates is split over threads"""
        if self.pks_ctx() is not self:
            return self.pks_ctx().pack_lwe(K, lwes, threads)
        K = np.ascontiguousarray(K, np.uint32)
        lwes = np.ascontiguousarray(lwes, np.uint32)
        k = lwes.shape[0]
        assert k <= self.N and lwes.shape[1:] == (self.nq, self.N + 1)
        step = 64
        ranges = [(j0, min(self.N, j0 + step)) for j0 in range(0, self.N, step)]
        parts = [self.rlwe() for _ in ranges]

        def run(t):
            j0, j1 = ranges[t]
            lib().orc_pks_partial(self.h, _p(K, u32p), _p(lwes, u32p), k, j0, j1, _p(parts[t], u32p))

        _parallel(run, range(len(ranges)), threads)
        acc = parts[0]
        for p in parts[1:]:
            acc = self.rlwe_add(acc, p)
        out = self.rlwe()
        lib().orc_pks_finish(self.h, _p(lwes, u32p), k, _p(acc, u32p), _p(out, u32p))
        return out

    def lwe_add(self, x, y) -> np.ndarray:
        x = np.ascontiguousarray(x, np.uint32)
        y = np.ascontiguousarray(y, np.uint32)
        out = np.zeros_like(x)
        lib().orc_lwe_add(self.h, _p(x, u32p), _p(y, u32p), _p(out, u32p))
        return out

    # -- WiSARD --------------------------------------------------------------
    def k1(self, s: int, l: int, a: int, layout: int = 0) -> int:
        """rows per RAM: layout 0 label-pruned (Def. 2), 1 and 2 class-packed
        (these need L = ceil(log2 l) <= log2 N, so that the tree holds tuple
        bits only)"""
        if layout and ceil_log2(l) > self.logN:
            raise ValueError("class-packed layouts need ceil(log2 l) <= log2 N")
        return int(lib().orc_k1_layout(self.h, s, l, a, layout))

    def train(self, s, l, a, pi, x_get, y_get, n, H, rams=None, threads=None, layout=0):
        """Alg. 6 over samples [0, n) for the RAMs in `rams` (default: all),
        accumulating into H ([k0][k1] RLWE, uint32).  x_get(i, k) returns the
        RGSW (numpy) of input bit k of sample i; y_get(i, u) that of label bit u.
        layout 0: label-pruned rows; 1: class-packed rows."""
        L = ceil_log2(l)
        self.k1(s, l, a, layout)  # rejects a class-packed layout the ring cannot hold
        k0 = -(-s // a)
        rams = list(range(k0)) if rams is None else list(rams)
        pi = np.ascontiguousarray(pi, np.uint32)
        keep = []

        def ptrs_for(j):
            xs = [None] * (n * s)
            for i in range(n):
                for t in range(min(a, s - j * a)):
                    k = int(pi[j * a + t])
                    r = x_get(i, k)
                    keep.append(r)
                    xs[i * s + k] = r
            ys = []
            for i in range(n):
                for u in range(L):
                    r = y_get(i, u)
                    keep.append(r)
                    ys.append(r)
            return _ptr_array(xs), _ptr_array(ys)

        def one(j):
            xp, yp = ptrs_for(j)
            lib().orc_train(self.h, s, l, a, _p(pi, u32p), xp, yp, n, j, j + 1, layout, _p(H, u32p))

        _parallel(one, rams, threads)
        return H

    def class_count(self, l, y_get, n, cnt):
        L = ceil_log2(l)
        ys = [y_get(i, u) for i in range(n) for u in range(L)]
        lib().orc_class_count(self.h, l, _ptr_array(ys), n, _p(cnt, u32p))
        return cnt

    def infer_one(self, s, l, a, pi, H, x_get, j, label) -> np.ndarray:
        """VP of RAM j for one sample and one label; x_get(k) -> RGSW of bit k."""
        pi = np.ascontiguousarray(pi, np.uint32)
        xs = [None] * s
        for t in range(min(a, s - j * a)):
            k = int(pi[j * a + t])
            xs[k] = np.ascontiguousarray(x_get(k), np.uint32)
        out = np.zeros((self.nq, self.N + 1), np.uint32)
        lib().orc_infer_one(self.h, s, l, a, _p(pi, u32p), _p(H, u32p), _ptr_array(xs), j, label,
                            _p(out, u32p))
        return out


    def rams_per_row(self, l: int, a: int) -> int:
        return int(lib().orc_rams_per_row(self.h, l, a))

    def model_rows(self, s: int, l: int, a: int, layout: int) -> int:
        return int(lib().orc_model_rows(self.h, s, l, a, layout))

    def pack_rams(self, s, l, a, H1) -> np.ndarray:
        """layout-2 rows from class-packed rows: row R = sum_t X^(t 2^(L+a)) H1[R r + t]"""
        H1 = np.ascontiguousarray(H1, np.uint32)
        k1 = self.k1(s, l, a, 1)
        out = np.zeros((self.model_rows(s, l, a, 2), k1, 2, self.nq, self.N), np.uint32)
        lib().orc_pack_rams(self.h, s, l, a, _p(H1, u32p), _p(out, u32p))
        return out

    def infer_packed(self, s, l, a, pi, H, x_get, j, layout=1) -> np.ndarray:
        """class-packed inference of RAM j for one sample: one VP, then the
        LWE of every class, [l][nq][N+1]; x_get(k) -> RGSW of bit k.  layout
        2 reads RAM j from its block of row j / r."""
        self.k1(s, l, a, layout)
        pi = np.ascontiguousarray(pi, np.uint32)
        xs = [None] * s
        for t in range(min(a, s - j * a)):
            k = int(pi[j * a + t])
            xs[k] = np.ascontiguousarray(x_get(k), np.uint32)
        out = np.zeros((l, self.nq, self.N + 1), np.uint32)
        lib().orc_infer_packed(self.h, s, l, a, _p(pi, u32p), _p(H, u32p), _ptr_array(xs), j, layout,
                               _p(out, u32p))
        return out


KS_LOG_BASE, KS_DIGITS = 4, 6  # the key switch's gadget (oracle.c)
PKS_LOG_BASE, PKS_DIGITS = 6, 5  # PackingKeySwitching's gadget (Ctx.pks_ctx)
# the gadget of the key-switched bootstrapping key's RGSW (its blind rotation's
# external products) on rings of two or more primes: 2 balanced digits of 15
# bits per prime (Ctx.bsk_ctx)
BSK_LOG_BASE, BSK_DIGITS = 15, 2


class KsKey:
    """bootstrapping key through a key switch: n, the binary LWE key s1, the
    key-switching key [N KS_DIGITS][n + 1] (uint32, modulus 2^32), the n
    RGSW(s1_i) and the context of their gadget"""

    def __init__(self, n, s1, ksk, bsk, gctx):
        self.n, self.s1, self.ksk, self.bsk, self.gctx = n, s1, ksk, bsk, gctx


def _parallel(fn, items, threads=None):
    items = list(items)
    if threads is None:
        threads = min(len(items), os.cpu_count() or 1, 16)
    if threads <= 1 or len(items) <= 1:
        for it in items:
            fn(it)
        return
    with ThreadPoolExecutor(threads) as ex:
        for f in [ex.submit(fn, it) for it in items]:
            f.result()
