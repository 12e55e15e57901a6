"""ctypes binding of libhwisard.so (C ABI in include/hwisard.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  Device buffers are torch tensors on the GPU (int32/int64
storage holding the ABI's uint32/uint64 words); work is enqueued on torch's
current stream.  The library must be built (``python -m
paper_2403_20190_amd.build``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhwisard.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhwisard.so is not built: run `python -m paper_2403_20190_amd.build` "
                      "(the encrypted WiSARD path has no CPU fallback)")

# One HIP runtime per process: load torch's runtime first, so that the
# library's libamdhip64.so.7 dependency resolves (by soname) to the copy torch
# uses for memory and streams instead of loading a second runtime.
import torch as _torch  # noqa: E402

if _torch.cuda.is_available():
    _torch.cuda.init()
_lib = C.CDLL(LIB_PATH)

HW_OK, HW_EINVAL, HW_ENOMEM, HW_EDEVICE, HW_EUNSUPPORTED, HW_EBUSY, HW_ECANCELLED = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "HW_OK", -1: "HW_EINVAL", -2: "HW_ENOMEM", -3: "HW_EDEVICE", -4: "HW_EUNSUPPORTED",
          -5: "HW_EBUSY", -6: "HW_ECANCELLED"}


class HwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


class Params(C.Structure):
    _fields_ = [("N", C.c_uint32), ("nq", C.c_uint32), ("primes", C.c_uint32 * 4), ("log_base", C.c_uint32),
                ("digits", C.c_uint32), ("sigma", C.c_double), ("plain_mod", C.c_uint64)]


class Shape(C.Structure):
    _fields_ = [("s", C.c_uint32), ("l", C.c_uint32), ("a", C.c_uint32), ("layout", C.c_uint32),
                ("perm_seed", C.c_uint64)]


class TrainJob(C.Structure):
    _fields_ = [("shape", Shape), ("x_rgsw", C.c_void_p), ("y_rgsw", C.c_void_p), ("n", C.c_uint64),
                ("model", C.c_void_p), ("class_count", C.c_void_p)]


class Job(C.Structure):
    """hw_job: one training (kind 0) or inference (kind 1) job of hw_batch_run"""
    _fields_ = [("ctx_index", C.c_uint32), ("kind", C.c_uint32), ("shape", Shape), ("x_rgsw", C.c_void_p),
                ("y_rgsw", C.c_void_p), ("n", C.c_uint64), ("model", C.c_void_p), ("class_count", C.c_void_p),
                ("ram_scores", C.c_void_p), ("class_scores", C.c_void_p)]


class EngineConfig(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("chunk", C.c_uint32), ("max_s", C.c_uint32), ("max_cells", C.c_uint32),
                ("arena_bytes", C.c_uint64), ("order", C.c_uint32), ("reserved", C.c_uint32)]


class BootKey(C.Structure):
    _fields_ = [("bsk", C.c_void_p), ("ksk", C.c_void_p), ("n", C.c_uint32), ("reserved", C.c_uint32)]


class KsBootKey:
    """a bootstrapping key through a key switch (hw_pbs_ks_keygen): the binary
    LWE key (uint8 [n]), its RGSW (bsk) and the key-switching key (ksk),
    device tensors"""

    def __init__(self, n, lwe_key, bsk, ksk):
        self.n, self.lwe_key, self.bsk, self.ksk = n, lwe_key, bsk, ksk


def _boot_key(bsk, n: int) -> BootKey:
    if isinstance(bsk, KsBootKey):
        return BootKey(bsk.bsk.data_ptr(), bsk.ksk.data_ptr(), bsk.n, 0)
    return BootKey(None if bsk is None else bsk.data_ptr(), None, n, 0)


class Request(C.Structure):
    _fields_ = [("job", C.c_uint32), ("kind", C.c_uint32), ("bits_host", C.c_void_p), ("labels_host", C.c_void_p),
                ("n", C.c_uint64), ("enc_seed", C.c_uint64), ("cells_host", C.c_void_p)]


NOALLOC_SCRATCH_BYTES = 256 << 20  # HW_NOALLOC_SCRATCH_BYTES
ACT_KINDS = {"ge": 0, "log": 1, "blog": 2}  # HW_ACT_GE, HW_ACT_LOG, HW_ACT_BLOG

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = 0, 1, 2, 3, 4

_vp, _u64, _u32, _i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
_SIG = {
    "hw_ctx_create": [C.POINTER(Params), _i32, C.POINTER(C.c_void_p)],
    "hw_ctx_params": [_vp, C.POINTER(Params)],
    "hw_sizes": [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64)],
    "hw_wisard_dims": [_vp, C.POINTER(Shape), C.POINTER(_u32), C.POINTER(_u32), C.POINTER(_u64)],
    "hw_permutation": [C.POINTER(Shape), _vp],
    "hw_wisard_model_rows": [_vp, C.POINTER(Shape), C.POINTER(_u32), C.POINTER(_u32)],
    "hw_wisard_pack_rams": [_vp, C.POINTER(Shape), _vp, _vp, _vp],
    "hw_keygen": [_vp, _u64, _vp, _vp],
    "hw_encrypt_rgsw_bits": [_vp, _vp, _vp, _u64, _u64, _u64, _vp, _vp],
    "hw_encrypt_rlwe": [_vp, _vp, _vp, _u64, _u64, _u64, _vp, _vp],
    "hw_decrypt_rlwe": [_vp, _vp, _vp, _u64, _vp, _vp],
    "hw_decrypt_lwe": [_vp, _vp, _vp, _u64, _vp, _vp],
    "hw_rgsw_export_canonical": [_vp, _vp, _u64, _vp, _vp],
    "hw_ntt": [_vp, _vp, _u64, _i32, _vp],
    "hw_external_product": [_vp, _vp, _vp, _u64, _vp, _vp],
    "hw_wisard_train_encrypted": [_vp, C.POINTER(Shape), _vp, _vp, _u64, _vp, _vp, _vp],
    "hw_wisard_train_encrypted_noalloc": [_vp, C.POINTER(Shape), _vp, _vp, _u64, _vp, _vp, _vp],
    "hw_wisard_infer_encrypted": [_vp, C.POINTER(Shape), _vp, _vp, _u64, _vp, _vp, _vp],
    "hw_rlwe_add": [_vp, _vp, _vp, _u64, _vp],
    "hw_pbs_keygen": [_vp, _vp, _u64, _u32, _vp, _vp],
    "hw_pbs": [_vp, _vp, _vp, _u64, _vp, _vp, _vp],
    "hw_activate_ge": [_vp, _vp, _vp, _u64, _u64, _u32, _vp, _vp],
    "hw_encrypted_argmax": [_vp, _vp, _vp, _u64, _u32, _u32, _vp, _vp],
    "hw_pbs_ks_sizes": [_vp, _u32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)],
    "hw_pbs_ks_keygen": [_vp, _vp, _u64, _u32, _vp, _vp, _vp, _vp],
    "hw_class_sums": [_vp, _vp, _u64, _u32, _u32, _vp, _vp],
    "hw_fm_act": [_vp, _vp, _vp, _vp, _vp, _u32, _u64, _u32, _vp, _vp],
    "hw_activate": [_vp, _vp, _vp, _u64, _u32, _u64, _u32, _vp, _vp],
    "hw_pks_keygen": [_vp, _vp, _u64, _vp, _vp],
    "hw_pks_key_export_canonical": [_vp, _vp, _vp, _vp],
    "hw_pack_lwe": [_vp, _vp, _vp, _u32, _u64, _vp, _vp],
    "hw_batch_train": [_vp, C.POINTER(TrainJob), _u32, _vp],
    "hw_batch_run": [C.POINTER(C.c_void_p), _u32, C.POINTER(Job), _u32, _vp],
    "hw_batch_plan_create": [_vp, C.POINTER(TrainJob), _u32, C.POINTER(C.c_void_p)],
    "hw_batch_plan_launch": [_vp, _vp],
    "hw_batch_plan_info": [_vp, C.POINTER(_u64), C.POINTER(_u32), C.POINTER(C.c_double), C.POINTER(_u64)],
    "hw_engine_create": [C.POINTER(Params), _i32, _vp, C.POINTER(EngineConfig), C.POINTER(C.c_void_p)],
    "hw_engine_add_job": [_vp, C.POINTER(Shape), _vp, _vp, _u64, C.POINTER(_u32)],
    "hw_engine_job_samples": [_vp, _u32, C.POINTER(_u64), C.POINTER(_u64)],
    "hw_request_seeds": [_u64, C.POINTER(_u64), C.POINTER(_u64)],
    "hw_microbench": [_i32, C.c_char_p, _u64, C.POINTER(C.c_double), C.POINTER(C.c_double), _vp],
    "hw_engine_submit": [_vp, C.POINTER(Request), C.POINTER(_u64)],
    "hw_engine_poll": [_vp, _u64, C.POINTER(_i32), C.POINTER(C.c_double)],
    "hw_engine_wait": [_vp, _u64, C.POINTER(_i32), C.POINTER(C.c_double)],
    "hw_engine_cancel": [_vp, _u64],
    "hw_engine_stats": [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u32)],
    "hw_tune_set": [_vp, C.c_char_p, _i32],
    "hw_tune_get": [_vp, C.c_char_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)],
    "hw_profile_enable": [_vp, _i32],
    "hw_profile_read": [_vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(_u64), C.POINTER(C.c_double)],
    "hw_profile_reset": [_vp],
}
for _n, _a in _SIG.items():
    _f = getattr(_lib, _n)
    _f.restype = C.c_int
    _f.argtypes = _a
_lib.hw_ctx_destroy.restype = None
_lib.hw_ctx_destroy.argtypes = [_vp]
_lib.hw_engine_destroy.restype = None
_lib.hw_engine_destroy.argtypes = [_vp]
_lib.hw_batch_plan_destroy.restype = None
_lib.hw_batch_plan_destroy.argtypes = [_vp]
_lib.hw_last_error.restype = C.c_char_p
_lib.hw_last_error.argtypes = []
_lib.hw_tune_variant_name.restype = C.c_char_p
_lib.hw_tune_variant_name.argtypes = [C.c_char_p, _i32]

TUNED_KERNELS = ("train", "infer", "train_batch", "infer_batch", "ntt", "ntt_inverse", "encrypt_rgsw")


def tune_variant_name(kernel: str, variant: int):
    r = _lib.hw_tune_variant_name(kernel.encode(), variant)
    return r.decode() if r else None


def exported_symbols():
    """Names the library exports (for the ABI test)."""
    return sorted(_SIG) + ["hw_ctx_destroy", "hw_engine_destroy", "hw_batch_plan_destroy", "hw_last_error",
                           "hw_tune_variant_name"]


def _check(st: int):
    if st != HW_OK:
        raise HwError(st, _lib.hw_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


LAYOUT_PRUNED, LAYOUT_PACKED, LAYOUT_RAM_PACKED = 0, 1, 2


def shape(s: int, l: int, a: int, perm_seed: int, layout: int = LAYOUT_PRUNED) -> Shape:
    """layout 0: label-pruned model rows (Def. 2); 1: class-packed rows (one
    VP per RAM at inference gives the scores of every class); 2: class-packed
    rows with several small RAMs per row"""
    return Shape(s, l, a, layout, perm_seed)


def permutation(sh: Shape) -> np.ndarray:
    out = np.zeros(max(1, sh.s), np.uint32)
    _check(_lib.hw_permutation(C.byref(sh), out.ctypes.data_as(C.c_void_p)))
    return out[:sh.s]


class Context:
    """One parameter set on one device (hw_ctx)."""

    def __init__(self, N: int, nq: int, p: int, primes=None, sigma: float = 3.2, device: int = 0,
                 log_base: int = 6, digits: int = 5):
        """(log_base, digits): the RGSW gadget, (6, 5) or, with nq >= 2, (15, 2)"""
        prm = Params()
        prm.N, prm.nq, prm.log_base, prm.digits, prm.sigma, prm.plain_mod = N, nq, log_base, digits, sigma, p
        for i, q in enumerate(primes or []):
            prm.primes[i] = q
        h = C.c_void_p()
        _check(_lib.hw_ctx_create(C.byref(prm), device, C.byref(h)))
        self._h = h
        out = Params()
        _check(_lib.hw_ctx_params(h, C.byref(out)))
        self.N, self.nq, self.p, self.device = N, nq, p, device
        self.log_base, self.digits = log_base, digits
        self.primes = [int(out.primes[i]) for i in range(nq)]
        k, r, g, w = _u64(), _u64(), _u64(), _u64()
        _check(_lib.hw_sizes(h, C.byref(k), C.byref(r), C.byref(g), C.byref(w)))
        self.sk_bytes = k.value
        self.rlwe_words, self.rgsw_words, self.lwe_words = r.value // 4, g.value // 4, w.value // 4

    def close(self):
        if getattr(self, "_h", None):
            _lib.hw_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry -------------------------------------------------------------
    def dims(self, sh: Shape):
        k0, k1, mb = _u32(), _u32(), _u64()
        _check(_lib.hw_wisard_dims(self._h, C.byref(sh), C.byref(k0), C.byref(k1), C.byref(mb)))
        return k0.value, k1.value, mb.value

    def model_rows(self, sh: Shape):
        """(rows of the model, RAMs per row)"""
        rows, rpr = _u32(), _u32()
        _check(_lib.hw_wisard_model_rows(self._h, C.byref(sh), C.byref(rows), C.byref(rpr)))
        return rows.value, rpr.value

    def pack_rams(self, sh: Shape, model_in, model_out):
        """layout-2 rows (sh.layout == 2) from the layout-1 rows of the same WiSARD"""
        _check(_lib.hw_wisard_pack_rams(self._h, C.byref(sh), _ptr(model_in), _ptr(model_out), _stream()))

    # -- client side ------------------------------------------------------------
    def keygen(self, seed: int, sk):
        _check(_lib.hw_keygen(self._h, seed, _ptr(sk), _stream()))

    def encrypt_rgsw_bits(self, sk, bits, seed: int, ct0: int, out):
        _check(_lib.hw_encrypt_rgsw_bits(self._h, _ptr(sk), _ptr(bits), bits.numel(), seed, ct0, _ptr(out),
                                         _stream()))

    def encrypt_rlwe(self, sk, msg, count: int, seed: int, ct0: int, out):
        _check(_lib.hw_encrypt_rlwe(self._h, _ptr(sk), _ptr(msg), count, seed, ct0, _ptr(out), _stream()))

    def decrypt_rlwe(self, sk, ct, count: int, out):
        _check(_lib.hw_decrypt_rlwe(self._h, _ptr(sk), _ptr(ct), count, _ptr(out), _stream()))

    def decrypt_lwe(self, sk, lwe, count: int, out):
        _check(_lib.hw_decrypt_lwe(self._h, _ptr(sk), _ptr(lwe), count, _ptr(out), _stream()))

    def rgsw_export(self, rgsw, count: int, out):
        _check(_lib.hw_rgsw_export_canonical(self._h, _ptr(rgsw), count, _ptr(out), _stream()))

    # -- ring / ciphertext kernels ------------------------------------------------
    def ntt(self, polys, count: int, inverse: bool):
        _check(_lib.hw_ntt(self._h, _ptr(polys), count, 1 if inverse else 0, _stream()))

    def external_product(self, rgsw, rin, count: int, rout):
        _check(_lib.hw_external_product(self._h, _ptr(rgsw), _ptr(rin), count, _ptr(rout), _stream()))

    # -- per-kernel timing ----------------------------------------------------------
    def profile(self, enable: bool = True):
        _check(_lib.hw_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, name: str):
        """(total ms, launches, algorithmic work) accumulated for kernel `name`"""
        ms, n, w = C.c_double(), _u64(), C.c_double()
        _check(_lib.hw_profile_read(self._h, name.encode(), C.byref(ms), C.byref(n), C.byref(w)))
        return ms.value, n.value, w.value

    def profile_reset(self):
        _check(_lib.hw_profile_reset(self._h))

    # -- server side ----------------------------------------------------------------
    def train(self, sh: Shape, x_rgsw, y_rgsw, n: int, model, class_count=None):
        _check(_lib.hw_wisard_train_encrypted(self._h, C.byref(sh), _ptr(x_rgsw), _ptr(y_rgsw), n, _ptr(model),
                                              _ptr(class_count), _stream()))

    def train_noalloc(self, sh: Shape, x_rgsw, y_rgsw, n: int, model, class_count=None):
        """train() through the entry point that allocates no device memory
        (a fixed library-held scratch; see NOALLOC_SCRATCH_BYTES)"""
        _check(_lib.hw_wisard_train_encrypted_noalloc(self._h, C.byref(sh), _ptr(x_rgsw), _ptr(y_rgsw), n,
                                                      _ptr(model), _ptr(class_count), _stream()))

    # -- programmable bootstrapping: Activate and EncryptedArgMax (OTF-act) --------
    def pbs_key_words(self, n: int) -> int:
        """uint32 words of a bootstrapping key for the first n key coefficients"""
        return 2 * n * self.rgsw_words

    def pbs_keygen(self, sk, seed: int, n: int, bsk):
        _check(_lib.hw_pbs_keygen(self._h, _ptr(sk), seed, n, _ptr(bsk), _stream()))

    def pbs_ks_keygen(self, sk, seed: int, n: int, device: str = "cuda") -> "KsBootKey":
        """bootstrapping key through a key switch to a binary LWE key of n
        coefficients (device tensors allocated here)"""
        import torch
        bb, kb = _u64(), _u64()
        _check(_lib.hw_pbs_ks_sizes(self._h, n, C.byref(bb), C.byref(kb)))
        lwe_key = torch.zeros(n, dtype=torch.uint8, device=device)
        bsk = torch.empty(bb.value // 4, dtype=torch.int32, device=device)
        ksk = torch.empty(kb.value, dtype=torch.int8, device=device)
        _check(_lib.hw_pbs_ks_keygen(self._h, _ptr(sk), seed, n, _ptr(lwe_key), _ptr(bsk), _ptr(ksk), _stream()))
        return KsBootKey(n, lwe_key, bsk, ksk)

    def pbs(self, bsk, n: int, lwe, count: int, V: int, out):
        """bootstrap with the constant test polynomial V (an integer below Q).
        bsk: a ring-key bootstrapping key (device tensor, n its coefficients)
        or a KsBootKey (n is then the key's)"""
        v = np.array([V % q for q in self.primes], np.uint32)
        k = _boot_key(bsk, n)
        _check(_lib.hw_pbs(self._h, C.byref(k), _ptr(lwe), count, v.ctypes.data_as(C.c_void_p), _ptr(out),
                           _stream()))

    def activate_ge(self, bsk, n: int, lwe, count: int, T: int, log_p_out: int, out):
        k = _boot_key(bsk, n)
        _check(_lib.hw_activate_ge(self._h, C.byref(k), _ptr(lwe), count, T, log_p_out, _ptr(out), _stream()))

    def class_sums(self, scores, n: int, l: int, k0: int, sums):
        _check(_lib.hw_class_sums(self._h, _ptr(scores), n, l, k0, _ptr(sums), _stream()))

    def activate(self, bsk, n: int, lwe, count: int, kind: str, param: int, log_p_out: int, out):
        """kind "ge" ([m >= param]), "log" (floor(log2(m + 1))) or "blog"
        (min(log, param)) over `count` LWE, output modulus 2^log_p_out"""
        k = _boot_key(bsk, n)
        _check(_lib.hw_activate(self._h, C.byref(k), _ptr(lwe), count, ACT_KINDS[kind], param, log_p_out,
                                _ptr(out), _stream()))

    def fm_act(self, sh: Shape, bsk, n: int, pks_key, model, kind: str, param: int, log_p_out: int, out):
        """FM-act: every cell of `model` activated (kind and param as in
        activate, output modulus 2^log_p_out) and packed back into its row;
        out may be model"""
        k = _boot_key(bsk, n)
        _check(_lib.hw_fm_act(self._h, C.byref(sh), C.byref(k), _ptr(pks_key), _ptr(model), ACT_KINDS[kind],
                              param, log_p_out, _ptr(out), _stream()))

    def encrypted_argmax(self, bsk, n: int, u, count: int, l: int, log_p_in: int, out):
        k = _boot_key(bsk, n)
        _check(_lib.hw_encrypted_argmax(self._h, C.byref(k), _ptr(u), count, l, log_p_in, _ptr(out), _stream()))

    @property
    def pks_key_words(self) -> int:
        """uint32 words of a PackingKeySwitching key: N x D rows"""
        return self.N * 5 * self.nq * self.rlwe_words

    def pks_keygen(self, sk, seed: int, key):
        _check(_lib.hw_pks_keygen(self._h, _ptr(sk), seed, _ptr(key), _stream()))

    def pks_key_export(self, key, out):
        _check(_lib.hw_pks_key_export_canonical(self._h, _ptr(key), _ptr(out), _stream()))

    def pack_lwe(self, key, lwe, k: int, count: int, out):
        """out[c] = PackingKeySwitching(lwe[c][0 .. k)) for c < count"""
        _check(_lib.hw_pack_lwe(self._h, _ptr(key), _ptr(lwe), k, count, _ptr(out), _stream()))

    def rlwe_add(self, dst, src, count: int):
        """dst += src over count RLWE ciphertexts (model merge, Sec. 3.7.2)"""
        _check(_lib.hw_rlwe_add(self._h, _ptr(dst), _ptr(src), count, _stream()))

    def batch_train(self, jobs):
        """jobs: iterable of (shape, x_rgsw, y_rgsw, n, model, class_count) -- one
        persistent launch over a queue of (job, RAM, piece of samples) items"""
        jobs = list(jobs)
        arr = (TrainJob * max(1, len(jobs)))()
        for i, (sh, x, y, n, model, cnt) in enumerate(jobs):
            arr[i] = TrainJob(sh, _ptr(x), _ptr(y), n, _ptr(model), _ptr(cnt))
        _check(_lib.hw_batch_train(self._h, arr, len(jobs), _stream()))

    def tune_set(self, kernel: str, variant: int):
        """force a schedule variant of a tuned kernel (-1: tune again)"""
        _check(_lib.hw_tune_set(self._h, kernel.encode(), variant))

    def tune_get(self, kernel: str):
        """(variant in use or -1 while tuning, timings taken, variants)"""
        v, t, n = _i32(), _i32(), _i32()
        _check(_lib.hw_tune_get(self._h, kernel.encode(), C.byref(v), C.byref(t), C.byref(n)))
        return v.value, t.value, n.value

    def schedule(self):
        """{kernel: description of the variant in use, or None while tuning}"""
        out = {}
        for k in TUNED_KERNELS:
            v, _, _ = self.tune_get(k)
            out[k] = tune_variant_name(k, v) if v >= 0 else None
        return out

    def batch_plan(self, jobs):
        """A BatchPlan for the jobs of batch_train: launches captured once into
        a HIP graph, replayed with plan.launch()."""
        return BatchPlan(self, jobs)

    def infer(self, sh: Shape, model, x_rgsw, n: int, ram_scores, class_scores=None):
        _check(_lib.hw_wisard_infer_encrypted(self._h, C.byref(sh), _ptr(model), _ptr(x_rgsw), n,
                                              _ptr(ram_scores), _ptr(class_scores), _stream()))


def request_seeds(enc_seed: int):
    """(seed_x, seed_y): the encryption seeds the serving engine derives from
    a request's enc_seed for its input and label bits"""
    a, b = _u64(), _u64()
    _check(_lib.hw_request_seeds(enc_seed, C.byref(a), C.byref(b)))
    return a.value, b.value


def microbench(kind: str, size: int = 0, device: int = 0):
    """(rate, best ms) of a device peak probe: "triad" (bytes/s over three
    arrays of `size` bytes) or one of "v_add_u32", "v_mul_lo_u32",
    "v_mul_hi_u32", "v_mad_u64_u32" (lane-instructions/s; size = loop trips)"""
    r, ms = C.c_double(), C.c_double()
    _check(_lib.hw_microbench(device, kind.encode(), size, C.byref(r), C.byref(ms), _stream()))
    return r.value, ms.value


def batch_run(ctxs, jobs):
    """hw_batch_run.  ctxs: list of Context; jobs: dicts with ctx (index),
    kind ("train" | "infer"), shape, x, n and: train -- y, model, cnt (optional);
    infer -- model, scores, sums (optional)."""
    ctxs = list(ctxs)
    jobs = list(jobs)
    harr = (C.c_void_p * max(1, len(ctxs)))(*[c._h for c in ctxs])
    arr = (Job * max(1, len(jobs)))()
    for i, J in enumerate(jobs):
        train = J["kind"] == "train"
        arr[i] = Job(J.get("ctx", 0), 0 if train else 1, J["shape"], _ptr(J["x"]), _ptr(J.get("y")), J["n"],
                     _ptr(J["model"]), _ptr(J.get("cnt")), _ptr(J.get("scores")), _ptr(J.get("sums")))
    _check(_lib.hw_batch_run(harr, len(ctxs), arr, len(jobs), _stream()))


class BatchPlan:
    """hw_batch_plan_*: the queue of a batch computed once and captured into
    a HIP graph; launch() replays it on the current stream.  The job buffers
    are kept referenced here for the plan's lifetime."""

    def __init__(self, ctx: "Context", jobs):
        jobs = list(jobs)
        arr = (TrainJob * max(1, len(jobs)))()
        for i, (sh, x, y, n, model, cnt) in enumerate(jobs):
            arr[i] = TrainJob(sh, _ptr(x), _ptr(y), n, _ptr(model), _ptr(cnt))
        h = C.c_void_p()
        _check(_lib.hw_batch_plan_create(ctx._h, arr, len(jobs), C.byref(h)))
        self._h, self._ctx, self._jobs = h, ctx, jobs
        it, mp, xp, ws = _u64(), _u32(), C.c_double(), _u64()
        _check(_lib.hw_batch_plan_info(h, C.byref(it), C.byref(mp), C.byref(xp), C.byref(ws)))
        self.items, self.max_pieces, self.external_products, self.workspace_bytes = (
            it.value, mp.value, xp.value, ws.value)

    def launch(self):
        _check(_lib.hw_batch_plan_launch(self._h, _stream()))

    def close(self):
        if self._h:
            _lib.hw_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Serving engine (hw_engine_*): continuous batching of train / infer
    requests against resident models.  Host buffers handed to submit() are
    kept alive here until the request has finished."""

    def __init__(self, N: int, nq: int, p: int, sk, slots: int = 4, chunk: int = 8, max_s: int = 4096,
                 max_cells: int = 4096, arena_bytes: int = 32 << 30, device: int = 0, sigma: float = 3.2,
                 order: str = "fifo", log_base: int = 6, digits: int = 5):
        """order: "fifo" (submission order) or "shortest" (least remaining work
        first); (log_base, digits): the RGSW gadget, as for Context"""
        prm = Params()
        prm.N, prm.nq, prm.log_base, prm.digits, prm.sigma, prm.plain_mod = N, nq, log_base, digits, sigma, p
        if order not in ("fifo", "shortest"):
            raise HwError(HW_EINVAL, "order must be 'fifo' or 'shortest'")
        cfg = EngineConfig(slots, chunk, max_s, max_cells, arena_bytes, 0 if order == "fifo" else 1, 0)
        h = C.c_void_p()
        _check(_lib.hw_engine_create(C.byref(prm), device, _ptr(sk), C.byref(cfg), C.byref(h)))
        self._h = h
        self._sk = sk
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.hw_engine_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_job(self, sh: Shape, model, class_count=None, trained: int = 0) -> int:
        """register a resident model that already holds `trained` samples"""
        j = _u32()
        _check(_lib.hw_engine_add_job(self._h, C.byref(sh), _ptr(model), _ptr(class_count), trained, C.byref(j)))
        L = max(0, int(sh.l - 1).bit_length())
        k0 = -(-sh.s // sh.a)
        self._keep[("job", j.value)] = (model, class_count, (sh.s, L, sh.l, k0))
        return j.value

    def job_samples(self, job: int):
        """(samples counted against the model, capacity p - 1)"""
        n, cap = _u64(), _u64()
        _check(_lib.hw_engine_job_samples(self._h, job, C.byref(n), C.byref(cap)))
        return n.value, cap.value

    def submit(self, job: int, kind: str, bits: np.ndarray, enc_seed: int, labels: np.ndarray = None,
               cells: np.ndarray = None) -> int:
        """bits: uint8 [n][s]; train: labels uint8 [n][L]; infer: cells uint64 [n][l][k0] (written)"""
        if ("job", job) not in self._keep:
            raise HwError(HW_EINVAL, "unknown job %d" % job)
        if kind not in ("train", "infer"):
            raise HwError(HW_EINVAL, "kind must be 'train' or 'infer'")
        s, L, l, k0 = self._keep[("job", job)][2]
        bits = np.ascontiguousarray(bits, np.uint8)
        if bits.ndim != 2 or bits.shape[1] != s or bits.shape[0] < 1:
            raise HwError(HW_EINVAL, "bits must be uint8 [n][s = %d], got shape %s" % (s, bits.shape))
        n = bits.shape[0]
        if kind == "train":
            labels = np.ascontiguousarray(labels if labels is not None else np.zeros((n, 0)), np.uint8)
            if labels.shape != (n, L):
                raise HwError(HW_EINVAL, "labels must be uint8 [n][L = %d], got shape %s" % (L, labels.shape))
            if cells is not None:
                raise HwError(HW_EINVAL, "a training request has no output cells")
        else:
            if labels is not None:
                raise HwError(HW_EINVAL, "an inference request has no labels")
            if (not isinstance(cells, np.ndarray) or cells.dtype != np.uint64 or cells.shape != (n, l, k0)
                    or not cells.flags.c_contiguous or not cells.flags.writeable):
                raise HwError(HW_EINVAL, "cells must be a writable C-contiguous uint64 array [n][l = %d][k0 = %d]"
                              % (l, k0))
        r = Request(job, 0 if kind == "train" else 1, bits.ctypes.data,
                    None if labels is None or labels.size == 0 else labels.ctypes.data, n, enc_seed,
                    None if cells is None else cells.ctypes.data)
        rid = _u64()
        _check(_lib.hw_engine_submit(self._h, C.byref(r), C.byref(rid)))
        self._keep[rid.value] = (bits, labels, cells)
        return rid.value

    def poll(self, rid: int):
        st, lat = _i32(), C.c_double()
        _check(_lib.hw_engine_poll(self._h, rid, C.byref(st), C.byref(lat)))
        return st.value, lat.value

    def wait(self, rid: int):
        st, lat = _i32(), C.c_double()
        _check(_lib.hw_engine_wait(self._h, rid, C.byref(st), C.byref(lat)))
        self._keep.pop(rid, None)
        return st.value, lat.value

    def cancel(self, rid: int):
        _check(_lib.hw_engine_cancel(self._h, rid))

    def stats(self):
        c, pk, pi = _u64(), _u64(), _u32()
        _check(_lib.hw_engine_stats(self._h, C.byref(c), C.byref(pk), C.byref(pi)))
        return {"chunks": c.value, "peak_arena_bytes": pk.value, "peak_inflight": pi.value}
