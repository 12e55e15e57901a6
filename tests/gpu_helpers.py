"""Helpers for the GPU parity tests: torch device buffers holding the ABI's
uint32/uint64 words, and a paired set-up that runs the same seeded workload
through the HIP library and through the CPU oracle independently."""
from __future__ import annotations

import numpy as np

import oracle as O


def dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}.get(a.dtype, a.dtype)
    return torch.from_numpy(a.view(view)).cuda()


def zeros_u32(*shape):
    import torch
    return torch.zeros(shape, dtype=torch.int32, device="cuda")


def zeros_u64(*shape):
    import torch
    return torch.zeros(shape, dtype=torch.int64, device="cuda")


def host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def host_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def label_bits_np(y, L):
    return np.array([[(int(v) >> u) & 1 for u in range(L)] for v in y], np.uint8).reshape(len(y), L)


class Pair:
    """Seeded WiSARD workload on both sides.  Seeds: key, input-bit
    encryption, label-bit encryption, permutation."""

    def __init__(self, N, nq, p, s, l, a, X, y, seed=7, layout=0, gadget=(6, 5)):
        from paper_2403_20190_amd import hwisard as HW
        self.HW = HW
        self.N, self.nq, self.p, self.s, self.l, self.a = N, nq, p, s, l, a
        self.X, self.y = np.asarray(X, np.uint8), np.asarray(y, np.int64)
        self.n = len(self.X)
        self.L = O.ceil_log2(l)
        self.seed_key, self.seed_x, self.seed_y, self.seed_perm = seed * 4 + 1, seed * 4 + 2, seed * 4 + 3, seed * 4 + 4
        self.ctx = HW.Context(N, nq, p, log_base=gadget[0], digits=gadget[1])
        self.orc = O.Ctx(N, nq, p, log_base=gadget[0], digits=gadget[1])
        self.layout = layout
        self.shape = HW.shape(s, l, a, self.seed_perm, layout)
        self.k0, self.k1, _ = self.ctx.dims(self.shape)
        self.pi = O.permutation(self.seed_perm, s)
        self.sk_o = self.orc.keygen(self.seed_key)
        self.sk = zeros_u32(N)
        self.ctx.keygen(self.seed_key, self.sk)
        self._xo = {}
        self._yo = {}

    # device side ------------------------------------------------------------
    def encrypt_dev(self, X=None, seed_x=None):
        X = self.X if X is None else X
        xb = dev(np.ascontiguousarray(X, np.uint8).reshape(-1))
        xr = zeros_u32(xb.numel(), self.ctx.rgsw_words)
        self.ctx.encrypt_rgsw_bits(self.sk, xb, self.seed_x if seed_x is None else seed_x, 0, xr)
        return xr

    def encrypt_labels_dev(self):
        if self.L == 0:
            return None
        yb = dev(label_bits_np(self.y, self.L).reshape(-1))
        yr = zeros_u32(yb.numel(), self.ctx.rgsw_words)
        self.ctx.encrypt_rgsw_bits(self.sk, yb, self.seed_y, 0, yr)
        return yr

    # oracle side (encrypts only what it needs, with the same draw indices) -----
    def xo(self, i, k, X=None, seed_x=None, tag="train"):
        X = self.X if X is None else X
        key = (tag, i, k)
        if key not in self._xo:
            self._xo[key] = self.orc.enc_rgsw(self.sk_o, int(X[i][k]), self.seed_x if seed_x is None else seed_x,
                                              i * self.s + k)
        return self._xo[key]

    def yo(self, i, u):
        key = (i, u)
        if key not in self._yo:
            self._yo[key] = self.orc.enc_rgsw(self.sk_o, (int(self.y[i]) >> u) & 1, self.seed_y, i * self.L + u)
        return self._yo[key]

    def oracle_train(self, rams, n=None):
        n = self.n if n is None else n
        H = np.zeros((self.k0, self.k1, 2, self.nq, self.N), np.uint32)
        # encrypt in parallel first (the oracle's own ciphertexts)
        need = [(i, int(self.pi[j * self.a + t])) for j in rams for i in range(n)
                for t in range(min(self.a, self.s - j * self.a))]
        O._parallel(lambda ik: self.xo(*ik), need)
        O._parallel(lambda iu: self.yo(*iu), [(i, u) for i in range(n) for u in range(self.L)])
        self.orc.train(self.s, self.l, self.a, self.pi, self.xo, self.yo, n, H, rams=rams, layout=self.layout)
        return H
