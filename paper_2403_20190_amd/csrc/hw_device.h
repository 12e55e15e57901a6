// hw_device.h -- device building blocks for gfx950: modular arithmetic on
// 32-bit lanes, the workgroup-wide negacyclic NTT and the fused external
// product (decompose -> NTT -> multiply-accumulate -> inverse NTT).
//
// Ring R_q = Z_q[X]/(X^N+1) (Sec. 2.1); external product of Sec. 2.5.1 with
// an RNS gadget of base 2^6 and 5 digits per prime, or (rings of two or more
// primes) of base 2^15 and 2 digits.
//
// Thread mapping.  One workgroup of T = N/8 threads owns one polynomial at a
// time; each thread keeps 8 coefficients in registers.  The NTT's log2 N
// stages are split into four phases of at most three stages; inside a phase
// every butterfly is thread-local (radix-8 on registers), and between phases
// the coefficients are exchanged through LDS.  In phase P a thread holds the
// 8 elements whose indices differ only in three consecutive bits:
//   P=0 (natural layout): k = t + T e
//   P=1: bits N/8..N/64 vary, P=2: bits N/512..N/4096 vary
//   P=3: k = 8t + e (the evaluation-domain layout used for all pointwise work)
// The LDS index k + 4*(k>>5) keeps every exchange free of bank conflicts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hw {

// ---------------------------------------------------------------------------
// per-prime constants and tables
// ---------------------------------------------------------------------------

struct PrimeTab {
  uint32_t q, two_q;
  uint32_t ninv, ninv_sh;   // N^{-1} mod q and its Shoup companion
  uint32_t r32, r32_sh;     // 2^32 mod q and companion
  uint32_t one_sh;          // floor(2^32 / q): Shoup companion of 1
  uint32_t delta;           // Delta mod q
};

constexpr int MAXQ = 3;

struct Tabs {
  PrimeTab pt[MAXQ];
  const uint2* fwd[MAXQ];   // [N]: (-psi^{brv(k)} mod 2^32, Shoup companion of psi^{brv(k)}), k >= 1
  const uint2* inv[MAXQ];   // [N]: (psi^{-brv(k)}, Shoup companion)
  const uint2* evx[MAXQ];   // [N]: the forward transform of X, psi^{2 brv(k) + 1}, with its Shoup companion
};

// ---------------------------------------------------------------------------
// modular arithmetic (q < 2^30, lazily reduced values below 4q < 2^32)
// ---------------------------------------------------------------------------

// a * b + c on 64 bits in one VALU instruction (v_mad_u64_u32, full rate on
// gfx950).  In asm because the compiler narrows a product whose high half is
// unused to mul_lo + add and splits a full product into mul_lo + mul_hi.
__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t d, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a), "v"(b), "v"(c));
  return d;
}

// x * w mod q in [0, 2q) for any 32-bit x (Shoup's method, w < q):
// x w - floor(x wsh / 2^32) q, the subtraction folded into a multiply-add
// with 2^32 - q (only the low 32 bits are kept)
__device__ __forceinline__ uint32_t mulsh(uint32_t x, uint32_t w, uint32_t wsh, uint32_t q) {
  const uint32_t qh = __umulhi(x, wsh);
  return (uint32_t)mad64(qh, 0u - q, (uint64_t)(x * w));
}

// [0, 2m) -> [0, m) for m < 2^31: min(x, x - m) picks x - m exactly when x >= m
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) { return min(x, x - m); }

__device__ __forceinline__ uint32_t addq(uint32_t a, uint32_t b, uint32_t q) { return csub(a + b, q); }
__device__ __forceinline__ uint32_t subq(uint32_t a, uint32_t b, uint32_t q) { return csub(a + q - b, q); }

// 64-bit value -> [0, q)
__device__ __forceinline__ uint32_t red64(uint64_t v, const PrimeTab& P) {
  const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  uint32_t r = mulsh(hi, P.r32, P.r32_sh, P.q) + mulsh(lo, 1u, P.one_sh, P.q);  // [0, 4q)
  return csub(csub(r, P.two_q), P.q);
}

// data x data product mod q, both in [0, q)
__device__ __forceinline__ uint32_t mulq(uint32_t a, uint32_t b, const PrimeTab& P) {
  return red64((uint64_t)a * b, P);
}

// -(y w mod q) mod 2^32 with y w mod q in [0, 2q) as in mulsh, from nw =
// -w mod 2^32 and w's Shoup companion: floor(y wsh / 2^32) q - y w, one
// multiply-add with q (only the low 32 bits are kept)
__device__ __forceinline__ uint32_t mulsh_neg(uint32_t y, uint32_t nw, uint32_t wsh, uint32_t q) {
  const uint32_t qh = __umulhi(y, wsh);
  return (uint32_t)mad64(qh, q, (uint64_t)(y * nw));
}

// Harvey butterflies: forward (Cooley-Tukey) on [0, 4q), inverse
// (Gentleman-Sande) on [0, 2q).  The forward twiddles come as (-w mod 2^32,
// Shoup companion of w): with nt = -t for the product t in [0, 2q),
// X + t = X - nt and X - t + 2q = X + 2q + nt, one subtraction and one
// three-operand add.  bf_fwd0 is the forward butterfly for an upper input
// already below 2q (the first stage: transform inputs are < 2q).
__device__ __forceinline__ void bf_fwd0(uint32_t& X, uint32_t& Y, uint32_t nw, uint32_t wsh, uint32_t q,
                                        uint32_t two_q) {
  const uint32_t x = X;
  const uint32_t nt = mulsh_neg(Y, nw, wsh, q);
  X = x - nt;
  Y = x + two_q + nt;
}

__device__ __forceinline__ void bf_fwd(uint32_t& X, uint32_t& Y, uint32_t nw, uint32_t wsh, uint32_t q,
                                       uint32_t two_q) {
  X = csub(X, two_q);
  bf_fwd0(X, Y, nw, wsh, q, two_q);
}

__device__ __forceinline__ void bf_inv(uint32_t& X, uint32_t& Y, uint32_t w, uint32_t wsh, uint32_t q,
                                       uint32_t two_q) {
  const uint32_t x = X, y = Y;
  X = csub(x + y, two_q);
  Y = mulsh(x - y + two_q, w, wsh, q);
}

// ---------------------------------------------------------------------------
// layouts
// ---------------------------------------------------------------------------

template <int LOGN>
struct Geo {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = N / 8;            // threads per polynomial
  static constexpr int R = LOGN - 9;         // stages in the last phase (1..3)
  static constexpr int LDSW = N + N / 8;     // padded words of one exchange buffer
  static_assert(LOGN >= 10 && LOGN <= 12, "N must be 1024, 2048 or 4096");
};

// Whether ext_prod transforms its digit polynomials two at a time: where
// the LDS of a second pair of exchange buffers still leaves room for the
// workgroups per CU the kernels run at (three at N = 2048; at N = 4096 two
// 512-thread workgroups would no longer fit), and with more than one prime
// (with one, the compiler's schedule of the pair spills registers).
template <int LOGN, int NQ>
__host__ __device__ constexpr bool xp_pair() { return LOGN <= 11 && NQ > 1; }

// exchange words (two buffers per polynomial in flight) of a kernel whose
// ext_prod runs with (PR) or without pairs
template <int LOGN, bool PR>
__host__ __device__ constexpr int xp_words() { return (PR ? 4 : 2) * Geo<LOGN>::LDSW; }

__host__ __device__ constexpr uint32_t lds_ix(uint32_t k) { return k + ((k >> 5) << 2); }

// In layouts P = 0..2 the index of element e of thread t splits into two
// disjoint bit fields, k = tpart(t) | (e << eshift), so its LDS index is
// lds_ix(tpart) + lds_ix(e << eshift): one base register plus an immediate.
template <int LOGN, int P>
__host__ __device__ constexpr int eshift() {
  return P == 0 ? LOGN - 3 : (P == 1 ? LOGN - 6 : LOGN - 9);
}

template <int LOGN, int P>
__device__ __forceinline__ uint32_t tpart(uint32_t t) {
  if constexpr (P == 0) {
    return t;
  } else {
    constexpr int b = eshift<LOGN, P>();
    return ((t >> b) << (b + 3)) | (t & ((1u << b) - 1));
  }
}

template <int LOGN, int P>
__device__ __forceinline__ uint32_t pos(uint32_t t, uint32_t e) {
  if constexpr (P == 3) return (t << 3) | e;
  else return tpart<LOGN, P>(t) | (e << eshift<LOGN, P>());
}

// Exchange through LDS from layout PF to layout PT.  Two buffers alternate
// (selected by the running counter xc) so that one barrier per exchange
// suffices: a buffer is written again only after the next exchange's barrier.
// K polynomials pass through one exchange; polynomial k uses the buffer of
// the running parity 2 k LDSW words further on, so the buffers of
// consecutive exchanges stay disjoint whatever their K.
template <int LOGN, int PF>
__device__ __forceinline__ void xput(const uint32_t (&x)[8], uint32_t* buf, uint32_t t) {
  if constexpr (PF == 3) {
    uint4* p = reinterpret_cast<uint4*>(buf + lds_ix(t << 3));
    p[0] = make_uint4(x[0], x[1], x[2], x[3]);
    p[1] = make_uint4(x[4], x[5], x[6], x[7]);
  } else {
    uint32_t* b = buf + lds_ix(tpart<LOGN, PF>(t));
#pragma unroll
    for (int e = 0; e < 8; ++e) b[lds_ix((uint32_t)e << eshift<LOGN, PF>())] = x[e];
  }
}

template <int LOGN, int PT>
__device__ __forceinline__ void xget(uint32_t (&x)[8], const uint32_t* buf, uint32_t t) {
  if constexpr (PT == 3) {
    const uint4* p = reinterpret_cast<const uint4*>(buf + lds_ix(t << 3));
    const uint4 u = p[0], v = p[1];
    x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w;
    x[4] = v.x; x[5] = v.y; x[6] = v.z; x[7] = v.w;
  } else {
    const uint32_t* b = buf + lds_ix(tpart<LOGN, PT>(t));
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = b[lds_ix((uint32_t)e << eshift<LOGN, PT>())];
  }
}

template <int LOGN, int PF, int PT, int K>
__device__ __forceinline__ void xchg_k(uint32_t (&x)[K][8], uint32_t* lds, uint32_t& xc, uint32_t t) {
  uint32_t* buf = lds + (xc & 1u) * Geo<LOGN>::LDSW;
  ++xc;
#pragma unroll
  for (int k = 0; k < K; ++k) xput<LOGN, PF>(x[k], buf + 2 * k * Geo<LOGN>::LDSW, t);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) xget<LOGN, PT>(x[k], buf + 2 * k * Geo<LOGN>::LDSW, t);
}

template <int LOGN, int PF, int PT>
__device__ __forceinline__ void xchg(uint32_t (&x)[8], uint32_t* lds, uint32_t& xc, uint32_t t) {
  xchg_k<LOGN, PF, PT, 1>(*reinterpret_cast<uint32_t(*)[1][8]>(&x), lds, xc, t);
}

// ---------------------------------------------------------------------------
// forward NTT (natural layout in registers -> layout P=3)
// ---------------------------------------------------------------------------
// Stage s (0 <= s < log2 N) pairs elements at distance N >> (s+1); the pair
// whose lower element has index k uses psi^{brv(2^s + (k >> (log2 N - s)))}.

// Twiddles of phase 0 are uniform over the workgroup and read from the global
// table (scalar loads); those of phases 1..3 are read from a copy of the
// prime's table in LDS (`twl`, N entries), a few per phase.

// copy the forward table of one prime into LDS (caller synchronises after)
template <int LOGN>
__device__ __forceinline__ void load_tw_lds(uint2* __restrict__ twl, const uint2* __restrict__ tab, uint32_t t) {
  constexpr int TT = Geo<LOGN>::T;
  const uint4* src = reinterpret_cast<const uint4*>(tab);
  uint4* dst = reinterpret_cast<uint4*>(twl);
#pragma unroll
  for (int e = 0; e < 4; ++e) (dst + TT * e)[t] = (src + TT * e)[t];
}

// three forward stages with twiddle (-w, Shoup) pairs w0 | w1,w2 | w3..w6
__device__ __forceinline__ void fwd8(uint32_t (&x)[8], const uint2 (&w)[7], uint32_t q, uint32_t two_q) {
#pragma unroll
  for (int e = 0; e < 4; ++e) bf_fwd(x[e], x[e + 4], w[0].x, w[0].y, q, two_q);
  bf_fwd(x[0], x[2], w[1].x, w[1].y, q, two_q);
  bf_fwd(x[1], x[3], w[1].x, w[1].y, q, two_q);
  bf_fwd(x[4], x[6], w[2].x, w[2].y, q, two_q);
  bf_fwd(x[5], x[7], w[2].x, w[2].y, q, two_q);
#pragma unroll
  for (int e = 0; e < 4; ++e) bf_fwd(x[2 * e], x[2 * e + 1], w[3 + e].x, w[3 + e].y, q, two_q);
}

// the seven twiddles of a radix-8 phase whose stage s0 index base is b0:
// 2^s0 + h, 2^{s0+1} + 2h + {0,1}, 2^{s0+2} + 4h + {0..3}
__device__ __forceinline__ void tw_phase(uint2 (&w)[7], const uint2* __restrict__ twl, uint32_t s0, uint32_t h) {
  w[0] = twl[(1u << s0) + h];
  const uint4 v = *reinterpret_cast<const uint4*>(twl + (2u << s0) + 2 * h);
  w[1] = make_uint2(v.x, v.y);
  w[2] = make_uint2(v.z, v.w);
  const uint4 u0 = *reinterpret_cast<const uint4*>(twl + (4u << s0) + 4 * h);
  const uint4 u1 = *reinterpret_cast<const uint4*>(twl + (4u << s0) + 4 * h + 2);
  w[3] = make_uint2(u0.x, u0.y);
  w[4] = make_uint2(u0.z, u0.w);
  w[5] = make_uint2(u1.x, u1.y);
  w[6] = make_uint2(u1.z, u1.w);
}

// K polynomials at once (sharing twiddle loads and exchanges).  Input
// values below 2q; output values are left in [0, 4q).
template <int LOGN, int K>
__device__ __forceinline__ void ntt_fwd_k(uint32_t (&x)[K][8], const uint2* __restrict__ tab,
                                          const uint2* __restrict__ twl, uint32_t q, uint32_t two_q, uint32_t* lds,
                                          uint32_t& xc, uint32_t t) {
  constexpr int R = Geo<LOGN>::R;
  {  // phase 0: stages 0..2, twiddles uniform over the workgroup
    const uint2 w1 = tab[1], w2 = tab[2], w3 = tab[3], w4 = tab[4], w5 = tab[5], w6 = tab[6], w7 = tab[7];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int e = 0; e < 4; ++e) bf_fwd0(x[k][e], x[k][e + 4], w1.x, w1.y, q, two_q);
      bf_fwd(x[k][0], x[k][2], w2.x, w2.y, q, two_q);
      bf_fwd(x[k][1], x[k][3], w2.x, w2.y, q, two_q);
      bf_fwd(x[k][4], x[k][6], w3.x, w3.y, q, two_q);
      bf_fwd(x[k][5], x[k][7], w3.x, w3.y, q, two_q);
      bf_fwd(x[k][0], x[k][1], w4.x, w4.y, q, two_q);
      bf_fwd(x[k][2], x[k][3], w5.x, w5.y, q, two_q);
      bf_fwd(x[k][4], x[k][5], w6.x, w6.y, q, two_q);
      bf_fwd(x[k][6], x[k][7], w7.x, w7.y, q, two_q);
    }
  }
  xchg_k<LOGN, 0, 1, K>(x, lds, xc, t);
  {
    uint2 w[7];
    tw_phase(w, twl, 3, t >> (LOGN - 6));
#pragma unroll
    for (int k = 0; k < K; ++k) fwd8(x[k], w, q, two_q);
  }
  xchg_k<LOGN, 1, 2, K>(x, lds, xc, t);
  {
    uint2 w[7];
    tw_phase(w, twl, 6, t >> (LOGN - 9));
#pragma unroll
    for (int k = 0; k < K; ++k) fwd8(x[k], w, q, two_q);
  }
  xchg_k<LOGN, 2, 3, K>(x, lds, xc, t);
  if constexpr (R == 3) {
    uint2 w[7];
    tw_phase(w, twl, 9, t);
#pragma unroll
    for (int k = 0; k < K; ++k) fwd8(x[k], w, q, two_q);
  } else if constexpr (R == 2) {
    const uint4 v = *reinterpret_cast<const uint4*>(twl + 512 + 2 * t);
    const uint4 u0 = *reinterpret_cast<const uint4*>(twl + 1024 + 4 * t);
    const uint4 u1 = *reinterpret_cast<const uint4*>(twl + 1024 + 4 * t + 2);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      bf_fwd(x[k][0], x[k][2], v.x, v.y, q, two_q);
      bf_fwd(x[k][1], x[k][3], v.x, v.y, q, two_q);
      bf_fwd(x[k][4], x[k][6], v.z, v.w, q, two_q);
      bf_fwd(x[k][5], x[k][7], v.z, v.w, q, two_q);
      bf_fwd(x[k][0], x[k][1], u0.x, u0.y, q, two_q);
      bf_fwd(x[k][2], x[k][3], u0.z, u0.w, q, two_q);
      bf_fwd(x[k][4], x[k][5], u1.x, u1.y, q, two_q);
      bf_fwd(x[k][6], x[k][7], u1.z, u1.w, q, two_q);
    }
  } else {
    const uint4 u0 = *reinterpret_cast<const uint4*>(twl + 512 + 4 * t);
    const uint4 u1 = *reinterpret_cast<const uint4*>(twl + 512 + 4 * t + 2);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      bf_fwd(x[k][0], x[k][1], u0.x, u0.y, q, two_q);
      bf_fwd(x[k][2], x[k][3], u0.z, u0.w, q, two_q);
      bf_fwd(x[k][4], x[k][5], u1.x, u1.y, q, two_q);
      bf_fwd(x[k][6], x[k][7], u1.z, u1.w, q, two_q);
    }
  }
}

template <int LOGN>
__device__ __forceinline__ void ntt_fwd(uint32_t (&x)[8], const uint2* __restrict__ tab, const uint2* __restrict__ twl,
                                        uint32_t q, uint32_t two_q, uint32_t* lds, uint32_t& xc, uint32_t t) {
  ntt_fwd_k<LOGN, 1>(*reinterpret_cast<uint32_t(*)[1][8]>(&x), tab, twl, q, two_q, lds, xc, t);
}

// ---------------------------------------------------------------------------
// inverse NTT (layout P=3 -> natural layout), input in [0, 2q), output [0, q)
// ---------------------------------------------------------------------------

// three inverse stages (s0+2, s0+1, s0) of a phase whose index bits vary with
// e, on K polynomials; base(s) gives 2^s + (k >> (log2 N - s)) with the
// e-dependent part removed
template <int K>
__device__ __forceinline__ void inv8_k(uint32_t (&x)[K][8], const uint2* __restrict__ tab, uint32_t i2,
                                       uint32_t i1, uint32_t i0, uint32_t q, uint32_t two_q) {
  uint2 w2[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) w2[e] = tab[i2 + e];
  const uint2 w1a = tab[i1], w1b = tab[i1 + 1], w0 = tab[i0];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int e = 0; e < 4; ++e) bf_inv(x[k][2 * e], x[k][2 * e + 1], w2[e].x, w2[e].y, q, two_q);
    bf_inv(x[k][0], x[k][2], w1a.x, w1a.y, q, two_q);
    bf_inv(x[k][1], x[k][3], w1a.x, w1a.y, q, two_q);
    bf_inv(x[k][4], x[k][6], w1b.x, w1b.y, q, two_q);
    bf_inv(x[k][5], x[k][7], w1b.x, w1b.y, q, two_q);
#pragma unroll
    for (int e = 0; e < 4; ++e) bf_inv(x[k][e], x[k][e + 4], w0.x, w0.y, q, two_q);
  }
}

// K polynomials at once (sharing twiddle loads and exchanges)
template <int LOGN, int K>
__device__ __forceinline__ void ntt_inv_k(uint32_t (&x)[K][8], const uint2* __restrict__ tab, const PrimeTab& P,
                                          uint32_t* lds, uint32_t& xc, uint32_t t) {
  constexpr int R = Geo<LOGN>::R;
  const uint32_t q = P.q, two_q = P.two_q;
  if constexpr (R == 3) {
    inv8_k<K>(x, tab, 2048 + (t << 2), 1024 + (t << 1), 512 + t, q, two_q);
  } else if constexpr (R == 2) {
    uint2 w2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w2[e] = tab[1024 + (t << 2) + e];
    const uint2 w1a = tab[512 + (t << 1)], w1b = tab[512 + (t << 1) + 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int e = 0; e < 4; ++e) bf_inv(x[k][2 * e], x[k][2 * e + 1], w2[e].x, w2[e].y, q, two_q);
      bf_inv(x[k][0], x[k][2], w1a.x, w1a.y, q, two_q);
      bf_inv(x[k][1], x[k][3], w1a.x, w1a.y, q, two_q);
      bf_inv(x[k][4], x[k][6], w1b.x, w1b.y, q, two_q);
      bf_inv(x[k][5], x[k][7], w1b.x, w1b.y, q, two_q);
    }
  } else {
    uint2 w2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w2[e] = tab[512 + (t << 2) + e];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) bf_inv(x[k][2 * e], x[k][2 * e + 1], w2[e].x, w2[e].y, q, two_q);
  }
  xchg_k<LOGN, 3, 2, K>(x, lds, xc, t);
  {
    const uint32_t tc = t >> (LOGN - 9);
    inv8_k<K>(x, tab, 256 + (tc << 2), 128 + (tc << 1), 64 + tc, q, two_q);
  }
  xchg_k<LOGN, 2, 1, K>(x, lds, xc, t);
  {
    const uint32_t tb = t >> (LOGN - 6);
    inv8_k<K>(x, tab, 32 + (tb << 2), 16 + (tb << 1), 8 + tb, q, two_q);
  }
  xchg_k<LOGN, 1, 0, K>(x, lds, xc, t);
  inv8_k<K>(x, tab, 4, 2, 1, q, two_q);
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int e = 0; e < 8; ++e) x[k][e] = csub(mulsh(x[k][e], P.ninv, P.ninv_sh, q), q);
}

template <int LOGN>
__device__ __forceinline__ void ntt_inv(uint32_t (&x)[8], const uint2* __restrict__ tab, const PrimeTab& P,
                                        uint32_t* lds, uint32_t& xc, uint32_t t) {
  ntt_inv_k<LOGN, 1>(*reinterpret_cast<uint32_t(*)[1][8]>(&x), tab, P, lds, xc, t);
}

// reduce forward-NTT output [0, 4q) -> [0, q)
__device__ __forceinline__ uint32_t red4q(uint32_t x, uint32_t q, uint32_t two_q) {
  return csub(csub(x, two_q), q);
}

// ---------------------------------------------------------------------------
// fused external product
// ---------------------------------------------------------------------------
// xin: the input RLWE [poly a=0,b=1][prime][N] in global memory; thread t
// reads only its own coefficients t + T e, so no synchronisation is needed
// between whoever wrote them (the same thread) and the transform.
// C: one RGSW in device layout [row 2D][poly 2][prime NQ][N] (evaluation
// domain, layout P=3).  For every output prime ip the 2D digit polynomials
// (the digits of b against rows 0..D-1, then those of a against rows
// D..2D-1) are transformed and multiplied into 64-bit accumulators; the two
// accumulators are brought back by the inverse NTT and handed to
// epi(ip, ha, hb) in the natural layout, values in [0, q).
// twl: LDS space for one prime's forward table (N uint2).  Outputs may alias
// xin only as dst == src (each thread reads then writes its own coefficient).

// What happens to h = C [.] xin, per output prime, coefficient k (natural):
//   XP_STORE     : dst[k] = h
//   XP_ADD       : dst[k] = src[k] + h            (CMUX: d0 + C [.] (d1 - d0))
//   XP_DEMUX     : dst[k] = src[k] - h, dst2[k] = h (CDEMUX)
//   XP_DEMUX_ACC : dst[k] += src[k] - h, dst2[k] += h (CDEMUX outputs added
//                  into accumulators)
enum XpMode : int { XP_STORE = 0, XP_ADD = 1, XP_DEMUX = 2, XP_DEMUX_ACC = 3 };

struct XpOut {
  uint32_t* dst;
  const uint32_t* src;
  uint32_t* dst2;
  int mode;
};

// Balanced base-2^6 digits of a centred residue v (|v| < 2^29), read off
// w = v + DIGIT_OFFSET, DIGIT_OFFSET = 32 (1 + 64 + 64^2 + 64^3): since
// v = sum_{j<4} d_j 64^j + d_4 64^4 with d_j in [-32, 32), the low 24 bits
// of w are the d_j + 32 and w >> 24 (arithmetic) is d_4.  These are the
// digits that repeating d = ((v + 32) mod 64) - 32, v = (v - d) / 64 gives;
// one bit-field extract per digit instead of that carry chain.  Returned as
// d + q, in [q - 32, q + 32]: congruent to d and below 2q, which is all the
// forward transform asks of its input (its reduced outputs are the same as
// for d mod q).
constexpr int32_t DIGIT_OFFSET = 32 * (1 + 64 + 4096 + 262144);

// The same for any gadget of DIG balanced base-2^LB digits per prime: the
// offset is 2^(LB-1) (1 + B + .. + B^(DIG-2)), the digits below the top one are
// LB-bit fields of w, the top one is w >> (LB (DIG - 1)) (arithmetic).  The
// default gadget is (5, 6); contexts on rings of two or more primes may use
// (2, 15), which the key-switched bootstrapping key always uses there.
template <int DIG, int LB>
__host__ __device__ constexpr int32_t digit_offset() {
  int64_t o = 0, b = 1;
  for (int j = 0; j + 1 < DIG; ++j, b <<= LB) o += b << (LB - 1);
  return (int32_t)o;
}
static_assert(digit_offset<5, 6>() == DIGIT_OFFSET, "the training gadget's offset");

template <int DIG, int LB>
__device__ __forceinline__ uint32_t digit_lift_g(int32_t w, int j, uint32_t q) {
  if (j < DIG - 1) return (((uint32_t)w >> (LB * j)) & ((1u << LB) - 1u)) + (q - (1u << (LB - 1)));
  return (uint32_t)((w >> (LB * (DIG - 1))) + (int32_t)q);
}

__device__ __forceinline__ uint32_t digit_lift(int32_t w, int j, uint32_t q) { return digit_lift_g<5, 6>(w, j, q); }

// The two RGSW gadgets the kernels are built for, by digits per prime: 5
// digits of 6 bits (the training default) and 2 digits of 15 bits (rings of
// two or more primes).
template <int DIG>
__host__ __device__ constexpr int gadget_lb() {
  static_assert(DIG == 5 || DIG == 2, "gadgets: 5 digits of 6 bits or 2 digits of 15 bits per prime");
  return DIG == 5 ? 6 : 15;
}

// inverse transforms of the a and b sums of output prime ip (inputs in [0, q))
// and the write of the external product by out.mode
template <int LOGN, int NQ, bool PR>
__device__ __forceinline__ void xp_finish(uint32_t (&ha)[8], uint32_t (&hb)[8], int ip, const Tabs& T, uint32_t* lds,
                                          uint32_t& xc, uint32_t t, const XpOut& out) {
  constexpr int N = 1 << LOGN, TT = N / 8;
  const PrimeTab P = T.pt[ip];
  if constexpr (PR) {  // both sums through one two-polynomial transform
    uint32_t h[2][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      h[0][e] = ha[e];
      h[1][e] = hb[e];
    }
    ntt_inv_k<LOGN, 2>(h, T.inv[ip], P, lds, xc, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ha[e] = h[0][e];
      hb[e] = h[1][e];
    }
  } else {
    ntt_inv<LOGN>(ha, T.inv[ip], P, lds, xc, t);
    ntt_inv<LOGN>(hb, T.inv[ip], P, lds, xc, t);
  }
  const size_t oa = (size_t)ip * N, ob = (size_t)(NQ + ip) * N;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const size_t ea = oa + TT * e, eb = ob + TT * e;
    if (out.mode == XP_STORE) {
      (out.dst + ea)[t] = ha[e];
      (out.dst + eb)[t] = hb[e];
    } else if (out.mode == XP_ADD) {
      (out.dst + ea)[t] = addq((out.src + ea)[t], ha[e], P.q);
      (out.dst + eb)[t] = addq((out.src + eb)[t], hb[e], P.q);
    } else if (out.mode == XP_DEMUX) {
      (out.dst + ea)[t] = subq((out.src + ea)[t], ha[e], P.q);
      (out.dst + eb)[t] = subq((out.src + eb)[t], hb[e], P.q);
      (out.dst2 + ea)[t] = ha[e];
      (out.dst2 + eb)[t] = hb[e];
    } else {
      (out.dst + ea)[t] = addq((out.dst + ea)[t], subq((out.src + ea)[t], ha[e], P.q), P.q);
      (out.dst + eb)[t] = addq((out.dst + eb)[t], subq((out.src + eb)[t], hb[e], P.q), P.q);
      (out.dst2 + ea)[t] = addq((out.dst2 + ea)[t], ha[e], P.q);
      (out.dst2 + eb)[t] = addq((out.dst2 + eb)[t], hb[e], P.q);
    }
  }
}

// DIG, LB: the RGSW's gadget, DIG balanced base-2^LB digits per prime (rows
// side * DIG NQ + i DIG + j); (5, 6) unless stated
template <int LOGN, int NQ, bool PR = xp_pair<LOGN, NQ>(), int DIG = 5, int LB = 6>
__device__ __forceinline__ void ext_prod(const uint32_t* __restrict__ xin, const uint32_t* __restrict__ C,
                                      const Tabs& T, uint32_t* lds, uint2* twl, uint32_t& xc, uint32_t t,
                                      XpOut out) {
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr int D = DIG * NQ;
  constexpr int32_t OFF = digit_offset<DIG, LB>();
  constexpr size_t ROW = (size_t)2 * NQ * N;
#pragma unroll 1
  for (int ip = 0; ip < NQ; ++ip) {
    const PrimeTab P = T.pt[ip];
    load_tw_lds<LOGN>(twl, T.fwd[ip], t);
    __syncthreads();
    uint64_t acc_a[8], acc_b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc_a[e] = acc_b[e] = 0;
    int cnt = 0;
#pragma unroll 1
    for (int g = 0; g < 2 * NQ; ++g) {  // g = side * NQ + i
      const int side = g / NQ, i = g - side * NQ;
      const int p = side == 0 ? 1 : 0;
      const uint32_t qi = T.pt[i].q;
      const uint32_t* src = xin + ((size_t)p * NQ + i) * N;
      int32_t w[8];  // centred residues plus DIGIT_OFFSET
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t r = (src + TT * e)[t];
        w[e] = (r > (qi - 1) / 2 ? (int32_t)(r - qi) : (int32_t)r) + OFF;
      }
      const uint32_t* crow = C + (size_t)(side * D + i * DIG) * ROW + (size_t)ip * N;
      if constexpr (PR) {
        // digits (0, 1), (2, 3), .. through one two-polynomial transform each
#pragma unroll 1
        for (int j = 0; j < DIG - 1; j += 2) {
          const uint4* c0 = reinterpret_cast<const uint4*>(crow + (size_t)j * ROW);
          const uint4* c1 = reinterpret_cast<const uint4*>(crow + (size_t)(j + 1) * ROW);
          const uint4 ca00 = c0[2 * t], ca01 = c0[2 * t + 1];
          const uint4 cb00 = (c0 + NQ * N / 4)[2 * t], cb01 = (c0 + NQ * N / 4)[2 * t + 1];
          const uint4 ca10 = c1[2 * t], ca11 = c1[2 * t + 1];
          const uint4 cb10 = (c1 + NQ * N / 4)[2 * t], cb11 = (c1 + NQ * N / 4)[2 * t + 1];
          uint32_t x[2][8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            x[0][e] = digit_lift_g<DIG, LB>(w[e], j, P.q);
            x[1][e] = digit_lift_g<DIG, LB>(w[e], j + 1, P.q);
          }
          ntt_fwd_k<LOGN, 2>(x, T.fwd[ip], twl, P.q, P.two_q, lds, xc, t);
          const uint32_t ca[2][8] = {{ca00.x, ca00.y, ca00.z, ca00.w, ca01.x, ca01.y, ca01.z, ca01.w},
                                     {ca10.x, ca10.y, ca10.z, ca10.w, ca11.x, ca11.y, ca11.z, ca11.w}};
          const uint32_t cb[2][8] = {{cb00.x, cb00.y, cb00.z, cb00.w, cb01.x, cb01.y, cb01.z, cb01.w},
                                     {cb10.x, cb10.y, cb10.z, cb10.w, cb11.x, cb11.y, cb11.z, cb11.w}};
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const uint32_t xr = red4q(x[k][e], P.q, P.two_q);
              acc_a[e] += (uint64_t)xr * ca[k][e];
              acc_b[e] += (uint64_t)xr * cb[k][e];
            }
          cnt += 2;
          if (cnt >= 14) {  // at most 15 products of two values below q since the last reduction
            cnt = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              acc_a[e] = red64(acc_a[e], P);
              acc_b[e] = red64(acc_b[e], P);
            }
          }
        }
      }
#pragma unroll 1
      for (int j = PR ? DIG / 2 * 2 : 0; j < DIG; ++j) {
        const uint4* cra = reinterpret_cast<const uint4*>(crow + (size_t)j * ROW);
        const uint4* crb = cra + (size_t)NQ * N / 4;
        const uint4 ca0 = cra[2 * t], ca1 = cra[2 * t + 1];
        const uint4 cb0 = crb[2 * t], cb1 = crb[2 * t + 1];
        uint32_t x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = digit_lift_g<DIG, LB>(w[e], j, P.q);
        ntt_fwd<LOGN>(x, T.fwd[ip], twl, P.q, P.two_q, lds, xc, t);
        const uint32_t ca[8] = {ca0.x, ca0.y, ca0.z, ca0.w, ca1.x, ca1.y, ca1.z, ca1.w};
        const uint32_t cb[8] = {cb0.x, cb0.y, cb0.z, cb0.w, cb1.x, cb1.y, cb1.z, cb1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t xr = red4q(x[e], P.q, P.two_q);
          acc_a[e] += (uint64_t)xr * ca[e];
          acc_b[e] += (uint64_t)xr * cb[e];
        }
        if (++cnt >= (PR ? 14 : 15)) {
          cnt = 0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            acc_a[e] = red64(acc_a[e], P);
            acc_b[e] = red64(acc_b[e], P);
          }
        }
      }
    }
    uint32_t ha[8], hb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ha[e] = red64(acc_a[e], P);
      hb[e] = red64(acc_b[e], P);
    }
    xp_finish<LOGN, NQ, PR>(ha, hb, ip, T, lds, xc, t, out);
  }
}

// External product with the trivial RLWE (0, Delta (X - 1)): the first CMUX
// of an IVP chain, whose accumulator starts at (0, Delta).  Its a side is
// zero, so only the D gadget rows of the b side take part, and each digit
// polynomial is d0 + d1 X with the scalar digits d0, d1 of the centred
// residues of -Delta and Delta.  Its transform at evaluation point k is
// d0 + d1 E[k] (E = the transform of X), so
//   acc[k] = sum_r d0_r C_r[k] + E[k] sum_r d1_r C_r[k]  (mod q)
// with small signed multipliers.  Both sums are reduced to [0, q) before the
// inverse transform, as in ext_prod, so the result is the same residues
// ext_prod computes for that input, without its 2 DIG nq^2 forward transforms
// and with half its RGSW reads.  DIG, LB: the RGSW's gadget, as in ext_prod.
template <int LOGN, int NQ, bool PR = xp_pair<LOGN, NQ>(), int DIG = 5, int LB = 6>
__device__ __forceinline__ void ext_prod_delta(const uint32_t* __restrict__ C, const Tabs& T, uint32_t* lds,
                                               uint32_t& xc, uint32_t t, XpOut out) {
  constexpr int N = 1 << LOGN;
  constexpr size_t ROW = (size_t)2 * NQ * N;
#pragma unroll 1
  for (int ip = 0; ip < NQ; ++ip) {
    const PrimeTab P = T.pt[ip];
    uint32_t h[2][8];  // a and b sums, reduced
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {  // one output polynomial at a time keeps the sums in registers
      int64_t s0[8], s1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) s0[e] = s1[e] = 0;
#pragma unroll 1
      for (int i = 0; i < NQ; ++i) {
        // centred residues of -Delta and Delta mod q_i, decomposed digit by digit
        // exactly as ext_prod decomposes its input (uniform over the workgroup)
        const uint32_t qi = T.pt[i].q, dl = T.pt[i].delta;
        const uint32_t r0 = dl ? qi - dl : 0u;
        int32_t v0 = r0 > (qi - 1) / 2 ? (int32_t)(r0 - qi) : (int32_t)r0;
        int32_t v1 = dl > (qi - 1) / 2 ? (int32_t)(dl - qi) : (int32_t)dl;
        constexpr int32_t H = 1 << (LB - 1), M = (1 << LB) - 1;
#pragma unroll 1
        for (int j = 0; j < DIG; ++j) {
          int32_t e0 = v0, e1 = v1;
          if (j < DIG - 1) {
            e0 = ((v0 + H) & M) - H;
            e1 = ((v1 + H) & M) - H;
            v0 = (v0 - e0) >> LB;
            v1 = (v1 - e1) >> LB;
          }
          const uint4* cr = reinterpret_cast<const uint4*>(C + (size_t)(i * DIG + j) * ROW +
                                                           ((size_t)side * NQ + ip) * N);
          const uint4 c0 = cr[2 * t], c1 = cr[2 * t + 1];
          const int32_t cv[8] = {(int32_t)c0.x, (int32_t)c0.y, (int32_t)c0.z, (int32_t)c0.w,
                                 (int32_t)c1.x, (int32_t)c1.y, (int32_t)c1.z, (int32_t)c1.w};
          const int64_t d0 = e0, d1 = e1;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            s0[e] += d0 * cv[e];
            s1[e] += d1 * cv[e];
          }
        }
      }
      // |s| < DIG NQ 2^(LB-1) q <= 2^(LB+4) q (DIG NQ <= 15): shifting by 2^(LB+4) q
      // makes it nonnegative, same residue
      const int64_t sh = (int64_t)P.q << (LB + 4);
      const uint4* ev = reinterpret_cast<const uint4*>(T.evx[ip] + 8 * (size_t)t);
#pragma unroll
      for (int hh = 0; hh < 4; ++hh) {
        const uint4 w = ev[hh];
        const uint32_t r0 = csub(mulsh(red64((uint64_t)(s1[2 * hh] + sh), P), w.x, w.y, P.q), P.q);
        const uint32_t r1 = csub(mulsh(red64((uint64_t)(s1[2 * hh + 1] + sh), P), w.z, w.w, P.q), P.q);
        h[side][2 * hh] = addq(red64((uint64_t)(s0[2 * hh] + sh), P), r0, P.q);
        h[side][2 * hh + 1] = addq(red64((uint64_t)(s0[2 * hh + 1] + sh), P), r1, P.q);
      }
    }
    xp_finish<LOGN, NQ, PR>(h[0], h[1], ip, T, lds, xc, t, out);
  }
}

// ---------------------------------------------------------------------------
// RLWE slots in global memory, natural layout
// ---------------------------------------------------------------------------

template <int LOGN, int NQ>
__device__ __forceinline__ void load_rlwe(uint32_t (&r)[2][NQ][8], const uint32_t* __restrict__ src, uint32_t t) {
  constexpr int N = 1 << LOGN, TT = N / 8;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
      for (int e = 0; e < 8; ++e) r[p][i][e] = src[((size_t)p * NQ + i) * N + t + TT * e];
}

// coefficient k of X^e * f (e in (-2N, 2N)), polynomial f of one prime
template <int LOGN>
__device__ __forceinline__ uint32_t rot_coef(const uint32_t* __restrict__ f, int32_t k, int32_t e, uint32_t q) {
  constexpr int32_t N = 1 << LOGN;
  int32_t u = k - e;
  u = (u % (2 * N) + 2 * N) % (2 * N);
  if (u < N) return f[u];
  const uint32_t v = f[u - N];
  return v ? q - v : 0u;
}

}  // namespace hw
