// hw_kernels.hip -- HIP kernels for gfx950 of the encrypted WiSARD hot path
// and their launchers.  Template parameters: LOGN = log2 N (10..12), NQ =
// number of primes (1..3); one workgroup of N/8 threads per polynomial job.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hw_device.h"
#include "hw_internal.h"

namespace hw {

typedef unsigned __int128 u128;

// Occupancy target of the external-product kernels (waves per SIMD, template
// parameter OCC of the training and inference kernels): 3 keeps every value
// in registers (about 150 VGPRs); 4 (N = 4096 only) lets two workgroups of
// 512 threads share a CU at the price of a few spilled registers.
constexpr int WAVES_XP = 3;

// ---------------------------------------------------------------------------
// counter-based generator: Philox4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation with
// truth table 0x96 (the compiler leaves two two-input XORs otherwise)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // each 32 x 32 -> 64-bit product in one instruction (both halves used)
    const uint64_t p0 = mad64(0xD2511F53u, c.x, 0ull), p1 = mad64(0xCD9E8D57u, c.z, 0ull);
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                   (uint32_t)p0);
  }
  return c;
}

// the two 64-bit draws 2*blk and 2*blk+1 of stream (seed, domain)
__device__ __forceinline__ void draw_pair(uint64_t seed, uint32_t domain, uint64_t blk, uint64_t& d0,
                                          uint64_t& d1) {
  const uint4 o = philox10(make_uint4((uint32_t)blk, (uint32_t)(blk >> 32), domain, 0u), (uint32_t)seed,
                           (uint32_t)(seed >> 32));
  d0 = (uint64_t)o.x | ((uint64_t)o.y << 32);
  d1 = (uint64_t)o.z | ((uint64_t)o.w << 32);
}

constexpr uint32_t DOM_KEY = 1, DOM_PERM = 2, DOM_ENC_A = 3, DOM_ENC_E = 4, DOM_ENC_A2 = 5;

// the four 32-bit draws 4*blk .. 4*blk+3 of stream (seed, domain)
__device__ __forceinline__ uint4 draw4(uint64_t seed, uint32_t domain, uint64_t blk) {
  return philox10(make_uint4((uint32_t)blk, (uint32_t)(blk >> 32), domain, 0u), (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// Uniform residues mod q of encryption draws x0 .. x0+K-1 (x0 a multiple of
// 4), from their 32-bit words of stream (seed, ENC_A): w mod q when
// w < floor(2^32 / q) q, which is exactly uniform; otherwise (probability
// (2^32 mod q) / 2^32, about 3e-5 near 2^30) the 64-bit draw x of
// (seed, ENC_A2) mod q.  floor(2^32 / q) q < 2^32 is one_sh * q in 32 bits.
// The accepted path is branch-free; one branch per call, almost never taken,
// replaces the rejected words.
template <int K>
__device__ __forceinline__ void uniform_k(uint64_t seed, uint64_t x0, const PrimeTab& P, uint32_t (&xa)[K]) {
  const uint32_t lim = P.one_sh * P.q;
  uint32_t rej = 0;
#pragma unroll
  for (int f = 0; f < K / 4; ++f) {
    const uint4 w = draw4(seed, DOM_ENC_A, (x0 >> 2) + f);
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xa[4 * f + u] = csub(mulsh(ww[u], 1u, P.one_sh, P.q), P.q);
      rej |= (uint32_t)(ww[u] >= lim) << (4 * f + u);
    }
  }
  if (__builtin_expect(rej != 0u, 0)) {
#pragma unroll 1
    for (int u = 0; u < K; ++u)
      if ((rej >> u) & 1u) {
        const uint64_t x = x0 + u;
        uint64_t d0, d1;
        draw_pair(seed, DOM_ENC_A2, x >> 1, d0, d1);
        xa[u] = red64((x & 1) ? d1 : d0, P);
      }
  }
}

// magnitude = the smallest k with r < T[k] (T[41] = 2^63 > r), i.e. the
// number of entries T[j] <= r: T is non-decreasing, so those form a prefix.
// Six fixed steps of 32, 16, .., 1 find it without data-dependent branches.
__device__ __forceinline__ int32_t cdt_sample(const uint64_t* T, uint64_t w) {
  const uint64_t r = w >> 1;
  int k = 0;
#pragma unroll
  for (int b = 32; b >= 1; b >>= 1)
    if (k + b <= 41 && T[k + b - 1] <= r) k += b;
  return (k != 0 && (w & 1)) ? -k : k;
}

// The same sample through a guide (Cdt::guide): the draw's bucket b = r >>
// (63 - CDT_GUIDE_BITS) starts the count at G[b], the number of T[j] <= b
// 2^(63 - CDT_GUIDE_BITS); when at most two T[j] fall inside the bucket, two
// comparisons finish it (T is non-decreasing and T[41] = 2^63 > r stops a
// scan at 41), else (a few buckets at the top of the range) the six-step
// search runs.  Equal to cdt_sample for every draw.
__device__ __forceinline__ int32_t cdt_sample_guided(const uint64_t* T, const uint8_t* G, uint64_t w) {
  const uint64_t r = w >> 1;
  const uint32_t g = G[(uint32_t)(r >> (63 - CDT_GUIDE_BITS))];
  if (__builtin_expect((g & CDT_GUIDE_WIDE) != 0u, 0)) return cdt_sample(T, w);
  int k = (int)g;
  k += T[k] <= r ? 1 : 0;
  k += T[k] <= r ? 1 : 0;
  return (k != 0 && (w & 1)) ? -k : k;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------

__global__ void k_keygen(uint32_t N, uint64_t seed, int32_t* sk) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  uint64_t d0, d1;
  draw_pair(seed, DOM_KEY, k >> 1, d0, d1);
  const uint64_t w = (k & 1) ? d1 : d0;
  sk[k] = (int32_t)(w % 3) - 1;
}

// Binary LWE key of n coefficients (the key the bootstrap switches to):
// s1_i = bit 0 of the 64-bit draw i of stream (seed, LWE_KEY)
constexpr uint32_t DOM_LWE_KEY = 7, DOM_KSK_A = 8, DOM_KSK_E = 9;

__global__ void k_lwe_keygen(uint32_t n, uint64_t seed, uint8_t* __restrict__ s1) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t d0, d1;
  draw_pair(seed, DOM_LWE_KEY, i >> 1, d0, d1);
  s1[i] = (uint8_t)(((i & 1) ? d1 : d0) & 1u);
}

// the four signed bytes m_l in [-128, 128) with sum_l m_l 2^(8l) = v mod 2^32
// (lowest first, a byte >= 128 taken as byte - 256 with a carry into the next;
// the carry out of the top byte has weight 2^32)
__device__ __forceinline__ void signed_bytes(uint32_t v, int8_t (&m)[4]) {
  uint32_t carry = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const uint32_t x = ((v >> (8 * l)) & 255u) + carry;
    carry = x >= 128u;
    m[l] = (int8_t)(int32_t)(carry ? (int32_t)x - 256 : (int32_t)x);
  }
}

// Key-switching key from the ring key s to s1 at modulus 2^32: row r = k D + j
// (D = KS digits, k < N, j < D) is A_r[i] = draw32(seed, KSK_A, r n + i) and
// B_r = sum_i A_r[i] s1_i + e_r + s_k 2^(28 - 4j), e_r = 2^13 c + u with c the
// Gaussian sample of draw64(seed, KSK_E, 2r) and u = (draw64(seed, KSK_E,
// 2r + 1) >> 51) - 2^12.  Stored for the contraction as signed bytes:
// out[(l (n + 1) + i) K + r] = byte l of A_r[i] (i < n) or of B_r (i = n),
// K = N D.  One workgroup of 256 threads per row.
__global__ __launch_bounds__(256) void k_ksk_gen(const int32_t* __restrict__ sk, const uint8_t* __restrict__ s1,
                                                 uint32_t n, uint64_t seed, uint32_t D, uint64_t K, Cdt cdt,
                                                 int8_t* __restrict__ out) {
  __shared__ uint32_t part[256];
  const uint64_t r = blockIdx.x;
  const uint32_t t = threadIdx.x;
  uint32_t dot = 0;
  for (uint32_t i = t; i < n; i += 256) {
    const uint64_t x = r * n + i;
    const uint4 w = draw4(seed, DOM_KSK_A, x >> 2);
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
    const uint32_t a = ww[x & 3];
    if (s1[i]) dot += a;
    int8_t m[4];
    signed_bytes(a, m);
#pragma unroll
    for (int l = 0; l < 4; ++l) out[((uint64_t)l * (n + 1) + i) * K + r] = m[l];
  }
  part[t] = dot;
  __syncthreads();
  for (uint32_t h = 128; h >= 1; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) {
    const uint32_t k = (uint32_t)(r / D), j = (uint32_t)(r - (uint64_t)k * D);
    uint64_t d0, d1;
    draw_pair(seed, DOM_KSK_E, r, d0, d1);
    const int64_t e = (int64_t)cdt_sample(cdt.T, d0) * 8192 + (int64_t)(d1 >> 51) - 4096;
    const uint32_t b = part[0] + (uint32_t)e + (uint32_t)((int64_t)sk[k] * ((int64_t)1 << (28 - 4 * j)));
    int8_t m[4];
    signed_bytes(b, m);
#pragma unroll
    for (int l = 0; l < 4; ++l) out[((uint64_t)l * (n + 1) + n) * K + r] = m[l];
  }
}

// The Fisher-Yates permutation of [0, s) with the generator's PERM stream
// (the host's make_perm, on the device): for k = s-1 down to 1, swap entries
// k and j = draw64(seed, PERM, s-1-k) mod (k+1).  One thread: the swaps are
// sequential, and s is at most a few thousand bits.
__global__ void k_perm(uint32_t s, uint64_t seed, uint32_t* __restrict__ pi) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (uint32_t k = 0; k < s; ++k) pi[k] = k;
  for (uint32_t k = s - 1; k >= 1 && k < s; --k) {
    const uint64_t x = (uint64_t)(s - 1 - k);
    uint64_t d0, d1;
    draw_pair(seed, DOM_PERM, x >> 1, d0, d1);
    const uint32_t j = (uint32_t)(((x & 1) ? d1 : d0) % (uint64_t)(k + 1));
    const uint32_t t = pi[k];
    pi[k] = pi[j];
    pi[j] = t;
  }
}

// sk_hat[i] = NTT(s mod q_i), evaluation layout; sk_hat[NQ + i] = its Shoup companions
template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_sk_hat(Tabs T, const int32_t* __restrict__ sk,
                                                          uint32_t* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8;
  const uint32_t t = threadIdx.x, i = blockIdx.x;
  const PrimeTab P = T.pt[i];
  uint32_t x[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int32_t v = sk[t + TT * e];
    x[e] = v < 0 ? (uint32_t)(v + (int32_t)P.q) : (uint32_t)v;
  }
  load_tw_lds<LOGN>(twl, T.fwd[i], t);
  __syncthreads();
  uint32_t xc = 0;
  ntt_fwd<LOGN>(x, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
  uint32_t v[8], w[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    v[e] = red4q(x[e], P.q, P.two_q);
    w[e] = (uint32_t)(((uint64_t)v[e] << 32) / P.q);  // Shoup companion floor(v 2^32 / q)
  }
  uint4* o = reinterpret_cast<uint4*>(out + (size_t)i * N + (t << 3));
  o[0] = make_uint4(v[0], v[1], v[2], v[3]);
  o[1] = make_uint4(v[4], v[5], v[6], v[7]);
  uint4* os = reinterpret_cast<uint4*>(out + (size_t)(NQ + i) * N + (t << 3));
  os[0] = make_uint4(w[0], w[1], w[2], w[3]);
  os[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

// the transformed key and its Shoup companions for thread t's entries 8t .. 8t+7 of prime i
template <int LOGN, int NQ>
__device__ __forceinline__ void load_sk_hat(const uint32_t* __restrict__ sk_hat, int i, uint32_t t,
                                            uint32_t (&sh)[8], uint32_t (&shs)[8]) {
  constexpr int N = 1 << LOGN;
  const uint4* sp = reinterpret_cast<const uint4*>(sk_hat + (size_t)i * N + (t << 3));
  const uint4* ss = reinterpret_cast<const uint4*>(sk_hat + (size_t)(NQ + i) * N + (t << 3));
  const uint4 s0 = sp[0], s1 = sp[1], c0 = ss[0], c1 = ss[1];
  sh[0] = s0.x; sh[1] = s0.y; sh[2] = s0.z; sh[3] = s0.w; sh[4] = s1.x; sh[5] = s1.y; sh[6] = s1.z; sh[7] = s1.w;
  shs[0] = c0.x; shs[1] = c0.y; shs[2] = c0.z; shs[3] = c0.w; shs[4] = c1.x; shs[5] = c1.y; shs[6] = c1.z;
  shs[7] = c1.w;
}

// ---------------------------------------------------------------------------
// encryption
// ---------------------------------------------------------------------------
// Draws of row `rid` (= ciphertext * rows + row): u_{i,k} is the uniform
// residue mod q_i of encryption draw (rid*NQ + i)*N + k (uniform_residue: its
// 32-bit word of stream ENC_A, with rejection), the coefficient k of a for an
// RLWE ciphertext and the value of a at psi^(2 brv(k) + 1) for an RGSW row;
// e_k is the CDT sample of 64-bit draw rid*N + k of stream ENC_E.
// Coefficient draws are generated four at a time and staged through LDS into
// the natural layout.

template <int LOGN>
__device__ __forceinline__ void gen_uniform(uint64_t seed, uint64_t x0, const PrimeTab& P,
                                            uint32_t* __restrict__ stage, uint32_t t, uint32_t (&x)[8]) {
  constexpr int N = 1 << LOGN, TT = N / 8;
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 2; ++f) {  // thread t draws coefficients 4b .. 4b+3, b = t + TT f
    const uint32_t b = t + TT * f;
    uint32_t r[4];
    uniform_k<4>(seed, x0 + 4 * (uint64_t)b, P, r);
    *reinterpret_cast<uint4*>(stage + 4 * b) = make_uint4(r[0], r[1], r[2], r[3]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = stage[t + TT * e];
}

// Errors of thread t's coefficients t + (N/8) e, e < 8: coefficient k takes
// error draw 8 (k mod N/8) + floor(k / (N/8)), so the thread's eight draws
// 8t .. 8t+7 are the four consecutive generator blocks base_blk + 4t .. +3
// (two 64-bit draws each) and need no exchange.
template <int LOGN>
__device__ __forceinline__ void gen_gauss(uint64_t seed, uint64_t base_blk, const uint64_t* cdt, uint32_t t,
                                          int32_t (&ev)[8]) {
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    uint64_t d0, d1;
    draw_pair(seed, DOM_ENC_E, base_blk + 4 * (uint64_t)t + f, d0, d1);
    ev[2 * f] = cdt_sample(cdt, d0);
    ev[2 * f + 1] = cdt_sample(cdt, d1);
  }
}

// gen_gauss with the guided CDT search (the guide in LDS)
template <int LOGN>
__device__ __forceinline__ void gen_gauss_guided(uint64_t seed, uint64_t base_blk, const uint64_t* cdt,
                                                 const uint8_t* guide, uint32_t t, int32_t (&ev)[8]) {
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    uint64_t d0, d1;
    draw_pair(seed, DOM_ENC_E, base_blk + 4 * (uint64_t)t + f, d0, d1);
    ev[2 * f] = cdt_sample_guided(cdt, guide, d0);
    ev[2 * f + 1] = cdt_sample_guided(cdt, guide, d1);
  }
}

// RGSW rows directly in the evaluation domain.  Draw k of prime i is the
// value of a at the point psi^(2 brv(k) + 1), which is position k of the
// forward transform's output (thread t holds positions 8t..8t+7, i.e. the
// draw pairs 4t..4t+3): a_hat needs no transform.  b_hat = a_hat * s_hat +
// NTT(e); the gadget constant m*base^j is added to every evaluation point
// (the transform of a constant polynomial is constant).  A workgroup builds
// R consecutive rows of one ciphertext, so each prime's twiddle table is
// copied to LDS once per R rows.  The errors use the guided CDT search.
template <int LOGN, int NQ, int R, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_enc_rgsw(Tabs T, Cdt cdt, EncArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  __shared__ uint64_t tab[42];
  __shared__ __attribute__((aligned(16))) uint8_t gtab[CDT_GUIDE_SIZE];
  constexpr int N = 1 << LOGN, D = DIG * NQ, ROWS = 2 * D;
  static_assert(ROWS % R == 0, "rows per workgroup must divide the rows of an RGSW");
  const uint32_t t = threadIdx.x, r0 = blockIdx.x * R;
  const uint64_t c = blockIdx.y + (uint64_t)blockIdx.z * gridDim.y;
  if (t < 42) tab[t] = cdt.T[t];
#pragma unroll 1
  for (uint32_t i = t; i < CDT_GUIDE_SIZE / 16; i += Geo<LOGN>::T)
    reinterpret_cast<uint4*>(gtab)[i] = reinterpret_cast<const uint4*>(cdt.guide)[i];
  const uint64_t ct = A.ct0 + c;
  const uint32_t m = A.bits[c];
  int32_t ev[R][8];
  __syncthreads();  // the CDT table and its guide in LDS
#pragma unroll
  for (int k = 0; k < R; ++k) gen_gauss_guided<LOGN>(A.seed, (ct * ROWS + r0 + k) * (N / 2), tab, gtab, t, ev[k]);
  uint32_t xc = 0;
#pragma unroll 1
  for (int i = 0; i < NQ; ++i) {
    const PrimeTab P = T.pt[i];
    __syncthreads();
    load_tw_lds<LOGN>(twl, T.fwd[i], t);
    uint32_t sh[8], shs[8];
    load_sk_hat<LOGN, NQ>(A.sk_hat, i, t, sh, shs);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t r = r0 + k;
      const uint64_t rid = ct * ROWS + r;
      uint32_t xa[8], xe[8];
      uniform_k<8>(A.seed, (rid * NQ + i) * (uint64_t)N + 8 * t, P, xa);  // evaluation positions 8t .. 8t+7
#pragma unroll
      for (int e = 0; e < 8; ++e) xe[e] = ev[k][e] < 0 ? (uint32_t)(ev[k][e] + (int32_t)P.q) : (uint32_t)ev[k][e];
      ntt_fwd<LOGN>(xe, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
      const bool brow = r < D;
      const uint32_t gi = (r % D) / DIG, gj = (r % D) % DIG;
      const uint32_t g = (m && gi == (uint32_t)i) ? (1u << (A.log_base * gj)) : 0u;
      uint32_t oa[8], ob[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t av = xa[e];
        const uint32_t ee = red4q(xe[e], P.q, P.two_q);
        const uint32_t bv = addq(csub(mulsh(av, sh[e], shs[e], P.q), P.q), ee, P.q);
        oa[e] = brow ? av : addq(av, g, P.q);
        ob[e] = brow ? addq(bv, g, P.q) : bv;
      }
      uint32_t* row = A.out + (c * ROWS + r) * (size_t)(2 * NQ * N);
      uint4* pa = reinterpret_cast<uint4*>(row + (size_t)i * N + (t << 3));
      uint4* pb = reinterpret_cast<uint4*>(row + (size_t)(NQ + i) * N + (t << 3));
      pa[0] = make_uint4(oa[0], oa[1], oa[2], oa[3]);
      pa[1] = make_uint4(oa[4], oa[5], oa[6], oa[7]);
      pb[0] = make_uint4(ob[0], ob[1], ob[2], ob[3]);
      pb[1] = make_uint4(ob[4], ob[5], ob[6], ob[7]);
    }
  }
}

// PackingKeySwitching key rows K[j][r] = RLWE_s(s_j G_r) in the evaluation
// domain, drawn like RGSW rows (ciphertext j, D rows): b_hat = a_hat * s_hat +
// NTT(e) + s_j G_r, the constant s_j 64^t added at every point of prime g
// for r = 5 g + t.  One workgroup per row.
template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_enc_pks(Tabs T, Cdt cdt, EncArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  __shared__ uint64_t tab[42];
  constexpr int N = 1 << LOGN, D = 5 * NQ;
  const uint32_t t = threadIdx.x, r = blockIdx.x, j = blockIdx.y;
  if (t < 42) tab[t] = cdt.T[t];
  const uint64_t rid = (uint64_t)j * D + r;
  const int32_t sj = A.sk[j];
  int32_t ev[8];
  __syncthreads();  // the CDT table in LDS
  gen_gauss<LOGN>(A.seed, rid * (N / 2), tab, t, ev);
  const uint32_t gi = r / 5, gt = r % 5;
  uint32_t* row = A.out + rid * (size_t)(2 * NQ * N);
  uint32_t xc = 0;
#pragma unroll 1
  for (int i = 0; i < NQ; ++i) {
    const PrimeTab P = T.pt[i];
    __syncthreads();
    load_tw_lds<LOGN>(twl, T.fwd[i], t);
    uint32_t sh[8], shs[8];
    load_sk_hat<LOGN, NQ>(A.sk_hat, i, t, sh, shs);
    uint32_t xa[8], xe[8];
    uniform_k<8>(A.seed, (rid * NQ + i) * (uint64_t)N + 8 * t, P, xa);  // evaluation positions 8t .. 8t+7
#pragma unroll
    for (int e = 0; e < 8; ++e) xe[e] = ev[e] < 0 ? (uint32_t)(ev[e] + (int32_t)P.q) : (uint32_t)ev[e];
    ntt_fwd<LOGN>(xe, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
    const uint32_t G = gi == (uint32_t)i ? (1u << (A.log_base * gt)) : 0u;
    const uint32_t g = sj == 0 || G == 0 ? 0u : (sj > 0 ? G : P.q - G);
    uint32_t ob[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      ob[e] = addq(addq(csub(mulsh(xa[e], sh[e], shs[e], P.q), P.q), red4q(xe[e], P.q, P.two_q), P.q), g, P.q);
    uint4* pa = reinterpret_cast<uint4*>(row + (size_t)i * N + (t << 3));
    uint4* pb = reinterpret_cast<uint4*>(row + (size_t)(NQ + i) * N + (t << 3));
    pa[0] = make_uint4(xa[0], xa[1], xa[2], xa[3]);
    pa[1] = make_uint4(xa[4], xa[5], xa[6], xa[7]);
    pb[0] = make_uint4(ob[0], ob[1], ob[2], ob[3]);
    pb[1] = make_uint4(ob[4], ob[5], ob[6], ob[7]);
  }
}

// RLWE encryption in the coefficient domain: b = a*s + Delta*msg + e
template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_enc_rlwe(Tabs T, Cdt cdt, EncArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  __shared__ __attribute__((aligned(16))) uint32_t stage[1 << LOGN];
  __shared__ uint64_t tab[42];
  constexpr int N = 1 << LOGN, TT = N / 8;
  const uint32_t t = threadIdx.x;
  const uint64_t c = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  if (t < 42) tab[t] = cdt.T[t];
  const uint64_t rid = A.ct0 + c;  // one row per ciphertext
  int32_t ev[8];
  __syncthreads();  // the CDT table in LDS
  gen_gauss<LOGN>(A.seed, rid * (N / 2), tab, t, ev);
  uint32_t* out = A.out + c * (size_t)(2 * NQ * N);
  uint32_t xc = 0;
#pragma unroll 1
  for (int i = 0; i < NQ; ++i) {
    const PrimeTab P = T.pt[i];
    __syncthreads();
    load_tw_lds<LOGN>(twl, T.fwd[i], t);
    uint32_t xa[8], a0[8];
    gen_uniform<LOGN>(A.seed, (rid * NQ + i) * (uint64_t)N, P, stage, t, xa);
#pragma unroll
    for (int e = 0; e < 8; ++e) a0[e] = xa[e];
    ntt_fwd<LOGN>(xa, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
    uint32_t sh[8], shs[8];
    load_sk_hat<LOGN, NQ>(A.sk_hat, i, t, sh, shs);
#pragma unroll
    for (int e = 0; e < 8; ++e) xa[e] = csub(mulsh(red4q(xa[e], P.q, P.two_q), sh[e], shs[e], P.q), P.q);
    ntt_inv<LOGN>(xa, T.inv[i], P, lds, xc, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t k = t + TT * e;
      const uint32_t ee = ev[e] < 0 ? (uint32_t)(ev[e] + (int32_t)P.q) : (uint32_t)ev[e];
      uint32_t b = addq(xa[e], ee, P.q);
      if (A.msg) b = addq(b, mulq(P.delta, red64(A.msg[c * N + k], P), P), P.q);
      out[(size_t)i * N + k] = a0[e];
      out[(size_t)(NQ + i) * N + k] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// decryption
// ---------------------------------------------------------------------------

__device__ __forceinline__ double u128_to_double(u128 v) {
  return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v;
}

// round(p * phi / Q) mod p with phi given by its residues (CRT), rounding half up
template <int NQ>
__device__ __forceinline__ uint64_t crt_decode(const uint32_t (&ph)[NQ], const Tabs& T, const CrtTab& K) {
  const u128 Q = ((u128)K.Q_hi << 64) | K.Q_lo;
  u128 acc = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const uint32_t y = mulq(ph[i], K.inv[i], T.pt[i]);
    const u128 M = ((u128)K.M_hi[i] << 64) | K.M_lo[i];
    acc += (u128)y * M;
    if (acc >= Q) acc -= Q;
  }
  const u128 num = (u128)K.p * acc + (((u128)K.half_hi << 64) | K.half_lo);
  uint64_t qt = (uint64_t)(u128_to_double(num) / u128_to_double(Q));
  while (qt > 0 && (u128)qt * Q > num) --qt;
  while ((u128)(qt + 1) * Q <= num) ++qt;
  return qt & (K.p - 1);
}

template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_dec_rlwe(Tabs T, CrtTab K, const uint32_t* __restrict__ sk_hat,
                                                            const uint32_t* __restrict__ ct,
                                                            uint64_t* __restrict__ msg) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8;
  const uint32_t t = threadIdx.x;
  const uint64_t c = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  const uint32_t* in = ct + c * (size_t)(2 * NQ * N);
  uint32_t ph[8][NQ];
  uint32_t xc = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const PrimeTab P = T.pt[i];
    __syncthreads();
    load_tw_lds<LOGN>(twl, T.fwd[i], t);
    uint32_t x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = in[(size_t)i * N + t + TT * e];
    ntt_fwd<LOGN>(x, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
    const uint4* sp = reinterpret_cast<const uint4*>(sk_hat + (size_t)i * N + (t << 3));
    const uint4 s0 = sp[0], s1 = sp[1];
    const uint32_t sh[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = mulq(red4q(x[e], P.q, P.two_q), sh[e], P);
    ntt_inv<LOGN>(x, T.inv[i], P, lds, xc, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) ph[e][i] = subq(in[(size_t)(NQ + i) * N + t + TT * e], x[e], P.q);
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) msg[c * N + t + TT * e] = crt_decode<NQ>(ph[e], T, K);
}

// one wavefront per LWE ciphertext
template <int NQ>
__global__ __launch_bounds__(256) void k_dec_lwe(Tabs T, CrtTab K, uint32_t N, const int32_t* __restrict__ sk,
                                                 const uint32_t* __restrict__ lwe, uint64_t count,
                                                 uint64_t* __restrict__ msg) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= count) return;
  const uint32_t* L = lwe + c * (size_t)NQ * (N + 1);
  uint32_t ph[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const uint32_t q = T.pt[i].q;
    uint64_t acc = 0;
    for (uint32_t k = lane; k < N; k += 64) {
      const int32_t s = sk[k];
      const uint32_t a = L[(size_t)i * (N + 1) + k];
      acc += s == 1 ? a : (s == -1 ? (a ? q - a : 0u) : 0u);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    ph[i] = subq(L[(size_t)i * (N + 1) + N], red64(acc, T.pt[i]), q);
  }
  if (lane == 0) msg[c] = crt_decode<NQ>(ph, T, K);
}

// ---------------------------------------------------------------------------
// transforms
// ---------------------------------------------------------------------------

// `per` consecutive polynomials of one prime per workgroup (the prime's
// forward table is copied to LDS once for all of them), two at a time at
// N <= 2048 (one exchange and one set of twiddle loads serve both)
template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_ntt(Tabs T, uint32_t* __restrict__ polys, uint64_t count,
                                                     uint32_t per, int inverse) {
  constexpr bool PR = LOGN <= 11;
  constexpr int KP = PR ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, PR>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8;
  const uint32_t t = threadIdx.x, i = blockIdx.x;
  const uint64_t grp = blockIdx.y + (uint64_t)blockIdx.z * gridDim.y;
  const PrimeTab P = T.pt[i];
  uint32_t xc = 0;
  if (!inverse) load_tw_lds<LOGN>(twl, T.fwd[i], t);  // read after the first exchange's barrier
#pragma unroll 1
  for (uint32_t k = 0; k < per; k += KP) {
    const uint64_t c = grp * per + k;
    if (c >= count) break;
    if (PR && k + 1 < per && c + 1 < count) {
      uint32_t* p[2] = {polys + (c * NQ + i) * (size_t)N, polys + ((c + 1) * NQ + i) * (size_t)N};
      uint32_t x[2][8];
      if (!inverse) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int e = 0; e < 8; ++e) x[m][e] = p[m][t + TT * e];
        ntt_fwd_k<LOGN, 2>(x, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          uint4* o = reinterpret_cast<uint4*>(p[m] + (t << 3));
          o[0] = make_uint4(red4q(x[m][0], P.q, P.two_q), red4q(x[m][1], P.q, P.two_q),
                            red4q(x[m][2], P.q, P.two_q), red4q(x[m][3], P.q, P.two_q));
          o[1] = make_uint4(red4q(x[m][4], P.q, P.two_q), red4q(x[m][5], P.q, P.two_q),
                            red4q(x[m][6], P.q, P.two_q), red4q(x[m][7], P.q, P.two_q));
        }
      } else {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const uint4* s = reinterpret_cast<const uint4*>(p[m] + (t << 3));
          const uint4 u = s[0], v = s[1];
          x[m][0] = u.x; x[m][1] = u.y; x[m][2] = u.z; x[m][3] = u.w;
          x[m][4] = v.x; x[m][5] = v.y; x[m][6] = v.z; x[m][7] = v.w;
        }
        __syncthreads();  // every thread has read its inputs before anyone overwrites them
        ntt_inv_k<LOGN, 2>(x, T.inv[i], P, lds, xc, t);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int e = 0; e < 8; ++e) p[m][t + TT * e] = x[m][e];
      }
      continue;
    }
    uint32_t* p = polys + (c * NQ + i) * (size_t)N;
    uint32_t x[8];
    if (!inverse) {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = p[t + TT * e];
      ntt_fwd<LOGN>(x, T.fwd[i], twl, P.q, P.two_q, lds, xc, t);
      uint4* o = reinterpret_cast<uint4*>(p + (t << 3));
      o[0] = make_uint4(red4q(x[0], P.q, P.two_q), red4q(x[1], P.q, P.two_q), red4q(x[2], P.q, P.two_q),
                        red4q(x[3], P.q, P.two_q));
      o[1] = make_uint4(red4q(x[4], P.q, P.two_q), red4q(x[5], P.q, P.two_q), red4q(x[6], P.q, P.two_q),
                        red4q(x[7], P.q, P.two_q));
    } else {
      const uint4* s = reinterpret_cast<const uint4*>(p + (t << 3));
      const uint4 u = s[0], v = s[1];
      x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w; x[4] = v.x; x[5] = v.y; x[6] = v.z; x[7] = v.w;
      __syncthreads();  // every thread has read its inputs before anyone overwrites them
      ntt_inv<LOGN>(x, T.inv[i], P, lds, xc, t);
#pragma unroll
      for (int e = 0; e < 8; ++e) p[t + TT * e] = x[e];
    }
  }
}

template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_rgsw_export(Tabs T, const uint32_t* __restrict__ rgsw,
                                                               uint32_t* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  constexpr int N = 1 << LOGN, TT = N / 8;
  const uint32_t t = threadIdx.x;
  const uint64_t poly = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;  // (ct, row, a|b)
  uint32_t xc = 0;
#pragma unroll 1
  for (int i = 0; i < NQ; ++i) {
    const PrimeTab P = T.pt[i];
    const size_t off = (poly * NQ + i) * (size_t)N;
    const uint4* s = reinterpret_cast<const uint4*>(rgsw + off + (t << 3));
    const uint4 u = s[0], v = s[1];
    uint32_t x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    ntt_inv<LOGN>(x, T.inv[i], P, lds, xc, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[off + t + TT * e] = x[e];
  }
}

template <int LOGN, int NQ, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(WAVES_XP, 8))) void k_xp(Tabs T, const uint32_t* __restrict__ rgsw,
                                                      const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                      uint64_t rgsw_words) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, xp_pair<LOGN, NQ>()>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN;
  const uint32_t t = threadIdx.x;
  const uint64_t c = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  uint32_t* o = out + c * (size_t)(2 * NQ * N);
  uint32_t xc = 0;
  ext_prod<LOGN, NQ, xp_pair<LOGN, NQ>(), DIG, gadget_lb<DIG>()>(in + c * (size_t)(2 * NQ * N), rgsw + c * rgsw_words,
                                                                T, lds, twl, xc, t, XpOut{o, nullptr, nullptr, XP_STORE});
}

// ---------------------------------------------------------------------------
// shared pieces of the training and inference kernels
// ---------------------------------------------------------------------------

// xin <- X^ex * acc - acc (coefficients t + T e of every polynomial)
template <int LOGN, int NQ>
__device__ __forceinline__ void rot_diff(const Tabs& T, const uint32_t* __restrict__ acc, int32_t ex,
                                         uint32_t* __restrict__ xin, uint32_t t) {
  constexpr int N = 1 << LOGN, TT = N / 8;
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w) {
    const uint32_t* f = acc + (size_t)w * N;
    uint32_t* o = xin + (size_t)w * N;
    const uint32_t q = T.pt[w % NQ].q;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int32_t k = t + TT * e;
      (o + TT * e)[t] = subq(rot_coef<LOGN>(f, k, ex, q), (f + TT * e)[t], q);
    }
  }
}

// CMUX step of a blind rotation: acc <- acc + C [.] (X^ex acc - acc)
template <int LOGN, int NQ, bool PR = xp_pair<LOGN, NQ>(), int DIG = 5>
__device__ __forceinline__ void cmux_rot(const Tabs& T, uint32_t* __restrict__ acc, int32_t ex,
                                         const uint32_t* __restrict__ C, uint32_t* __restrict__ xin, uint32_t* lds,
                                         uint2* twl, uint32_t& xc, uint32_t t) {
  rot_diff<LOGN, NQ>(T, acc, ex, xin, t);
  ext_prod<LOGN, NQ, PR, DIG, gadget_lb<DIG>()>(xin, C, T, lds, twl, xc, t, XpOut{acc, acc, nullptr, XP_ADD});
  __syncthreads();  // the next rotation reads coefficients other threads wrote
}

template <int LOGN, int NQ>
__device__ __forceinline__ void copy_rlwe(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint32_t t) {
  constexpr int N = 1 << LOGN, TT = N / 8;
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w)
#pragma unroll
    for (int e = 0; e < 8; ++e) (dst + (size_t)w * N + TT * e)[t] = (src + (size_t)w * N + TT * e)[t];
}

// ---------------------------------------------------------------------------
// training: one workgroup per (RAM, sample)
// ---------------------------------------------------------------------------
// The workgroup's block holds k1 output slots and one input slot (xin).
// Slot 0 is the accumulator of the rotation chain (CMUX(C_t, X^{2^t} acc,
// acc)); the CDEMUX tree then expands it in place: level i turns slot j into
// (slot j - C_i [.] slot j, C_i [.] slot j) at slots j and j + 2^i.  The
// `ram == k0` workgroup builds the class counter from the label bits alone.

// Tree node u (created by the level that splits it off) leads to a cell of a
// class below l: with z >= L iff (u mod 2^L) < l, else always (Def. 2: a
// model row holds only those cells).  Leaf d sits in row leaf_row(d) of the
// model: (d >> L) l + (d mod 2^L) when z >= L, d otherwise.
__device__ __forceinline__ bool node_live(uint32_t u, uint32_t z, uint32_t L, uint32_t l) {
  return z < L || (u & ((1u << L) - 1u)) < l;
}

__device__ __forceinline__ uint32_t leaf_row(uint32_t d, uint32_t z, uint32_t L, uint32_t l) {
  return z < L ? d : (d >> L) * l + (d & ((1u << L) - 1u));
}

// dst (=|+=) src over one RLWE, each thread its own coefficients t + T e
template <int LOGN, int NQ>
__device__ __forceinline__ void acc_rlwe(const Tabs& T, uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                         bool store, uint32_t t) {
  constexpr int N = 1 << LOGN, TT = N / 8;
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w) {
    const uint32_t q = T.pt[w % NQ].q;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const size_t k = (size_t)w * N + TT * e + t;
      dst[k] = store ? src[k] : addq(dst[k], src[k], q);
    }
  }
}

// IVP of one (sample, RAM) into its block: acc = (0, Delta), the rotation
// chain over bits z..nb-1, then (when `tree`) the CDEMUX tree over bits
// 0..z-1 creating only the live nodes (a split whose new branch is not live
// is skipped).
// bit(u) returns the RGSW of bit u of the IVP index; the index has L label
// bits and l classes.  Without `dest` leaf d is left in slot d.  With
// `dest`, live leaf d goes to dest[leaf_row(d)] instead: stored when
// `store`, else added (the last tree level writes there directly).
template <int LOGN, int NQ, bool PR = xp_pair<LOGN, NQ>(), int DIG = 5, class BitFn>
__device__ __forceinline__ void ivp_block(const Tabs& T, uint32_t* __restrict__ slot0, uint32_t* __restrict__ xin,
                                          uint32_t nb, uint32_t L, uint32_t l, BitFn&& bit, uint32_t* lds,
                                          uint2* twl, uint32_t t, uint32_t* __restrict__ dest = nullptr,
                                          bool store = false, bool tree = true) {
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr size_t RW = (size_t)2 * NQ * N;
  const uint32_t nr = nb < (uint32_t)LOGN ? nb : (uint32_t)LOGN;
  const uint32_t z = nb - nr;
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w) {
    const uint32_t d0 = w >= NQ ? T.pt[w - NQ].delta : 0u;
#pragma unroll
    for (int e = 0; e < 8; ++e) (slot0 + (size_t)w * N + TT * e)[t] = (e == 0 && t == 0) ? d0 : 0u;
  }
  __syncthreads();
  uint32_t xc = 0;
  if (nr > 0) {  // the first CMUX acts on (0, Delta): X acc - acc = (0, Delta (X - 1))
    ext_prod_delta<LOGN, NQ, PR, DIG, gadget_lb<DIG>()>(bit(z), T, lds, xc, t, XpOut{slot0, slot0, nullptr, XP_ADD});
    __syncthreads();
  }
#pragma unroll 1
  for (uint32_t st = 1; st < nr; ++st)
    cmux_rot<LOGN, NQ, PR, DIG>(T, slot0, 1 << st, bit(z + st), xin, lds, twl, xc, t);
  if (!tree) return;
#pragma unroll 1
  for (uint32_t lev = 0; lev < z; ++lev) {
    const uint32_t* C = bit(lev);
    const uint32_t n = 1u << lev;
    const bool last = dest && lev + 1 == z;
#pragma unroll 1
    for (uint32_t j = 0; j < n; ++j) {
      if (!node_live(j, z, L, l)) continue;
      uint32_t* sj = slot0 + j * RW;
      if (node_live(j + n, z, L, l)) {
        copy_rlwe<LOGN, NQ>(xin, sj, t);
        if (last)
          ext_prod<LOGN, NQ, PR, DIG, gadget_lb<DIG>()>(
              xin, C, T, lds, twl, xc, t,
              XpOut{dest + leaf_row(j, z, L, l) * RW, xin, dest + leaf_row(j + n, z, L, l) * RW,
                    store ? XP_DEMUX : XP_DEMUX_ACC});
        else
          ext_prod<LOGN, NQ, PR, DIG, gadget_lb<DIG>()>(xin, C, T, lds, twl, xc, t,
                                                        XpOut{sj, xin, slot0 + (j + n) * RW, XP_DEMUX});
      } else if (last) {  // unsplit live leaf
        acc_rlwe<LOGN, NQ>(T, dest + leaf_row(j, z, L, l) * RW, sj, store, t);
      }
    }
  }
  if (dest && z == 0) acc_rlwe<LOGN, NQ>(T, dest, slot0, store, t);  // no tree: the chain's accumulator
}

__device__ __forceinline__ uint32_t ram_bits(uint32_t ram, uint32_t k0, uint32_t s, uint32_t a, uint32_t L) {
  if (ram >= k0) return L;  // the class counter: label bits only
  const uint32_t rem = s - ram * a;
  return L + (rem < a ? rem : a);
}

// model rows of a RAM with nb index bits: its live leaves
__device__ __forceinline__ uint32_t ram_rows(uint32_t nb, uint32_t logN, uint32_t L, uint32_t l) {
  const uint32_t z = nb - (nb < logN ? nb : logN);
  return z >= L ? l << (z - L) : 1u << z;
}

// Two model layouts.  Layout 0 (label-pruned rows): the IVP index is [label
// bits, tuple bits], the label bits are the lowest tree levels and only the
// leaves of classes below l are rows.  Layout 1 (class-packed rows): the
// index is [tuple bits, label bits]; the tree holds tuple bits only, every
// leaf is a row and the class of a cell sets its coefficient, so one VP over
// the tuple bits reads the cells of all classes.  tree_L / tree_l give the
// label bits at the bottom of the tree and their classes: (L, l), or (0, 1)
// for layout 1, for which node_live, leaf_row and ram_rows keep every node.
__device__ __forceinline__ uint32_t tree_L(uint32_t layout, uint32_t L) { return layout ? 0u : L; }
__device__ __forceinline__ uint32_t tree_l(uint32_t layout, uint32_t l) { return layout ? 1u : l; }

// RGSW of bit u of the IVP index of (sample gi, RAM ram), nb index bits; the
// class counter (ram == k0) has only label bits
__device__ __forceinline__ const uint32_t* index_bit(uint32_t layout, uint32_t u, uint32_t nb, uint32_t L,
                                                     const uint32_t* __restrict__ x, const uint32_t* __restrict__ y,
                                                     const uint32_t* __restrict__ perm, uint64_t gi, uint32_t s,
                                                     uint32_t ram, uint32_t a, uint64_t rgsw_words) {
  if (layout == 0) {
    if (u < L) return y + (gi * L + u) * rgsw_words;
    return x + (gi * s + perm[ram * a + (u - L)]) * rgsw_words;
  }
  const uint32_t aj = nb - L;
  if (u < aj) return x + (gi * s + perm[ram * a + u]) * rgsw_words;
  return y + (gi * L + (u - aj)) * rgsw_words;
}

template <int LOGN, int NQ, int OCC, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_train(Tabs T, TrainArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, xp_pair<LOGN, NQ>()>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr size_t RW = (size_t)2 * NQ * (1 << LOGN);
  const uint32_t t = threadIdx.x;
  uint32_t ram, smp;
  if (A.map == 0) {  // 2-D grid, RAMs of one sample on consecutive workgroups
    ram = blockIdx.x;
    smp = blockIdx.y;
  } else {  // 1-D grid; XCD x (= workgroup id mod 8) takes the x-th eighth of the items
    const uint32_t G = A.nram * A.nsub, per = (G + 7) >> 3;
    const uint32_t lg = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    if (lg >= G) return;
    ram = lg % A.nram;
    smp = lg / A.nram;
  }
  const uint64_t gi = A.i0 + smp;
  uint32_t* slot0 = A.out + ((size_t)smp * (A.k0 + 1) + ram) * (A.kt + 1) * RW;
  const uint32_t nb = ram_bits(ram, A.k0, A.s, A.a, A.L);
  ivp_block<LOGN, NQ, xp_pair<LOGN, NQ>(), DIG>(T, slot0, slot0 + (size_t)A.kt * RW, nb, tree_L(A.layout, A.L),
                                               tree_l(A.layout, A.l),
                      [&](uint32_t u) -> const uint32_t* {
                        return index_bit(A.layout, u, nb, A.L, A.x_rgsw, A.y_rgsw, A.perm, gi, A.s, ram, A.a,
                                         A.rgsw_words);
                      },
                      lds, twl, t, nullptr, false, A.tree != 0);
}

// One level of the CDEMUX tree for a whole sub-batch, after k_train has run
// the chains alone (A.tree = 0): one workgroup per (sample, RAM, live split
// at level A.lev).  The splits of a level all use the RGSW of bit A.lev: the
// label bits' are shared by every RAM of a sample (layout 0), a tuple bit's
// by the splits of one (sample, RAM).  Items are numbered (sample, RAM,
// split) with the split fastest and each XCD (workgroup id mod 8) takes a
// contiguous eighth of them, so the workgroups that read one RGSW run
// side by side on one XCD and share its L2, where the chain's workgroup
// would stream that RGSW once per node.  Split j of node j (slot j) writes
// h = C [.] slot j to slot j + 2^lev, then slot j -= h: the bits of the
// in-workgroup tree (XP_DEMUX), with no input copy (ext_prod reads every
// input coefficient before the subtraction, each thread its own).
template <int LOGN, int NQ, int OCC, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_train_level(
    Tabs T, TrainArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, xp_pair<LOGN, NQ>()>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr size_t RW = (size_t)2 * NQ * N;
  const uint32_t t = threadIdx.x;
  const uint64_t G = (uint64_t)A.nram * A.nsub * A.smax, per = (G + 7) >> 3;
  const uint64_t it = (uint64_t)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (it >= G) return;
  const uint32_t sp = (uint32_t)(it % A.smax);
  const uint64_t rs = it / A.smax;
  const uint32_t ram = (uint32_t)(rs % A.nram), smp = (uint32_t)(rs / A.nram);
  const uint32_t nb = ram_bits(ram, A.k0, A.s, A.a, A.L);
  const uint32_t z = nb - (nb < (uint32_t)LOGN ? nb : (uint32_t)LOGN);
  if (A.lev >= z) return;
  const uint32_t n = 1u << A.lev, tL = tree_L(A.layout, A.L), tl = tree_l(A.layout, A.l);
  uint32_t j = 0, c = 0;  // the sp-th live split of the level (uniform over the workgroup)
  for (; j < n; ++j)
    if (node_live(j, z, tL, tl) && node_live(j + n, z, tL, tl)) {
      if (c == sp) break;
      ++c;
    }
  if (j == n) return;
  const uint64_t gi = A.i0 + smp;
  uint32_t* slot0 = A.out + ((size_t)smp * (A.k0 + 1) + ram) * (A.kt + 1) * RW;
  uint32_t* sj = slot0 + (size_t)j * RW;
  uint32_t* sn = slot0 + (size_t)(j + n) * RW;
  const uint32_t* C = index_bit(A.layout, A.lev, nb, A.L, A.x_rgsw, A.y_rgsw, A.perm, gi, A.s, ram, A.a,
                                A.rgsw_words);
  uint32_t xc = 0;
  ext_prod<LOGN, NQ, xp_pair<LOGN, NQ>(), DIG, gadget_lb<DIG>()>(sj, C, T, lds, twl, xc, t,
                                                                XpOut{sn, nullptr, nullptr, XP_STORE});
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w) {
    const uint32_t q = T.pt[w % NQ].q;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const size_t k = (size_t)w * N + TT * e + t;
      sj[k] = subq(sj[k], sn[k], q);
    }
  }
}

// ---------------------------------------------------------------------------
// batched training: one persistent launch over many jobs of one parameter set
// ---------------------------------------------------------------------------
// An item is (job, RAM, piece): the piece's samples [piece*per, ...) run the
// IVP of that RAM one after another in the workgroup's private scratch (k1
// slots + the input slot); the last CDEMUX level of each sample adds its 2^z
// outputs into the piece's destination: the model row itself for piece 0 (no
// other item writes it), else the piece's accumulator in the workspace
// (stored by the piece's first sample).  Items come from a queue (a device counter),
// longest first; a workgroup leaves when the queue is exhausted.
// k_reduce_batch then adds the accumulators of pieces >= 1 into the models.

template <int LOGN, int NQ, int OCC, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_train_batch(
    Tabs T, BatchArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, false>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  __shared__ uint32_t next;
  constexpr size_t RW = (size_t)2 * NQ * (1 << LOGN);
  const uint32_t t = threadIdx.x;
  uint32_t* slot0 = A.ws + (size_t)blockIdx.x * A.scratch_words;
#pragma unroll 1
  for (;;) {
    if (t == 0) next = atomicAdd(A.counter, 1u);
    __syncthreads();
    // uniform over the workgroup: item and job descriptors then come through
    // scalar loads and their address arithmetic stays on the scalar unit
    const uint32_t it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= A.nitems) break;
    const BItem I = A.items[it];
    const BJob J = A.jobs[I.job];
    const uint32_t nb = ram_bits(I.ram, J.k0, J.s, J.a, J.L);
    uint32_t* dest = I.piece == 0 ? (I.ram < J.k0 ? J.model + (size_t)I.ram * J.k1 * RW : J.cnt)
                                  : A.acc + J.acc0 + ((size_t)(I.piece - 1) * J.nram + I.ram) * J.k1 * RW;
    const uint32_t s0 = I.piece * J.per;
    const uint32_t s1 = s0 + J.per < J.nsmp ? s0 + J.per : J.nsmp;
#pragma unroll 1
    for (uint32_t smp = s0; smp < s1; ++smp) {
      const uint64_t gi = smp;
      // single transforms: with pairs the queue state next to them spills registers
      ivp_block<LOGN, NQ, false, DIG>(T, slot0, slot0 + (size_t)J.kt * RW, nb, tree_L(J.layout, J.L),
                                 tree_l(J.layout, J.l),
                          [&](uint32_t u) -> const uint32_t* {
                            return index_bit(J.layout, u, nb, J.L, J.x, J.y, J.perm, gi, J.s, I.ram, J.a,
                                             A.rgsw_words);
                          },
                          lds, twl, t, dest, I.piece != 0 && smp == s0);
      __syncthreads();
    }
  }
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// model[j][d] (+ counter) += the accumulators of pieces 1..pieces-1 of every
// job with more than one piece; one thread per model word, the job found by
// binary search over the prefix words0 (jobs with one piece span no words)
__global__ __launch_bounds__(256) void k_reduce_batch(Tabs T, const BJob* __restrict__ jobs, uint32_t njobs,
                                                      uint64_t total, uint32_t logN, uint32_t N, uint32_t nq,
                                                      const uint32_t* __restrict__ acc) {
  const size_t RW = (size_t)2 * nq * N;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (size_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = njobs;  // last job with words0 <= w
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (jobs[mid].words0 <= w) lo = mid; else hi = mid;
    }
    const BJob J = jobs[lo];
    const size_t per_ram = (size_t)J.k1 * RW;
    const size_t model_words = (size_t)J.k0 * per_ram;
    const size_t x = w - J.words0;
    uint32_t ram;
    size_t off;  // word within the RAM's k1 slots
    if (x < model_words) {
      ram = (uint32_t)(x / per_ram);
      off = x - (size_t)ram * per_ram;
      if (off / RW >= ram_rows(ram_bits(ram, J.k0, J.s, J.a, J.L), logN, tree_L(J.layout, J.L),
                               tree_l(J.layout, J.l)))
        continue;
    } else {
      ram = J.k0;
      off = x - model_words;
    }
    const PrimeTab P = T.pt[(off / N) % nq];
    const uint32_t* src = acc + J.acc0 + (size_t)ram * per_ram + off;
    const size_t stride = (size_t)J.nram * per_ram;  // one piece
    uint64_t sum = 0;
    for (uint32_t p = 1; p < J.pieces; ++p) sum += src[(size_t)(p - 1) * stride];
    uint32_t* dst = x < model_words ? J.model + x : J.cnt + off;
    *dst = addq(*dst, red64(sum, P), P.q);
  }
}

// model[j][row] += sum over the sub-batch of out[smp][j][leaf] for every live
// leaf of RAM j (row = leaf_row(leaf)); cnt += sum of out[smp][k0][0].  One
// thread per model word.
__global__ __launch_bounds__(256) void k_reduce_model(Tabs T, ReduceArgs A) {
  const size_t RW = (size_t)2 * A.nq * A.N;
  const size_t per_ram = (size_t)A.k1 * RW;
  const size_t model_words = (size_t)A.k0 * per_ram;
  const size_t total = model_words + (A.cnt ? RW : 0);
  const size_t blk = (size_t)(A.kt + 1) * RW;      // one (sample, RAM) block: the tree's leaves + input slot
  const size_t stride = (size_t)(A.k0 + 1) * blk;  // one sample
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (size_t)gridDim.x * blockDim.x) {
    uint32_t ram, d;
    size_t rem;
    if (w < model_words) {
      ram = (uint32_t)(w / per_ram);
      rem = w - (size_t)ram * per_ram;
      const uint32_t row = (uint32_t)(rem / RW);
      rem -= (size_t)row * RW;
      const uint32_t nb = ram_bits(ram, A.k0, A.s, A.a, A.L);
      const uint32_t pL = tree_L(A.layout, A.L), pl = tree_l(A.layout, A.l);
      if (row >= ram_rows(nb, A.logN, pL, pl)) continue;
      const uint32_t z = nb - (nb < A.logN ? nb : A.logN);
      d = z < pL ? row : ((row / pl) << pL) + row % pl;  // the leaf of this row
    } else {
      ram = A.k0;
      d = 0;
      rem = w - model_words;
    }
    const uint32_t i = (uint32_t)((rem / A.N) % A.nq);
    const PrimeTab P = T.pt[i];
    const size_t src = (size_t)ram * blk + (size_t)d * RW + rem;
    uint64_t acc = 0;
    for (uint64_t s = 0; s < A.n_sub; ++s) acc += A.out[s * stride + src];
    uint32_t* dst = (w < model_words) ? (A.model + w) : (A.cnt + rem);
    *dst = addq(*dst, red64(acc, P), P.q);
  }
}

// layout 2 rows (several RAMs per row): dst[R] (+)= the sum over samples s
// and the RAMs t of the row of X^(t 2^nbf) src(s, R rpr + t).  Coefficient k
// of X^e f is f[k - e] for k >= e and -f[N + k - e] below (0 <= e < N).  One
// thread per output word; the class counter's words follow the rows.
__global__ __launch_bounds__(256) void k_row_pack(Tabs T, RowPackArgs A) {
  const size_t RW = (size_t)2 * A.nq * A.N;
  const size_t row_words = (size_t)A.rows * RW;
  const size_t total = row_words + (A.cnt && !A.store ? RW : 0);
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (size_t)gridDim.x * blockDim.x) {
    uint64_t acc = 0;
    uint32_t* dst;
    uint32_t i;
    if (w < row_words) {
      const uint32_t R = (uint32_t)(w / RW);
      const size_t rem = w - (size_t)R * RW;
      const uint32_t k = (uint32_t)(rem % A.N);
      const size_t poly = rem - k;  // the polynomial's first word within an RLWE
      i = (uint32_t)((rem / A.N) % A.nq);
      const uint32_t q = T.pt[i].q;
      for (uint32_t t = 0; t < A.rpr; ++t) {
        const uint32_t j = R * A.rpr + t;
        if (j >= A.k0) break;
        const uint32_t e = t << A.nbf;  // t 2^nbf < N
        const bool wrap = k < e;
        const uint32_t* src = A.src + (size_t)j * A.rstride + poly + (wrap ? k + A.N - e : k - e);
        for (uint64_t sm = 0; sm < A.nsmp; ++sm) {
          const uint32_t v = src[sm * A.sstride];
          acc += wrap ? (v ? q - v : 0u) : v;
        }
      }
      dst = A.dst + w;
    } else {  // class counter: sample sums of RAM block k0, unrotated
      const size_t rem = w - row_words;
      i = (uint32_t)((rem / A.N) % A.nq);
      const uint32_t* src = A.src + (size_t)A.k0 * A.rstride + rem;
      for (uint64_t sm = 0; sm < A.nsmp; ++sm) acc += src[sm * A.sstride];
      dst = A.cnt + rem;
    }
    const PrimeTab P = T.pt[i];
    const uint32_t r = red64(acc, P);
    *dst = A.store ? r : addq(*dst, r, P.q);
  }
}

// ---------------------------------------------------------------------------
// inference: one workgroup per (RAM, label, sample), or per (RAM, sample)
// ---------------------------------------------------------------------------
// Layout 0: Vertical Packing of row `ram` of the model for the label bits of
// c (clear) and the sample's tuple bits (encrypted).  Levels of the selection
// tree that carry label bits select exactly; only the 2^{z-L} - 1 CMUXes
// whose outputs reach the result are evaluated (the discarded ones do not
// change it).  Layout 1: one VP over the tuple bits (the full tree over the
// row's 2^z leaves, then the chain); the label bits above them are clear
// zeros, and the cell of class c ends at coefficient c 2^(a_j - z), so the
// workgroup extracts the LWE of every class.  Layout 2 reads RAM j from row
// j / rpr, whose block from coefficient (j mod rpr) 2^nbf holds it; the
// extraction indices move by that offset.

// The VP of (sample gi, RAM ram, label lab) with the workgroup's slots acc
// (A.slots RLWE) and input slot xin; writes its LWE score(s) into A.scores.
template <int LOGN, int NQ, bool PR = xp_pair<LOGN, NQ>(), int DIG = 5>
__device__ __forceinline__ void vp_one(const Tabs& T, const InferArgs& A, uint64_t gi, uint32_t ram, uint32_t lab,
                                       uint32_t* __restrict__ acc, uint32_t* __restrict__ xin, uint32_t* lds,
                                       uint2* twl, uint32_t t) {
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr size_t RW = (size_t)2 * NQ * N;
  const uint32_t rem = A.s - ram * A.a;
  const uint32_t aj = rem < A.a ? rem : A.a;
  const uint32_t nb = A.L + aj;
  const uint32_t nr = nb < (uint32_t)LOGN ? nb : (uint32_t)LOGN;
  const uint32_t z = nb - nr;
  const uint32_t TL = tree_L(A.layout, A.L);  // label bits at the bottom of the tree
  const uint32_t tl = tree_l(A.layout, A.l);  // rows per group of leaves
  const uint32_t* H = A.model + (size_t)(ram / A.rpr) * A.k1 * RW;
  const uint32_t off = (ram % A.rpr) << A.nbf;  // 0 unless layout 2
  auto xbit = [&](uint32_t u) -> const uint32_t* {
    return A.x_rgsw + (gi * A.s + A.perm[ram * A.a + (u - TL)]) * A.rgsw_words;
  };
  uint32_t xc = 0;
  if (z > TL) {
    // encrypted levels z-1 .. TL over the leaves lab + (w << TL); the clear
    // levels below TL then select leaf index lab exactly
#pragma unroll 1
    for (int lev = (int)z - 1; lev >= (int)TL; --lev) {
      const uint32_t* C = xbit((uint32_t)lev);
      const uint32_t cnt = 1u << (lev - TL);
#pragma unroll 1
      for (uint32_t w = 0; w < cnt; ++w) {
        const bool leaf = lev == (int)z - 1;
        // leaves lab + 2^TL w and lab + 2^TL (w + cnt) are rows w tl + lab and (w + cnt) tl + lab
        const uint32_t* lo = leaf ? H + (size_t)(w * tl + lab) * RW : acc + (size_t)w * RW;
        const uint32_t* hi = leaf ? H + (size_t)((w + cnt) * tl + lab) * RW : acc + (size_t)(w + cnt) * RW;
        uint32_t* dst = acc + (size_t)w * RW;
#pragma unroll 1
        for (int pw = 0; pw < 2 * NQ; ++pw) {
          const uint32_t q = T.pt[pw % NQ].q;
          const size_t o = (size_t)pw * N;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            (xin + o + TT * e)[t] = subq((hi + o + TT * e)[t], (lo + o + TT * e)[t], q);
        }
        ext_prod<LOGN, NQ, PR, DIG, gadget_lb<DIG>()>(xin, C, T, lds, twl, xc, t, XpOut{dst, lo, nullptr, XP_ADD});
      }
    }
  } else {
    copy_rlwe<LOGN, NQ>(acc, H + (size_t)(lab & ((1u << z) - 1)) * RW, t);
  }
  __syncthreads();
#pragma unroll 1
  for (uint32_t st = 0; st < nr; ++st) {
    const uint32_t u = z + st;
    const int32_t ex = -(1 << st);
    if (A.layout && u >= aj) break;  // the label bits on top: clear zeros, no rotation
    if (!A.layout && u < A.L) {
      if ((lab >> u) & 1u) {  // clear bit 1: exact rotation by X^{-2^st}
        rot_diff<LOGN, NQ>(T, acc, ex, xin, t);  // xin = X^ex acc - acc
        __syncthreads();
#pragma unroll 1
        for (int w = 0; w < 2 * NQ; ++w) {
          const uint32_t q = T.pt[w % NQ].q;
          const size_t o = (size_t)w * N;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            (acc + o + TT * e)[t] = addq((acc + o + TT * e)[t], (xin + o + TT * e)[t], q);
        }
        __syncthreads();
      }
      continue;
    }
    cmux_rot<LOGN, NQ, PR, DIG>(T, acc, ex, xbit(u), xin, lds, twl, xc, t);
  }
  // ExtractLWE(acc, idx) for the class(es) of this workgroup: a'_k = a_{idx-k}
  // for k <= idx, -a_{N+idx-k} above, b' = b_idx; idx = 0 for layout 0,
  // off + c 2^(a_j - z) for class c of layouts 1-2 (below N: off + 2^nbf <= N)
  const uint32_t nout = A.layout ? A.l : 1u;
#pragma unroll 1
  for (uint32_t cc = 0; cc < nout; ++cc) {
    const uint32_t cls = A.layout ? cc : lab;
    const uint32_t idx = A.layout ? off + (cc << (aj - z)) : 0u;
    uint32_t* out = A.scores + ((gi * A.l + cls) * A.k0 + ram) * (size_t)NQ * (N + 1);
#pragma unroll 1
    for (int i = 0; i < NQ; ++i) {
      const uint32_t q = T.pt[i].q;
      const uint32_t* a = acc + (size_t)i * N;
      uint32_t* o = out + (size_t)i * (N + 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t k = t + TT * e;
        const bool lo = k <= idx;
        const uint32_t x = a[lo ? idx - k : N + idx - k];
        (o + TT * e)[t] = (lo || x == 0) ? x : q - x;
      }
      if (t == 0) o[N] = acc[(size_t)(NQ + i) * N + idx];
    }
  }
}

template <int LOGN, int NQ, int OCC, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_infer(Tabs T, InferArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, xp_pair<LOGN, NQ>()>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr size_t RW = (size_t)2 * NQ * (1 << LOGN);
  const uint32_t t = threadIdx.x;
  uint32_t ram, lab, smp;
  if (A.map == 0) {  // 3-D grid (RAM, label, sample)
    ram = blockIdx.x;
    lab = blockIdx.y;
    smp = blockIdx.z;
  } else {  // 1-D grid, the labels of one (sample, RAM) adjacent, XCD x takes the x-th eighth
    const uint32_t G = A.k0 * A.nlab * A.nsub, per = (G + 7) >> 3;
    const uint32_t lg = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    if (lg >= G) return;
    lab = lg % A.nlab;
    ram = (lg / A.nlab) % A.k0;
    smp = lg / A.nlab / A.k0;
  }
  uint32_t* acc = A.scratch + (((size_t)smp * A.nlab + lab) * A.k0 + ram) * (A.slots + 1) * RW;
  vp_one<LOGN, NQ, xp_pair<LOGN, NQ>(), DIG>(T, A, A.i0 + smp, ram, lab, acc, acc + (size_t)A.slots * RW, lds, twl, t);
}

// ---------------------------------------------------------------------------
// batched inference: one persistent launch over many jobs of one parameter set
// ---------------------------------------------------------------------------
// An item is (job, RAM, label, piece): the VPs of the piece's samples [piece
// per, ...) for that RAM and label (every label at once for layouts 1-2),
// one after another in the workgroup's private slots.  Each VP writes its
// own scores, so no reduction follows.  Items come from a queue (a device
// counter), longest first; a workgroup leaves when the queue is exhausted.
template <int LOGN, int NQ, int OCC, int DIG = 5>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_infer_batch(
    Tabs T, IBatchArgs B) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, false>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  __shared__ uint32_t next;
  const uint32_t t = threadIdx.x;
  uint32_t* acc = B.ws + (size_t)blockIdx.x * B.scratch_words;
#pragma unroll 1
  for (;;) {
    if (t == 0) next = atomicAdd(B.counter, 1u);
    __syncthreads();
    const uint32_t it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= B.nitems) break;
    const IItem I = B.items[it];
    const IJob& J = B.jobs[I.job];
    const uint32_t s0 = I.piece * J.per;
    const uint32_t s1 = s0 + J.per < J.nsmp ? s0 + J.per : J.nsmp;
    const size_t slot_words = (size_t)J.args.slots * 2 * NQ * (1 << LOGN);
#pragma unroll 1
    for (uint32_t smp = s0; smp < s1; ++smp) {
      // single transforms: with pairs the queue state next to them spills registers
      vp_one<LOGN, NQ, false, DIG>(T, J.args, smp, I.ram, I.lab, acc, acc + slot_words, lds, twl, t);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// PackingKeySwitching: count groups of k LWE -> one RLWE each
// ---------------------------------------------------------------------------
// out = (0, sum_i b_i X^i) - sum_{j,r} P_{j,r} K[j][r] with P_{j,r} = sum_i
// d_r(a_{i,j}) X^i.  k_pks_partial: one workgroup per (group, output prime,
// block of PKS_J key coordinates) builds each P_{j,r} in registers (thread t
// holds i = t + T e), transforms it and multiply-accumulates it with the
// evaluation-domain key rows; the block's partial sums (a and b parts) go to
// the workspace in the evaluation domain.  k_pks_finish adds the blocks,
// transforms back and subtracts from (0, sum_i b_i X^i).
constexpr uint32_t PKS_J = 32;

template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(WAVES_XP, 8))) void k_pks_partial(
    Tabs T, PksArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8, D = 5 * NQ;
  constexpr size_t ROW = (size_t)2 * NQ * N, LW = (size_t)NQ * (N + 1);
  const uint32_t t = threadIdx.x, ip = blockIdx.y, jb = blockIdx.z;
  const uint64_t c = blockIdx.x;  // group fastest: concurrent workgroups share the key block in L2
  const uint32_t* lwe = A.lwe + c * A.k * LW;
  const PrimeTab P = T.pt[ip];
  load_tw_lds<LOGN>(twl, T.fwd[ip], t);  // read after the first exchange's barrier
  uint64_t acc_a[8], acc_b[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) acc_a[e] = acc_b[e] = 0;
  int cnt = 0;
  uint32_t xc = 0;
  const uint32_t j1 = (jb + 1) * PKS_J < (uint32_t)N ? (jb + 1) * PKS_J : (uint32_t)N;
#pragma unroll 1
  for (uint32_t j = jb * PKS_J; j < j1; ++j) {
#pragma unroll 1
    for (int g = 0; g < NQ; ++g) {
      const uint32_t qg = T.pt[g].q;
      int32_t v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t i = t + TT * e;
        const uint32_t r = i < A.k ? lwe[(size_t)i * LW + (size_t)g * (N + 1) + j] : 0u;
        v[e] = (r > (qg - 1) / 2 ? (int32_t)(r - qg) : (int32_t)r) + DIGIT_OFFSET;
      }
#pragma unroll 1
      for (int dt = 0; dt < 5; ++dt) {
        const uint4* kra = reinterpret_cast<const uint4*>(A.key + ((size_t)j * D + g * 5 + dt) * ROW + (size_t)ip * N);
        const uint4* krb = kra + (size_t)NQ * N / 4;
        const uint4 ka0 = kra[2 * t], ka1 = kra[2 * t + 1];
        const uint4 kb0 = krb[2 * t], kb1 = krb[2 * t + 1];
        uint32_t x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = digit_lift(v[e], dt, P.q);  // v: centred residues + DIGIT_OFFSET
        ntt_fwd<LOGN>(x, T.fwd[ip], twl, P.q, P.two_q, lds, xc, t);
        const uint32_t ka[8] = {ka0.x, ka0.y, ka0.z, ka0.w, ka1.x, ka1.y, ka1.z, ka1.w};
        const uint32_t kb[8] = {kb0.x, kb0.y, kb0.z, kb0.w, kb1.x, kb1.y, kb1.z, kb1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t xr = red4q(x[e], P.q, P.two_q);
          acc_a[e] += (uint64_t)xr * ka[e];
          acc_b[e] += (uint64_t)xr * kb[e];
        }
        if (++cnt == 15) {
          cnt = 0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            acc_a[e] = red64(acc_a[e], P);
            acc_b[e] = red64(acc_b[e], P);
          }
        }
      }
    }
  }
  uint32_t* o = A.part + ((c * NQ + ip) * gridDim.z + jb) * (size_t)(2 * N);
  uint4* oa = reinterpret_cast<uint4*>(o + (t << 3));
  uint4* ob = reinterpret_cast<uint4*>(o + N + (t << 3));
  oa[0] = make_uint4(red64(acc_a[0], P), red64(acc_a[1], P), red64(acc_a[2], P), red64(acc_a[3], P));
  oa[1] = make_uint4(red64(acc_a[4], P), red64(acc_a[5], P), red64(acc_a[6], P), red64(acc_a[7], P));
  ob[0] = make_uint4(red64(acc_b[0], P), red64(acc_b[1], P), red64(acc_b[2], P), red64(acc_b[3], P));
  ob[1] = make_uint4(red64(acc_b[4], P), red64(acc_b[5], P), red64(acc_b[6], P), red64(acc_b[7], P));
}

template <int LOGN, int NQ>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_pks_finish(Tabs T, PksArgs A, uint32_t nblk) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * Geo<LOGN>::LDSW];
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr size_t LW = (size_t)NQ * (N + 1);
  const uint32_t t = threadIdx.x, ip = blockIdx.x;
  const uint64_t c = blockIdx.y;
  const PrimeTab P = T.pt[ip];
  const uint32_t* part = A.part + (c * NQ + ip) * (size_t)nblk * (2 * N);
  uint64_t sa[8], sb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) sa[e] = sb[e] = 0;
#pragma unroll 1
  for (uint32_t b = 0; b < nblk; ++b) {  // at most 128 words below 2^30 each: no overflow
    const uint4* pa = reinterpret_cast<const uint4*>(part + (size_t)b * 2 * N + (t << 3));
    const uint4* pb = reinterpret_cast<const uint4*>(part + (size_t)b * 2 * N + N + (t << 3));
    const uint4 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
    sa[0] += a0.x; sa[1] += a0.y; sa[2] += a0.z; sa[3] += a0.w;
    sa[4] += a1.x; sa[5] += a1.y; sa[6] += a1.z; sa[7] += a1.w;
    sb[0] += b0.x; sb[1] += b0.y; sb[2] += b0.z; sb[3] += b0.w;
    sb[4] += b1.x; sb[5] += b1.y; sb[6] += b1.z; sb[7] += b1.w;
  }
  uint32_t ha[8], hb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    ha[e] = red64(sa[e], P);
    hb[e] = red64(sb[e], P);
  }
  uint32_t xc = 0;
  ntt_inv<LOGN>(ha, T.inv[ip], P, lds, xc, t);
  ntt_inv<LOGN>(hb, T.inv[ip], P, lds, xc, t);
  const uint32_t* lwe = A.lwe + c * A.k * LW;
  uint32_t* out = A.out + c * (size_t)(2 * NQ * N);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t i = t + TT * e;
    const uint32_t b = i < A.k ? lwe[(size_t)i * LW + (size_t)ip * (N + 1) + N] : 0u;
    out[(size_t)ip * N + i] = subq(0u, ha[e], P.q);
    out[(size_t)(NQ + ip) * N + i] = subq(b, hb[e], P.q);
  }
}

// dst += src over `words` words of RLWE ciphertexts (2 nq N words each),
// residue by residue; a thread adds four consecutive words (16-byte accesses)
__global__ __launch_bounds__(256) void k_rlwe_add(Tabs T, uint32_t* __restrict__ dst,
                                                  const uint32_t* __restrict__ src, uint64_t words, uint32_t N,
                                                  uint32_t nq) {
  const uint64_t n4 = words / 4;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n4; v += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t q = T.pt[(uint32_t)((4 * v / N) % nq)].q;  // N >= 4: four words share a prime
    const uint4 a = reinterpret_cast<const uint4*>(dst)[v], b = reinterpret_cast<const uint4*>(src)[v];
    reinterpret_cast<uint4*>(dst)[v] = make_uint4(addq(a.x, b.x, q), addq(a.y, b.y, q), addq(a.z, b.z, q),
                                                  addq(a.w, b.w, q));
  }
}

// sums[i][c] = sum_j scores[i][c][j] (LWE addition), one thread per word
__global__ __launch_bounds__(256) void k_class_sums(Tabs T, SumArgs A) {
  const size_t LW = (size_t)A.nq * (A.N + 1);
  const size_t total = (size_t)A.n * A.l * LW;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (size_t)gridDim.x * blockDim.x) {
    const size_t ic = w / LW, rem = w - ic * LW;
    const uint32_t i = (uint32_t)(rem / (A.N + 1));
    const uint32_t* src = A.scores + ic * A.k0 * LW + rem;
    uint64_t acc = 0;
    for (uint32_t j = 0; j < A.k0; ++j) acc += src[(size_t)j * LW];
    A.sums[w] = red64(acc, T.pt[i]);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// launch a 1-D family of `count` jobs as exact rectangles of (x, y) blocks;
// a kernel recovers its job as blockIdx.x + blockIdx.y * gridDim.x (or the
// same over y, z when x indexes something else)
template <class F>
static hipError_t for_rect(uint64_t count, F&& f) {
  uint64_t done = 0;
  while (done < count) {
    const uint64_t left = count - done;
    uint32_t x, y;
    if (left <= 65535) {
      x = (uint32_t)left;
      y = 1;
    } else {
      x = 65535;
      y = (uint32_t)(left / 65535 < 65535 ? left / 65535 : 65535);
    }
    const hipError_t e = f(done, dim3(x, y));
    if (e != hipSuccess) return e;
    done += (uint64_t)x * y;
  }
  return hipSuccess;
}

#define HW_DISPATCH(logN, nq, ...)                                                     \
  do {                                                                                 \
    if (logN == 10 && nq == 1) { constexpr int LN = 10, NQ = 1; __VA_ARGS__; }         \
    else if (logN == 10 && nq == 2) { constexpr int LN = 10, NQ = 2; __VA_ARGS__; }    \
    else if (logN == 10 && nq == 3) { constexpr int LN = 10, NQ = 3; __VA_ARGS__; }    \
    else if (logN == 11 && nq == 1) { constexpr int LN = 11, NQ = 1; __VA_ARGS__; }    \
    else if (logN == 11 && nq == 2) { constexpr int LN = 11, NQ = 2; __VA_ARGS__; }    \
    else if (logN == 11 && nq == 3) { constexpr int LN = 11, NQ = 3; __VA_ARGS__; }    \
    else if (logN == 12 && nq == 1) { constexpr int LN = 12, NQ = 1; __VA_ARGS__; }    \
    else if (logN == 12 && nq == 2) { constexpr int LN = 12, NQ = 2; __VA_ARGS__; }    \
    else if (logN == 12 && nq == 3) { constexpr int LN = 12, NQ = 3; __VA_ARGS__; }    \
    else return hipErrorInvalidValue;                                                  \
  } while (0)

// HW_DISPATCH with the occupancy target OC: 4 exists for log2 N = 12 only
#define HW_DISPATCH_OCC(logN, nq, occ, ...)                                              \
  do {                                                                                 \
    if (logN == 12 && occ == 4) {                                                      \
      if (nq == 1) { constexpr int LN = 12, NQ = 1, OC = 4; __VA_ARGS__; }             \
      else if (nq == 2) { constexpr int LN = 12, NQ = 2, OC = 4; __VA_ARGS__; }        \
      else if (nq == 3) { constexpr int LN = 12, NQ = 3, OC = 4; __VA_ARGS__; }        \
      else return hipErrorInvalidValue;                                                \
    } else {                                                                           \
      HW_DISPATCH(logN, nq, constexpr int OC = WAVES_XP; __VA_ARGS__);                 \
    }                                                                                  \
  } while (0)

// The gadget of the RGSW a launch reads, as DG (digits per prime): 5 (6-bit
// digits) on any ring, 2 (15-bit digits) on rings of two or more primes; the
// 2-digit kernels are built for those rings only.
#define HW_DISPATCH_G(logN, nq, dig, ...)                                                     \
  do {                                                                                        \
    if (dig == 5) {                                                                           \
      constexpr int DG = 5;                                                                   \
      HW_DISPATCH(logN, nq, __VA_ARGS__);                                                     \
    } else if (dig == 2 && nq >= 2) {                                                         \
      constexpr int DG = 2;                                                                   \
      HW_DISPATCH(logN, nq, if constexpr (NQ >= 2) { __VA_ARGS__; } else return hipErrorInvalidValue;); \
    } else {                                                                                  \
      return hipErrorInvalidValue;                                                            \
    }                                                                                         \
  } while (0)

#define HW_DISPATCH_GOCC(logN, nq, occ, dig, ...)                                             \
  do {                                                                                        \
    if (dig == 5) {                                                                           \
      constexpr int DG = 5;                                                                   \
      HW_DISPATCH_OCC(logN, nq, occ, __VA_ARGS__);                                            \
    } else if (dig == 2 && nq >= 2) {                                                         \
      constexpr int DG = 2;                                                                   \
      HW_DISPATCH_OCC(logN, nq, occ, if constexpr (NQ >= 2) { __VA_ARGS__; } else return hipErrorInvalidValue;); \
    } else {                                                                                  \
      return hipErrorInvalidValue;                                                            \
    }                                                                                         \
  } while (0)

hipError_t launch_keygen(uint32_t N, uint64_t seed, int32_t* sk, hipStream_t st) {
  hipLaunchKernelGGL(k_keygen, dim3((N + 255) / 256), dim3(256), 0, st, N, seed, sk);
  return hipGetLastError();
}

hipError_t launch_lwe_keygen(uint32_t n, uint64_t seed, uint8_t* s1, hipStream_t st) {
  hipLaunchKernelGGL(k_lwe_keygen, dim3((n + 255) / 256), dim3(256), 0, st, n, seed, s1);
  return hipGetLastError();
}

hipError_t launch_ksk_gen(const int32_t* sk, const uint8_t* s1, uint32_t N, uint32_t n, uint64_t seed, uint32_t D,
                          const Cdt& cdt, int8_t* out, hipStream_t st) {
  const uint64_t K = (uint64_t)N * D;
  hipLaunchKernelGGL(k_ksk_gen, dim3((uint32_t)K), dim3(256), 0, st, sk, s1, n, seed, D, K, cdt, out);
  return hipGetLastError();
}

hipError_t launch_sk_hat(int logN, int nq, const Tabs& T, const int32_t* sk, uint32_t* sk_hat, hipStream_t st) {
  HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_sk_hat<LN, NQ>), dim3(NQ), dim3(Geo<LN>::T), 0, st, T, sk, sk_hat));
  return hipGetLastError();
}

hipError_t launch_enc_rgsw(int logN, int nq, int dig, const Tabs& T, const Cdt& cdt, const EncArgs& A,
                           uint64_t count, int rows_per_wg, hipStream_t st) {
  const size_t rg = (size_t)2 * dig * nq * 2 * nq * ((size_t)1 << logN);
  const uint32_t rows = 2 * dig * nq;
  if (rows_per_wg < 1 || rows % rows_per_wg) return hipErrorInvalidValue;
  return for_rect(count, [&](uint64_t off, dim3 g) -> hipError_t {
    EncArgs B = A;
    B.bits = A.bits + off;
    B.out = A.out + off * rg;
    B.ct0 = A.ct0 + off;
    const dim3 grid(rows / rows_per_wg, g.x, g.y);
    switch (rows_per_wg) {
      case 1:
        HW_DISPATCH_G(logN, nq, dig, hipLaunchKernelGGL((k_enc_rgsw<LN, NQ, 1, DG>), grid, dim3(Geo<LN>::T), 0, st,
                                                         T, cdt, B));
        break;
      case 2:
        HW_DISPATCH_G(logN, nq, dig, hipLaunchKernelGGL((k_enc_rgsw<LN, NQ, 2, DG>), grid, dim3(Geo<LN>::T), 0, st,
                                                         T, cdt, B));
        break;
      case 5:
        if (dig != 5) return hipErrorInvalidValue;
        HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_enc_rgsw<LN, NQ, 5>), grid, dim3(Geo<LN>::T), 0, st, T, cdt, B));
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_enc_rlwe(int logN, int nq, const Tabs& T, const Cdt& cdt, const EncArgs& A, uint64_t count,
                           hipStream_t st) {
  const size_t N = 1u << logN;
  return for_rect(count, [&](uint64_t off, dim3 g) -> hipError_t {
    EncArgs B = A;
    B.ct0 = A.ct0 + off;
    B.out = A.out + off * 2 * nq * N;
    B.msg = A.msg ? A.msg + off * N : nullptr;
    HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_enc_rlwe<LN, NQ>), g, dim3(Geo<LN>::T), 0, st, T, cdt, B));
    return hipGetLastError();
  });
}

hipError_t launch_dec_rlwe(int logN, int nq, const Tabs& T, const CrtTab& K, const uint32_t* sk_hat,
                           const uint32_t* ct, uint64_t count, uint64_t* msg, hipStream_t st) {
  const size_t N = 1u << logN;
  return for_rect(count, [&](uint64_t off, dim3 g) -> hipError_t {
    HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_dec_rlwe<LN, NQ>), g, dim3(Geo<LN>::T), 0, st, T, K, sk_hat,
                                              ct + off * 2 * nq * N, msg + off * N));
    return hipGetLastError();
  });
}

hipError_t launch_dec_lwe(int logN, int nq, const Tabs& T, const CrtTab& K, const int32_t* sk,
                          const uint32_t* lwe, uint64_t count, uint64_t* msg, hipStream_t st) {
  const uint32_t N = 1u << logN;
  const uint64_t per_launch = 4ull * 65535 * 256;
  for (uint64_t off = 0; off < count; off += per_launch) {
    const uint64_t c = count - off < per_launch ? count - off : per_launch;
    const uint32_t blocks = (uint32_t)((c + 3) / 4);
    const uint32_t* l = lwe + off * (size_t)nq * (N + 1);
    if (nq == 1) hipLaunchKernelGGL(k_dec_lwe<1>, dim3(blocks), dim3(256), 0, st, T, K, N, sk, l, c, msg + off);
    else if (nq == 2) hipLaunchKernelGGL(k_dec_lwe<2>, dim3(blocks), dim3(256), 0, st, T, K, N, sk, l, c, msg + off);
    else if (nq == 3) hipLaunchKernelGGL(k_dec_lwe<3>, dim3(blocks), dim3(256), 0, st, T, K, N, sk, l, c, msg + off);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rgsw_export(int logN, int nq, int dig, const Tabs& T, const uint32_t* rgsw, uint64_t count,
                              uint32_t* out, hipStream_t st) {
  const size_t N = 1u << logN;
  const uint64_t polys = count * 2 * dig * nq * 2;
  return for_rect(polys, [&](uint64_t off, dim3 g) -> hipError_t {
    HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_rgsw_export<LN, NQ>), g, dim3(Geo<LN>::T), 0, st, T,
                                              rgsw + off * nq * N, out + off * nq * N));
    return hipGetLastError();
  });
}

hipError_t launch_ntt(int logN, int nq, const Tabs& T, uint32_t* polys, uint64_t count, int inverse,
                      uint32_t per, hipStream_t st) {
  const size_t N = 1u << logN;
  if (per < 1) return hipErrorInvalidValue;
  const uint64_t groups = (count + per - 1) / per;
  return for_rect(groups, [&](uint64_t off, dim3 g) -> hipError_t {
    HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_ntt<LN, NQ>), dim3(NQ, g.x, g.y), dim3(Geo<LN>::T), 0, st, T,
                                              polys + off * per * nq * N, count - off * per, per, inverse));
    return hipGetLastError();
  });
}

hipError_t launch_xp(int logN, int nq, int dig, const Tabs& T, const uint32_t* rgsw, const uint32_t* in,
                     uint64_t count, uint32_t* out, hipStream_t st) {
  const size_t N = 1u << logN;
  const uint64_t rw = 2ull * nq * N, gw = 2ull * dig * nq * rw;
  return for_rect(count, [&](uint64_t off, dim3 g) -> hipError_t {
    HW_DISPATCH_G(logN, nq, dig, hipLaunchKernelGGL((k_xp<LN, NQ, DG>), g, dim3(Geo<LN>::T), 0, st, T, rgsw + off * gw,
                                                     in + off * rw, out + off * rw, gw));
    return hipGetLastError();
  });
}

hipError_t launch_perm(uint32_t s, uint64_t seed, uint32_t* pi, hipStream_t st) {
  if (s == 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm, dim3(1), dim3(64), 0, st, s, seed, pi);
  return hipGetLastError();
}

hipError_t launch_train(int logN, int nq, int dig, const Tabs& T, const TrainArgs& A, int occ, hipStream_t st) {
  const uint64_t G = (uint64_t)A.nram * A.nsub;
  if (G == 0) return hipSuccess;
  if (G > (1u << 22)) return hipErrorInvalidValue;
  const dim3 grid = A.map == 0 ? dim3(A.nram, A.nsub) : dim3((uint32_t)((G + 7) / 8 * 8));
  HW_DISPATCH_GOCC(logN, nq, occ, dig,
                   hipLaunchKernelGGL((k_train<LN, NQ, OC, DG>), grid, dim3(Geo<LN>::T), 0, st, T, A));
  return hipGetLastError();
}

hipError_t launch_train_level(int logN, int nq, int dig, const Tabs& T, const TrainArgs& A, int occ,
                              hipStream_t st) {
  const uint64_t G = (uint64_t)A.nram * A.nsub * A.smax;
  if (G == 0) return hipSuccess;
  if (G > (1ull << 30)) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)((G + 7) / 8 * 8));
  HW_DISPATCH_GOCC(logN, nq, occ, dig,
                   hipLaunchKernelGGL((k_train_level<LN, NQ, OC, DG>), grid, dim3(Geo<LN>::T), 0, st, T, A));
  return hipGetLastError();
}

template <int LN, int NQ, int OC, int DG>
static hipError_t batch_grid_t(uint32_t* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_train_batch<LN, NQ, OC, DG>,
                                                     Geo<LN>::T, 0);
  if (e != hipSuccess) return e;
  *grid = (uint32_t)(cus * (per_cu > 0 ? per_cu : 1));
  return hipSuccess;
}

hipError_t batch_grid(int logN, int nq, int dig, int occ, uint32_t* grid) {
  HW_DISPATCH_GOCC(logN, nq, occ, dig, return batch_grid_t<LN, NQ, OC, DG>(grid));
  return hipSuccess;
}

hipError_t launch_train_batch(int logN, int nq, int dig, const Tabs& T, const BatchArgs& A, uint32_t grid, int occ,
                              hipStream_t st) {
  if (grid > A.nitems) grid = A.nitems;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, A.counter, 1u);
  HW_DISPATCH_GOCC(logN, nq, occ, dig,
                   hipLaunchKernelGGL((k_train_batch<LN, NQ, OC, DG>), dim3(grid), dim3(Geo<LN>::T), 0, st, T, A));
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const Tabs& T, const BJob* jobs, uint32_t njobs, uint64_t total, uint32_t logN,
                               uint32_t N, uint32_t nq, const uint32_t* acc, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_batch, dim3(blocks), dim3(256), 0, st, T, jobs, njobs, total, logN, N, nq, acc);
  return hipGetLastError();
}

hipError_t launch_reduce_model(const Tabs& T, const ReduceArgs& A, hipStream_t st) {
  const size_t RW = (size_t)2 * A.nq * A.N;
  const size_t total = (size_t)A.k0 * A.k1 * RW + (A.cnt ? RW : 0);
  const uint32_t blocks = (uint32_t)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_reduce_model, dim3(blocks), dim3(256), 0, st, T, A);
  return hipGetLastError();
}

hipError_t launch_row_pack(const Tabs& T, const RowPackArgs& A, hipStream_t st) {
  const size_t RW = (size_t)2 * A.nq * A.N;
  const size_t total = (size_t)A.rows * RW + (A.cnt && !A.store ? RW : 0);
  if (total == 0) return hipSuccess;
  if (A.rpr == 0 || ((size_t)(A.rpr - 1) << A.nbf) >= A.N) return hipErrorInvalidValue;
  const uint32_t blocks = (uint32_t)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_row_pack, dim3(blocks), dim3(256), 0, st, T, A);
  return hipGetLastError();
}

hipError_t launch_infer(int logN, int nq, int dig, const Tabs& T, const InferArgs& A, int occ, hipStream_t st) {
  if (A.rpr == 0) return hipErrorInvalidValue;
  const uint64_t G = (uint64_t)A.k0 * A.nlab * A.nsub;
  if (G == 0) return hipSuccess;
  if (G > (1u << 22)) return hipErrorInvalidValue;
  const dim3 grid = A.map == 0 ? dim3(A.k0, A.nlab, A.nsub) : dim3((uint32_t)((G + 7) / 8 * 8));
  HW_DISPATCH_GOCC(logN, nq, occ, dig,
                   hipLaunchKernelGGL((k_infer<LN, NQ, OC, DG>), grid, dim3(Geo<LN>::T), 0, st, T, A));
  return hipGetLastError();
}

template <int LN, int NQ, int OC, int DG>
static hipError_t infer_batch_grid_t(uint32_t* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_infer_batch<LN, NQ, OC, DG>,
                                                     Geo<LN>::T, 0);
  if (e != hipSuccess) return e;
  *grid = (uint32_t)(cus * (per_cu > 0 ? per_cu : 1));
  return hipSuccess;
}

hipError_t infer_batch_grid(int logN, int nq, int dig, int occ, uint32_t* grid) {
  HW_DISPATCH_GOCC(logN, nq, occ, dig, return infer_batch_grid_t<LN, NQ, OC, DG>(grid));
  return hipSuccess;
}

hipError_t launch_infer_batch(int logN, int nq, int dig, const Tabs& T, const IBatchArgs& B, uint32_t grid, int occ,
                              hipStream_t st) {
  if (grid > B.nitems) grid = B.nitems;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, B.counter, 1u);
  HW_DISPATCH_GOCC(logN, nq, occ, dig,
                   hipLaunchKernelGGL((k_infer_batch<LN, NQ, OC, DG>), dim3(grid), dim3(Geo<LN>::T), 0, st, T, B));
  return hipGetLastError();
}

hipError_t launch_enc_pks(int logN, int nq, const Tabs& T, const Cdt& cdt, const EncArgs& A, hipStream_t st) {
  const uint32_t N = 1u << logN;
  HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_enc_pks<LN, NQ>), dim3(5 * NQ, N), dim3(Geo<LN>::T), 0, st, T, cdt, A));
  return hipGetLastError();
}

uint32_t pks_blocks(int logN) { return ((1u << logN) + PKS_J - 1) / PKS_J; }

hipError_t launch_pks(int logN, int nq, const Tabs& T, const PksArgs& A, uint32_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  const uint32_t nblk = pks_blocks(logN);
  HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_pks_partial<LN, NQ>), dim3(count, NQ, nblk), dim3(Geo<LN>::T), 0, st,
                                            T, A));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  HW_DISPATCH(logN, nq, hipLaunchKernelGGL((k_pks_finish<LN, NQ>), dim3(NQ, count), dim3(Geo<LN>::T), 0, st, T, A,
                                            nblk));
  return hipGetLastError();
}

hipError_t launch_rlwe_add(const Tabs& T, uint32_t* dst, const uint32_t* src, uint64_t words, uint32_t N, uint32_t nq,
                           hipStream_t st) {
  const uint64_t n4 = words / 4;
  const uint32_t blocks = (uint32_t)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(k_rlwe_add, dim3(blocks), dim3(256), 0, st, T, dst, src, words, N, nq);
  return hipGetLastError();
}

hipError_t launch_class_sums(const Tabs& T, const SumArgs& A, hipStream_t st) {
  const size_t total = (size_t)A.n * A.l * A.nq * (A.N + 1);
  const uint32_t blocks = (uint32_t)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_class_sums, dim3(blocks), dim3(256), 0, st, T, A);
  return hipGetLastError();
}

}  // namespace hw
