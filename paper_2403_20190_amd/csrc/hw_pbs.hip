// hw_pbs.hip -- programmable bootstrapping of LWE ciphertexts (Sec. 2.5.3),
// the Activate and EncryptedArgMax functions of OTF-act (Sec. 3.5.2, Alg. 7)
// built from bootstraps that each decide one sign, and FM-act (Sec. 3.5.3).
//
// Bootstrap (constant test polynomial V) over the ring key s (ternary, mask
// length n <= N): switch the ciphertext's mask and body from Q to 2N
// (round(2N x / Q)), start from the trivial RLWE (0, X^{-b~} TV) with
// TV = V (1 + X + ... + X^{N-1}), multiply it by X^{a~_k s_k} for k < n with
// two CMUXes against bsk[2k] = RGSW([s_k = 1]) and bsk[2k+1] = RGSW([s_k = -1]),
// and extract coefficient 0: V when the switched phase lies in [0, N), -V
// otherwise.  Through a key switch: the ciphertext goes to modulus 2^32, is
// key-switched to a binary key s1 of n coefficients (digits, a contraction on
// the matrix cores, a combine), then to 2N, and the blind rotation runs one
// CMUX per coefficient of s1 against bsk[i] = RGSW(s1_i).  The circuits
// (bits, activate, argmax) combine bootstraps with exact linear operations on
// LWE ciphertexts; their steps and constants are stated at hw_activate and
// hw_encrypted_argmax in include/hwisard.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/hwisard.h"
#include "hw_ctx.h"
#include "hw_device.h"

namespace hw {
namespace {

typedef unsigned __int128 u128;

__device__ __forceinline__ double u128_dbl(u128 x) {
  return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}

// round(two_n x / Q) mod two_n (two_n a power of two) of the integer x in
// [0, Q) with residues r, rounding half up: floor((two_n x + floor(Q/2)) / Q)
template <int NQ>
__device__ __forceinline__ uint32_t switch_2n(const uint32_t (&r)[NQ], const Tabs& T, const CrtTab& K,
                                              uint32_t two_n) {
  const u128 Q = ((u128)K.Q_hi << 64) | K.Q_lo;
  u128 x = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const uint32_t y = mulq(r[i], K.inv[i], T.pt[i]);
    const u128 M = ((u128)K.M_hi[i] << 64) | K.M_lo[i];
    x += (u128)y * M;
    if (x >= Q) x -= Q;
  }
  const u128 num = (u128)two_n * x + (((u128)K.half_hi << 64) | K.half_lo);
  uint64_t qt = (uint64_t)(u128_dbl(num) / u128_dbl(Q));
  while (qt > 0 && (u128)qt * Q > num) --qt;
  while ((u128)(qt + 1) * Q <= num) ++qt;
  return (uint32_t)(qt & (two_n - 1));
}

// modulus switch of `count` LWE ciphertexts: out[c][k] for the first n mask
// coefficients, out[c][n] for the body; one thread per value
template <int NQ>
__global__ __launch_bounds__(256) void k_pbs_switch(Tabs T, CrtTab K, uint32_t N, uint32_t n,
                                                    const uint32_t* __restrict__ lwe, uint64_t count,
                                                    uint32_t* __restrict__ out) {
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= count * (n + 1)) return;
  const uint64_t c = g / (n + 1);
  const uint32_t k = (uint32_t)(g - c * (n + 1));
  const uint32_t idx = k < n ? k : N;
  uint32_t r[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) r[i] = lwe[(c * NQ + i) * (N + 1) + idx];
  out[g] = switch_2n<NQ>(r, T, K, 2 * N);
}

struct RotArgs {
  const uint32_t* bsk;   // [2n] RGSW (ring key) or [n] RGSW (binary key), device layout
  const uint32_t* ms;    // [count][n + 1] switched mask and body
  uint32_t* slots;       // [count][2] RLWE: the accumulator and the CMUX input
  uint32_t* out;         // [count] LWE
  uint64_t rgsw_words;
  uint64_t count;
  uint32_t n;
  uint32_t binary;       // 1: one CMUX per coefficient against bsk[k] (binary key)
  uint32_t v[MAXQ];      // V mod q_i
};

// xin <- X^ex acc - acc, each thread its coefficients t + T e of every polynomial
template <int LOGN, int NQ>
__device__ __forceinline__ void pbs_rot_diff(const Tabs& T, const uint32_t* __restrict__ acc, int32_t ex,
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

// blind rotation and extraction: one workgroup per ciphertext; DIG, LB: the
// bootstrapping key's gadget (the ring key's is the context's, the
// key-switched key's 2 digits of 15 bits on rings of two or more primes)
template <int LOGN, int NQ, int DIG, int LB>
__global__ __launch_bounds__(Geo<LOGN>::T) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_pbs_rotate(
    Tabs T, RotArgs A) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[xp_words<LOGN, xp_pair<LOGN, NQ>()>()];
  __shared__ __attribute__((aligned(16))) uint2 twl[1 << LOGN];
  constexpr int N = 1 << LOGN, TT = N / 8;
  constexpr size_t RW = (size_t)2 * NQ * N;
  const uint32_t t = threadIdx.x;
  const uint64_t c = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
  if (c >= A.count) return;
  const uint32_t* ms = A.ms + c * (A.n + 1);
  uint32_t* acc = A.slots + c * 2 * RW;
  uint32_t* xin = acc + RW;
  const uint32_t bt = ms[A.n];
  // (0, X^{-b~} TV): coefficient k of X^{-b~} TV is V when (k + b~) mod 2N < N, else -V
#pragma unroll 1
  for (int w = 0; w < 2 * NQ; ++w) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t k = t + TT * e;
      uint32_t val = 0;
      if (w >= NQ) {
        const uint32_t v = A.v[w - NQ], q = T.pt[w - NQ].q;
        val = ((k + bt) & (2 * N - 1)) < (uint32_t)N ? v : (v ? q - v : 0u);
      }
      acc[(size_t)w * N + k] = val;
    }
  }
  __syncthreads();
  uint32_t xc = 0;
#pragma unroll 1
  for (uint32_t k = 0; k < A.n; ++k) {
    const int32_t a = (int32_t)ms[k];
#pragma unroll 1
    for (int sg = 0; sg < (A.binary ? 1 : 2); ++sg) {
      pbs_rot_diff<LOGN, NQ>(T, acc, sg ? -a : a, xin, t);
      const size_t row = A.binary ? (size_t)k : (size_t)(2 * k + sg);
      ext_prod<LOGN, NQ, xp_pair<LOGN, NQ>(), DIG, LB>(xin, A.bsk + row * A.rgsw_words, T, lds, twl, xc, t,
                                                       XpOut{acc, acc, nullptr, XP_ADD});
      __syncthreads();  // the next rotation reads coefficients other threads wrote
    }
  }
  // ExtractLWE(ACC, 0): a'_0 = a_0, a'_j = -a_{N-j}, b' = b_0
  uint32_t* o = A.out + c * (size_t)NQ * (N + 1);
#pragma unroll 1
  for (int i = 0; i < NQ; ++i) {
    const uint32_t q = T.pt[i].q;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t j = t + TT * e;
      const uint32_t av = acc[(size_t)i * N + (j ? N - j : 0)];
      o[(size_t)i * (N + 1) + j] = j ? (av ? q - av : 0u) : av;
    }
    if (t == 0) o[(size_t)i * (N + 1) + N] = acc[(size_t)(NQ + i) * N];
  }
}

// ---- key switch to the binary LWE key (modulus 2^32) ----------------------

constexpr uint32_t KS_DIGITS = 6;  // balanced base-16 digits of the top 24 bits
// gadget of the key-switched bootstrapping key's RGSW on rings of two or more
// primes: 2 balanced digits of 15 bits per prime (exact for primes below 2^30;
// the digit size of the paper's HE1 TFHE parameter set, Sec. 4)
constexpr int BSK_DIG = 2, BSK_LB = 15;

// round(2^32 x / Q) mod 2^32 (half up) of x in [0, Q) with residues r
template <int NQ>
__device__ __forceinline__ uint32_t switch_2_32(const uint32_t (&r)[NQ], const Tabs& T, const CrtTab& K) {
  const u128 Q = ((u128)K.Q_hi << 64) | K.Q_lo;
  u128 x = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const uint32_t y = mulq(r[i], K.inv[i], T.pt[i]);
    const u128 M = ((u128)K.M_hi[i] << 64) | K.M_lo[i];
    x += (u128)y * M;
    if (x >= Q) x -= Q;
  }
  const u128 num = (x << 32) + (((u128)K.half_hi << 64) | K.half_lo);
  uint64_t qt = (uint64_t)(u128_dbl(num) / u128_dbl(Q));
  while (qt > 0 && (u128)qt * Q > num) --qt;
  while ((u128)(qt + 1) * Q <= num) ++qt;
  return (uint32_t)qt;
}

// Digits of the key switch: for ciphertext c and mask coefficient k < N, the
// switched a'_k, rounded to its top 24 bits (t = round(a' / 2^8) mod 2^24),
// as KS_DIGITS balanced base-16 digits d_j (weight 2^(28 - 4j)) into
// dig[c][k KS_DIGITS + j]; for k = N the switched body into body[c].  One
// thread per (c, k <= N).
template <int NQ>
__global__ __launch_bounds__(256) void k_ks_digits(Tabs T, CrtTab K, uint32_t N, const uint32_t* __restrict__ lwe,
                                                   uint64_t count, int8_t* __restrict__ dig,
                                                   uint32_t* __restrict__ body) {
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= count * (N + 1)) return;
  const uint64_t c = g / (N + 1);
  const uint32_t k = (uint32_t)(g - c * (N + 1));
  uint32_t r[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) r[i] = lwe[(c * NQ + i) * (N + 1) + k];
  const uint32_t a = switch_2_32<NQ>(r, T, K);
  if (k == N) {
    body[c] = a;
    return;
  }
  uint32_t t = (uint32_t)((((uint64_t)a + 128u) >> 8) & 0xFFFFFFu);
  int32_t carry = 0;
  int8_t d[KS_DIGITS];
#pragma unroll
  for (int j = KS_DIGITS - 1; j >= 0; --j) {
    int32_t x = (int32_t)(t & 15u) + carry;
    t >>= 4;
    carry = x >= 8;
    d[j] = (int8_t)(carry ? x - 16 : x);
  }
  int8_t* o = dig + c * ((uint64_t)N * KS_DIGITS) + (uint64_t)k * KS_DIGITS;
#pragma unroll
  for (int j = 0; j < (int)KS_DIGITS; ++j) o[j] = d[j];
}

typedef int v4i __attribute__((ext_vector_type(4)));

// The key switch's contraction C[c][col] = sum_r dig[c][r] ksk[col][r] over
// r < Kd = N KS_DIGITS: signed bytes in, exact 32-bit sums out (|sum| <= 8 x
// 128 x Kd < 2^31 for N <= 4096).  MFMA 16x16x32 (i8 -> i32): each wave
// computes a 16 x 16 tile of C; lane l feeds A[l mod 16][8 (l / 16) + 0..7]
// (8 consecutive bytes of a row of dig) and B[8 (l / 16) + 0..7][l mod 16]
// (8 consecutive bytes of a row of ksk, which holds the key column-major) and
// receives C[4 (l / 16) + 0..3][l mod 16].  Four waves per workgroup cover
// 64 columns; rows of dig and ksk are Kd bytes (a multiple of 32), dig has
// (a multiple of) 16 rows per block row, ksk (a multiple of) 64 rows.
__global__ __launch_bounds__(256) void k_ks_gemm(const int8_t* __restrict__ dig, const int8_t* __restrict__ ksk,
                                                 uint64_t Kd, uint32_t cols, int32_t* __restrict__ C) {
  const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t row0 = (uint64_t)blockIdx.y * 16, col0 = (uint64_t)blockIdx.x * 64 + w * 16;
  const int8_t* pa = dig + (row0 + (l & 15)) * Kd + 8 * (l >> 4);
  const int8_t* pb = ksk + (col0 + (l & 15)) * Kd + 8 * (l >> 4);
  v4i acc = {0, 0, 0, 0};
#pragma unroll 4
  for (uint64_t k = 0; k < Kd; k += 32) {
    const long a = *reinterpret_cast<const long*>(pa + k);
    const long b = *reinterpret_cast<const long*>(pb + k);
    acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) C[(row0 + 4 * (l >> 4) + i) * cols + col0 + (l & 15)] = acc[i];
}

// The switched ciphertext from the contraction and its modulus switch to 2N:
// v_i = sum_l C[c][l (n + 1) + i] 2^(8l) mod 2^32 is sum_r d_r KSK_r[i]; the key
// switch gives a_i = -v_i (i < n), b = body - v_n (mod 2^32), and
// ms[c][i] = round(2N x / 2^32) mod 2N of each.  One thread per (c, i <= n).
__global__ __launch_bounds__(256) void k_ks_combine(const int32_t* __restrict__ C, uint32_t cols, uint32_t n,
                                                    const uint32_t* __restrict__ body, uint64_t count,
                                                    uint32_t log2n2, uint32_t* __restrict__ ms) {
  const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= count * (n + 1)) return;
  const uint64_t c = g / (n + 1);
  const uint32_t i = (uint32_t)(g - c * (n + 1));
  uint32_t v = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) v += (uint32_t)C[c * cols + (uint64_t)l * (n + 1) + i] << (8 * l);
  const uint32_t x = (i < n ? 0u : body[c]) - v;
  const uint32_t sh = 32 - log2n2;
  ms[g] = (uint32_t)((((uint64_t)x + (1ull << (sh - 1))) >> sh) & ((1ull << log2n2) - 1));
}

struct LinArgs {
  const uint32_t* x;   // [count] LWE at stride sx words
  const uint32_t* y;   // may be null
  uint32_t* out;       // may alias x or y (each word is read before it is written)
  uint64_t sx, sy, so;
  uint64_t count;
  uint32_t N, nq;
  uint32_t ax[MAXQ], by[MAXQ], g[MAXQ];  // residues of alpha, beta and the body constant
};

// out = alpha x + beta y + (0, g), mod each q_i
__global__ __launch_bounds__(256) void k_lwe_lin(Tabs T, LinArgs A) {
  const uint64_t lw = (uint64_t)A.nq * (A.N + 1);
  const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= A.count * lw) return;
  const uint64_t c = w / lw;
  const uint32_t r = (uint32_t)(w - c * lw);
  const uint32_t i = r / (A.N + 1), k = r - i * (A.N + 1);
  const PrimeTab P = T.pt[i];
  uint32_t v = mulq(A.ax[i], A.x[c * A.sx + r], P);
  if (A.y) v = addq(v, mulq(A.by[i], A.y[c * A.sy + r], P), P.q);
  if (k == A.N) v = addq(v, A.g[i], P.q);
  A.out[c * A.so + r] = v;
}

// ExtractLWE at coefficients 0..K-1 of each of `rows` RLWE (coefficient
// domain): cell (r, k) gets a'_j = a_{k-j} for j <= k, -a_{N+k-j} for j > k,
// b' = b_k, as [prime][N + 1]; one thread per output word
struct CellArgs {
  const uint32_t* rows;  // [rows][2][nq][N]
  uint32_t* out;         // [rows][K] LWE
  uint64_t nrows;
  uint32_t K, N, nq;
};

__global__ __launch_bounds__(256) void k_extract_cells(Tabs T, CellArgs A) {
  const uint64_t lw = (uint64_t)A.nq * (A.N + 1);
  const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= A.nrows * A.K * lw) return;
  const uint64_t cell = w / lw;
  const uint32_t rem = (uint32_t)(w - cell * lw);
  const uint32_t i = rem / (A.N + 1), j = rem - i * (A.N + 1);
  const uint64_t r = cell / A.K;
  const uint32_t k = (uint32_t)(cell - r * A.K);
  const uint32_t* row = A.rows + r * 2 * A.nq * A.N;
  uint32_t v;
  if (j == A.N) {
    v = row[(size_t)(A.nq + i) * A.N + k];
  } else if (j <= k) {
    v = row[(size_t)i * A.N + (k - j)];
  } else {
    const uint32_t x = row[(size_t)i * A.N + (A.N + k - j)];
    v = x ? T.pt[i].q - x : 0u;
  }
  A.out[w] = v;
}

// the bootstrapping-key bits of the first n key coefficients: [s_k = 1], [s_k = -1]
__global__ void k_pbs_bits(const int32_t* __restrict__ sk, uint32_t n, uint8_t* __restrict__ bits) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  bits[2 * k] = sk[k] == 1;
  bits[2 * k + 1] = sk[k] == -1;
}

}  // namespace
}  // namespace hw

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

using hw::u128;

// kernel templates for the supported (log2 N, primes)
#define PBS_DISPATCH(logN, nq, ...)                                                  \
  do {                                                                               \
    if (logN == 10 && nq == 1) { constexpr int LN = 10, NQ = 1; __VA_ARGS__; }       \
    else if (logN == 10 && nq == 2) { constexpr int LN = 10, NQ = 2; __VA_ARGS__; }  \
    else if (logN == 10 && nq == 3) { constexpr int LN = 10, NQ = 3; __VA_ARGS__; }  \
    else if (logN == 11 && nq == 1) { constexpr int LN = 11, NQ = 1; __VA_ARGS__; }  \
    else if (logN == 11 && nq == 2) { constexpr int LN = 11, NQ = 2; __VA_ARGS__; }  \
    else if (logN == 11 && nq == 3) { constexpr int LN = 11, NQ = 3; __VA_ARGS__; }  \
    else if (logN == 12 && nq == 1) { constexpr int LN = 12, NQ = 1; __VA_ARGS__; }  \
    else if (logN == 12 && nq == 2) { constexpr int LN = 12, NQ = 2; __VA_ARGS__; }  \
    else if (logN == 12 && nq == 3) { constexpr int LN = 12, NQ = 3; __VA_ARGS__; }  \
    else return hipErrorInvalidValue;                                                \
  } while (0)

struct Pbs {
  hw_ctx* c;
  const uint32_t* bsk;
  const int8_t* ksk;  // key switch to the binary LWE key; nullptr: the ring key
  uint32_t n;
  hipStream_t st;
  uint32_t* ms;     // [cmax][n + 1]
  uint32_t* slots;  // [cmax][2] RLWE
  int8_t* dig;      // key switch: [cmax rounded up to 16][N KS_DIGITS] digits
  int32_t* C;       // key switch: [same rows][cols] contraction
  uint32_t* body;   // key switch: [same rows] switched bodies
  uint32_t cols;    // key switch: 4 (n + 1) rounded up to 64
  size_t lw;        // words of an LWE ciphertext
};

// digits per prime of a bootstrapping key's RGSW: the key-switched key's use
// the coarser gadget on rings of two or more primes (a one-prime ring's 30-bit
// modulus leaves no room for its noise, so there they use the context's); the
// ring key's use the context's gadget, as hw_encrypt_rgsw_bits makes them
uint32_t bsk_digits(const hw_ctx* c, bool ks) { return ks && c->prm.nq >= 2 ? hw::BSK_DIG : c->prm.digits; }

// words of one RGSW of a bootstrapping key
size_t bsk_rgsw_words(const hw_ctx* c, bool ks) { return (size_t)2 * bsk_digits(c, ks) * c->prm.nq * rlwe_words(c); }

// columns of the key switch's contraction for an LWE key of n coefficients:
// four signed bytes of each of the n + 1 words, padded to 64
uint32_t ks_cols(uint32_t n) { return ((4 * (n + 1) + 63) / 64) * 64; }

uint32_t res_of(u128 x, uint32_t q) { return (uint32_t)(x % q); }

// residue of a signed integer (|v| < 2^63) mod q
uint32_t res_signed(int64_t v, uint32_t q) {
  const int64_t r = v % (int64_t)q;
  return (uint32_t)(r < 0 ? r + (int64_t)q : r);
}

// out = alpha x + beta y + (0, g) over `count` ciphertexts at the given strides (in LWE units)
hipError_t lin(const Pbs& B, uint64_t count, uint32_t* out, uint64_t so, int64_t alpha, const uint32_t* x,
               uint64_t sx, int64_t beta = 0, const uint32_t* y = nullptr, uint64_t sy = 0, u128 g = 0,
               bool g_neg = false) {
  hw_ctx* c = B.c;
  hw::LinArgs A{};
  A.x = x;
  A.y = y;
  A.out = out;
  A.sx = sx * B.lw;
  A.sy = sy * B.lw;
  A.so = so * B.lw;
  A.count = count;
  A.N = c->prm.N;
  A.nq = c->prm.nq;
  for (uint32_t i = 0; i < c->prm.nq; ++i) {
    const uint32_t q = c->tabs.pt[i].q;
    A.ax[i] = res_signed(alpha, q);
    A.by[i] = res_signed(beta, q);
    const uint32_t gr = res_of(g, q);
    A.g[i] = g_neg ? (gr ? q - gr : 0u) : gr;
  }
  const uint64_t words = count * B.lw;
  if (!words) return hipSuccess;
  hipLaunchKernelGGL(hw::k_lwe_lin, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, B.st, c->tabs, A);
  return hipGetLastError();
}

// out[j] = PBS(in[j], V) for j < count (count <= the workspace's cmax); contiguous arrays
hipError_t pbs(const Pbs& B, uint64_t count, const uint32_t* in, uint32_t* out, u128 V) {
  hw_ctx* c = B.c;
  if (!count) return hipSuccess;
  const uint32_t N = c->prm.N, nq = c->prm.nq;
  if (B.ksk) {  // key switch to the binary key at 2^32, then to 2N
    const uint64_t vals = count * (N + 1);
    const dim3 gd((uint32_t)((vals + 255) / 256));
    if (nq == 1) hipLaunchKernelGGL(hw::k_ks_digits<1>, gd, dim3(256), 0, B.st, c->tabs, c->crt, N, in, count, B.dig, B.body);
    else if (nq == 2) hipLaunchKernelGGL(hw::k_ks_digits<2>, gd, dim3(256), 0, B.st, c->tabs, c->crt, N, in, count, B.dig, B.body);
    else hipLaunchKernelGGL(hw::k_ks_digits<3>, gd, dim3(256), 0, B.st, c->tabs, c->crt, N, in, count, B.dig, B.body);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t Kd = (uint64_t)N * hw::KS_DIGITS;
    hipLaunchKernelGGL(hw::k_ks_gemm, dim3(B.cols / 64, (uint32_t)((count + 15) / 16)), dim3(256), 0, B.st, B.dig,
                       B.ksk, Kd, B.cols, B.C);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t outs = count * (B.n + 1);
    hipLaunchKernelGGL(hw::k_ks_combine, dim3((uint32_t)((outs + 255) / 256)), dim3(256), 0, B.st, B.C, B.cols, B.n,
                       B.body, count, (uint32_t)c->logN + 1, B.ms);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    const uint64_t vals = count * (B.n + 1);
    const dim3 gs((uint32_t)((vals + 255) / 256));
    if (nq == 1) hipLaunchKernelGGL(hw::k_pbs_switch<1>, gs, dim3(256), 0, B.st, c->tabs, c->crt, N, B.n, in, count, B.ms);
    else if (nq == 2) hipLaunchKernelGGL(hw::k_pbs_switch<2>, gs, dim3(256), 0, B.st, c->tabs, c->crt, N, B.n, in, count, B.ms);
    else hipLaunchKernelGGL(hw::k_pbs_switch<3>, gs, dim3(256), 0, B.st, c->tabs, c->crt, N, B.n, in, count, B.ms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hw::RotArgs A{};
  A.bsk = B.bsk;
  A.ms = B.ms;
  A.slots = B.slots;
  A.out = out;
  A.rgsw_words = bsk_rgsw_words(c, B.ksk != nullptr);
  A.count = count;
  A.n = B.n;
  A.binary = B.ksk != nullptr;
  for (uint32_t i = 0; i < nq; ++i) A.v[i] = res_of(V, c->tabs.pt[i].q);
  const dim3 g((uint32_t)std::min<uint64_t>(count, 65535), (uint32_t)((count + 65534) / 65535));
  if (bsk_digits(c, B.ksk != nullptr) == hw::BSK_DIG)
    PBS_DISPATCH(c->logN, nq, if constexpr (NQ >= 2) {
      hipLaunchKernelGGL((hw::k_pbs_rotate<LN, NQ, hw::BSK_DIG, hw::BSK_LB>), g, dim3(hw::Geo<LN>::T), 0, B.st,
                         c->tabs, A);
    } else return hipErrorInvalidValue;);
  else
    PBS_DISPATCH(c->logN, nq,
                 hipLaunchKernelGGL((hw::k_pbs_rotate<LN, NQ, 5, 6>), g, dim3(hw::Geo<LN>::T), 0, B.st, c->tabs, A));
  return hipGetLastError();
}

// the bits of the messages of x (phase ~ floor(Q/p) m, m < p = 2^P), least
// significant first: E[k] (count LWE each, contiguous) with phase ~ 2 V_b bit_k.
// x is consumed (it ends as the encryption of 0); y and o are scratch.
hipError_t bits(const Pbs& B, uint64_t count, uint32_t P, uint32_t* x, uint32_t* const* E, uint32_t* y,
                uint32_t* o) {
  const u128 Q = B.c->Q;
  const u128 vb = (Q >> P) / 2;
  for (uint32_t k = 0; k < P; ++k) {
    hipError_t e = lin(B, count, y, 1, (int64_t)1 << (P - 1 - k), x, 1, 0, nullptr, 0, Q / 4);
    if (e == hipSuccess) e = pbs(B, count, y, o, vb);
    if (e == hipSuccess) e = lin(B, count, E[k], 1, -1, o, 1, 0, nullptr, 0, vb);
    if (e == hipSuccess) e = lin(B, count, x, 1, 1, x, 1, -((int64_t)1 << k), E[k], 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hw_status pbs_setup(hw_ctx* c, const hw_boot_key* key, uint64_t count, size_t extra_lwe, hipStream_t st, Pbs* B,
                    uint64_t* cmax, uint32_t** lwes) {
  const uint32_t n = key->n;
  B->c = c;
  B->bsk = key->bsk;
  B->ksk = reinterpret_cast<const int8_t*>(key->ksk);
  B->n = n;
  B->st = st;
  B->lw = lwe_words(c);
  B->cols = B->ksk ? ks_cols(n) : 0;
  const size_t kd = (size_t)c->prm.N * hw::KS_DIGITS;
  // per ciphertext: the switched values, two RLWE slots, extra_lwe LWE
  // temporaries; with the key switch also its digits, contraction and body
  const size_t per = (size_t)(n + 1) * 4 + 2 * rlwe_words(c) * 4 + extra_lwe * B->lw * 4 +
                     (B->ksk ? kd + (size_t)B->cols * 4 + 4 : 0);
  uint64_t m = std::max<uint64_t>(1, c->ws_budget / per);
  m = std::min<uint64_t>(m, count);
  if (B->ksk && m > 16) m -= m % 16;
  const uint64_t m16 = (m + 15) / 16 * 16;  // rows of the contraction
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_slots = up(m * 2 * rlwe_words(c) * 4), b_ms = up(m * (n + 1) * 4);
  const size_t b_dig = B->ksk ? up(m16 * kd) : 0, b_c = B->ksk ? up(m16 * B->cols * 4) : 0;
  const size_t b_body = B->ksk ? up(m16 * 4) : 0;
  CHECK(ensure_ws(c, b_slots + b_ms + b_dig + b_c + b_body + m * extra_lwe * B->lw * 4 + 256));
  char* base = static_cast<char*>(c->d_ws);
  B->slots = reinterpret_cast<uint32_t*>(base);
  B->ms = reinterpret_cast<uint32_t*>(base + b_slots);
  B->dig = B->ksk ? reinterpret_cast<int8_t*>(base + b_slots + b_ms) : nullptr;
  B->C = B->ksk ? reinterpret_cast<int32_t*>(base + b_slots + b_ms + b_dig) : nullptr;
  B->body = B->ksk ? reinterpret_cast<uint32_t*>(base + b_slots + b_ms + b_dig + b_c) : nullptr;
  *lwes = reinterpret_cast<uint32_t*>(base + b_slots + b_ms + b_dig + b_c + b_body);
  *cmax = m;
  return HW_OK;
}

// FM-act works through the model in chunks of about this many cells (two
// LWE buffers of that size are allocated for the call)
constexpr uint64_t FM_CHUNK_CELLS = 65536;

constexpr uint32_t KS_MAX_N = 8192;  // longest binary LWE key

hw_status check_pbs(hw_ctx* c, const hw_boot_key* key) {
  if (!key || !key->bsk) return fail(HW_EINVAL, "null bootstrapping key");
  if (key->ksk) {
    if (key->n < 1 || key->n > KS_MAX_N) return fail(HW_EINVAL, "n = %u out of range [1, %u]", key->n, KS_MAX_N);
  } else if (key->n < 1 || key->n > c->prm.N) {
    return fail(HW_EINVAL, "n = %u out of range [1, N = %u]", key->n, c->prm.N);
  }
  return HW_OK;
}

}  // namespace

extern "C" hw_status hw_pbs_keygen(hw_ctx* c, const int32_t* sk, uint64_t seed, uint32_t n, uint32_t* bsk,
                                   hipStream_t st) {
  CHECK(enter(c));
  if (!sk || !bsk) return fail(HW_EINVAL, "null buffer");
  if (n < 1 || n > c->prm.N) return fail(HW_EINVAL, "n = %u out of range [1, N = %u]", n, c->prm.N);
  CHECK(ensure_ws(c, 2 * (size_t)n));
  uint8_t* bits = static_cast<uint8_t*>(c->d_ws);
  hipLaunchKernelGGL(hw::k_pbs_bits, dim3((n + 255) / 256), dim3(256), 0, st, sk, n, bits);
  HIP_TRY(hipGetLastError());
  return hw_encrypt_rgsw_bits(c, sk, bits, 2 * (uint64_t)n, seed, 0, bsk, st);
}

extern "C" hw_status hw_pbs_ks_sizes(const hw_ctx* c, uint32_t n, uint64_t* bsk_bytes, uint64_t* ksk_bytes) {
  if (!c || !bsk_bytes || !ksk_bytes) return fail(HW_EINVAL, "null argument");
  if (n < 1 || n > KS_MAX_N) return fail(HW_EINVAL, "n = %u out of range [1, %u]", n, KS_MAX_N);
  *bsk_bytes = (uint64_t)n * bsk_rgsw_words(c, true) * 4;
  *ksk_bytes = (uint64_t)ks_cols(n) * c->prm.N * hw::KS_DIGITS;
  return ok();
}

extern "C" hw_status hw_pbs_ks_keygen(hw_ctx* c, const int32_t* sk, uint64_t seed, uint32_t n, uint8_t* lwe_key,
                                      uint32_t* bsk, int8_t* ksk, hipStream_t st) {
  CHECK(enter(c));
  if (!sk || !lwe_key || !bsk || !ksk) return fail(HW_EINVAL, "null buffer");
  if (n < 1 || n > KS_MAX_N) return fail(HW_EINVAL, "n = %u out of range [1, %u]", n, KS_MAX_N);
  HIP_TRY(hw::launch_lwe_keygen(n, seed, lwe_key, st));
  // RGSW(s1_i) with the bootstrapping key's gadget, ciphertexts 0..n-1 of stream seed
  if (bsk_digits(c, true) != c->prm.digits) {
    HIP_TRY(hw::launch_sk_hat(c->logN, c->prm.nq, c->tabs, sk, c->d_skhat, st));
    hw::EncArgs A{};
    A.sk = sk;
    A.sk_hat = c->d_skhat;
    A.bits = lwe_key;
    A.out = bsk;
    A.seed = seed;
    A.ct0 = 0;
    A.log_base = hw::BSK_LB;
    HIP_TRY(hw::launch_enc_rgsw(c->logN, c->prm.nq, hw::BSK_DIG, c->tabs, c->cdt, A, n, 2, st));
  } else {
    CHECK(hw_encrypt_rgsw_bits(c, sk, lwe_key, n, seed, 0, bsk, st));
  }
  // the padding rows of the contraction's key are read but never used: zero them
  const uint64_t kd = (uint64_t)c->prm.N * hw::KS_DIGITS;
  const uint64_t used = (uint64_t)4 * (n + 1) * kd, all = (uint64_t)ks_cols(n) * kd;
  if (all > used) HIP_TRY(hipMemsetAsync(ksk + used, 0, all - used, st));
  HIP_TRY(hw::launch_ksk_gen(sk, lwe_key, c->prm.N, n, seed, hw::KS_DIGITS, c->cdt, ksk, st));
  return ok();
}

extern "C" hw_status hw_pbs(hw_ctx* c, const hw_boot_key* key, const uint32_t* lwe, uint64_t count,
                            const uint32_t* v, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  CHECK(check_pbs(c, key));
  if (count == 0) return ok();
  if (!lwe || !out || !v) return fail(HW_EINVAL, "null buffer");
  if (lwe == out) return fail(HW_EINVAL, "output must not alias input");
  u128 V = 0;
  {  // the constant from its residues (CRT), so that one value is used for every prime
    for (uint32_t i = 0; i < c->prm.nq; ++i) {
      if (v[i] >= c->tabs.pt[i].q) return fail(HW_EINVAL, "v[%u] not below q_%u", i, i);
      const uint32_t q = c->tabs.pt[i].q;
      const u128 M = c->Q / q;
      const uint64_t y = (uint64_t)((u128)v[i] * c->crt.inv[i] % q);
      V = (V + (u128)y * M) % c->Q;
    }
  }
  Pbs B;
  uint64_t cmax = 0;
  uint32_t* tmp = nullptr;
  CHECK(pbs_setup(c, key, count, 0, st, &B, &cmax, &tmp));
  for (uint64_t c0 = 0; c0 < count; c0 += cmax) {
    const uint64_t m = std::min(cmax, count - c0);
    HIP_TRY(timed(c, "pbs", (double)m, st, [&] { return pbs(B, m, lwe + c0 * B.lw, out + c0 * B.lw, V); }));
  }
  return ok();
}

// the activation of `kind` (HW_ACT_*) over `count` LWE: the argument checks of
// hw_activate, then the circuits stated there
static hw_status activate_core(hw_ctx* c, const hw_boot_key* key, const uint32_t* lwe, uint64_t count,
                               uint32_t kind, uint64_t param, uint32_t log_p_out, uint32_t* out, hipStream_t st) {
  CHECK(check_pbs(c, key));
  const uint64_t p = c->prm.plain_mod;
  uint32_t P = 0;
  while ((1ull << P) < p) ++P;
  if (P < 3) return fail(HW_EINVAL, "the activation needs p >= 8 (p = %llu)", (unsigned long long)p);
  if (kind > HW_ACT_BLOG) return fail(HW_EINVAL, "kind = %u: must be HW_ACT_GE, HW_ACT_LOG or HW_ACT_BLOG", kind);
  if (kind == HW_ACT_GE && (param < 1 || param > p))
    return fail(HW_EINVAL, "T = %llu out of range [1, p = %llu]", (unsigned long long)param, (unsigned long long)p);
  if (kind == HW_ACT_BLOG && param < 1) return fail(HW_EINVAL, "the b-log cap must be >= 1");
  if (log_p_out < 1 || log_p_out > 60) return fail(HW_EINVAL, "log_p_out = %u out of range [1, 60]", log_p_out);
  if (kind != HW_ACT_GE && log_p_out < 3) return fail(HW_EINVAL, "log and b-log need log_p_out >= 3");
  if (count == 0) return ok();
  if (!lwe || !out) return fail(HW_EINVAL, "null buffer");
  const u128 Q = c->Q, vc = Q / 16, vo = (Q >> log_p_out) / 2;
  // temporaries per ciphertext: x, y, o, the carry or OR chain, and the P bits
  Pbs B;
  uint64_t cmax = 0;
  uint32_t* tmp = nullptr;
  CHECK(pbs_setup(c, key, count, 4 + P, st, &B, &cmax, &tmp));
  // log / b-log: outputs o_1 .. o_top, constant k (1 - o_0)
  const uint32_t top = kind == HW_ACT_LOG || param >= P ? P - 1 : (uint32_t)param;
  const int64_t kc = kind == HW_ACT_LOG || param >= P ? P : (int64_t)param;
  for (uint64_t c0 = 0; c0 < count; c0 += cmax) {
    const uint64_t m = std::min(cmax, count - c0);
    uint32_t* x = tmp;
    uint32_t* y = x + cmax * B.lw;
    uint32_t* o = y + cmax * B.lw;
    uint32_t* chain = o + cmax * B.lw;
    uint32_t* res = out + c0 * B.lw;
    std::vector<uint32_t*> E(P);
    for (uint32_t k = 0; k < P; ++k) E[k] = chain + (k + 1) * cmax * B.lw;
    auto run_ge = [&]() -> hipError_t {
      const uint64_t t = p - param;
      hipError_t e = lin(B, m, x, 1, 1, lwe + c0 * B.lw, 1);
      if (e == hipSuccess) e = bits(B, m, P, x, E.data(), y, o);
      if (e == hipSuccess) e = lin(B, m, chain, 1, 0, x, 1);  // carry 0
      for (uint32_t k = 0; e == hipSuccess && k < P; ++k) {
        const u128 thr = ((t >> k) & 1) ? vc : 3 * vc;
        const u128 V = k + 1 == P ? vo : vc;
        e = lin(B, m, y, 1, (int64_t)1 << (P - 3), E[k], 1, 1, chain, 1, thr, true);
        if (e == hipSuccess) e = pbs(B, m, y, o, V);
        if (e == hipSuccess) e = lin(B, m, k + 1 == P ? res : chain, 1, 1, o, 1, 0, nullptr, 0, V);
      }
      return e;
    };
    auto run_log = [&]() -> hipError_t {
      const int64_t sh = (int64_t)1 << (P - 3);
      hipError_t e = lin(B, m, x, 1, 1, lwe + c0 * B.lw, 1, 0, nullptr, 0, Q / p);  // m + 1
      if (e == hipSuccess) e = bits(B, m, P, x, E.data(), y, o);
      if (e == hipSuccess) e = lin(B, m, chain, 1, sh, E[P - 1], 1);
      if (e == hipSuccess) e = lin(B, m, res, 1, 0, x, 1, 0, nullptr, 0, (u128)kc * 2 * vo);
      if (e == hipSuccess && top == P - 1) {
        e = lin(B, m, y, 1, sh, E[P - 1], 1, 0, nullptr, 0, vc, true);
        if (e == hipSuccess) e = pbs(B, m, y, o, vo);
        if (e == hipSuccess) e = lin(B, m, res, 1, 1, res, 1, 1, o, 1, vo);
      }
      for (int i = (int)P - 2; e == hipSuccess && i >= 0; --i) {
        e = lin(B, m, y, 1, sh, E[i], 1, 1, chain, 1, vc, true);  // OR decision
        if (e == hipSuccess) e = pbs(B, m, y, o, vo);               // o_i at the output scale (o + V_o)
        if (e == hipSuccess && i == 0) e = lin(B, m, res, 1, 1, res, 1, -kc, o, 1, (u128)kc * vo, true);
        if (e == hipSuccess && i > 0 && (uint32_t)i <= top) e = lin(B, m, res, 1, 1, res, 1, 1, o, 1, vo);
        // back at the chain scale: 2^(log_p_out - 3) (o + V_o)
        if (e == hipSuccess && i > 0)
          e = lin(B, m, chain, 1, (int64_t)1 << (log_p_out - 3), o, 1, 0, nullptr, 0, ((u128)1 << (log_p_out - 3)) * vo);
      }
      return e;
    };
    HIP_TRY(timed(c, "activate", (double)m, st, [&] { return kind == HW_ACT_GE ? run_ge() : run_log(); }));
  }
  return ok();
}

extern "C" hw_status hw_activate(hw_ctx* c, const hw_boot_key* key, const uint32_t* lwe, uint64_t count,
                               uint32_t kind, uint64_t param, uint32_t log_p_out, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  return activate_core(c, key, lwe, count, kind, param, log_p_out, out, st);
}

extern "C" hw_status hw_activate_ge(hw_ctx* c, const hw_boot_key* key, const uint32_t* lwe, uint64_t count,
                                    uint64_t T, uint32_t log_p_out, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  return activate_core(c, key, lwe, count, HW_ACT_GE, T, log_p_out, out, st);
}

extern "C" hw_status hw_encrypted_argmax(hw_ctx* c, const hw_boot_key* key, const uint32_t* u,
                                         uint64_t count, uint32_t l, uint32_t log_p_in, uint32_t* out,
                                         hipStream_t st) {
  CHECK(enter(c));
  CHECK(check_pbs(c, key));
  if (l < 2 || l > 64) return fail(HW_EINVAL, "l = %u out of range [2, 64]", l);
  if (log_p_in < 3 || log_p_in > 20) return fail(HW_EINVAL, "log_p_in = %u out of range [3, 20]", log_p_in);
  if (count == 0) return ok();
  if (!u || !out) return fail(HW_EINVAL, "null buffer");
  const uint32_t P = log_p_in;
  uint32_t L = 0;
  while ((1u << L) < l) ++L;
  const u128 Q = c->Q, vi = (Q >> P) / 2, vc = Q / 16, vx = (Q >> (L + 1)) / 2;
  const u128 s8 = ((u128)1 << (P - 3)) * 2 * vi;
  // temporaries per sample: d, y, o, acc, the P bits, l (l - 1) G values and l W values
  const size_t ntmp = 4 + P + (size_t)l * (l - 1) + l;
  Pbs B;
  uint64_t cmax = 0;
  uint32_t* tmp = nullptr;
  CHECK(pbs_setup(c, key, count, ntmp, st, &B, &cmax, &tmp));
  for (uint64_t c0 = 0; c0 < count; c0 += cmax) {
    const uint64_t m = std::min(cmax, count - c0);
    const size_t A = cmax * B.lw;  // words of one temporary array
    uint32_t* d = tmp;
    uint32_t* y = d + A;
    uint32_t* o = y + A;
    uint32_t* acc = o + A;
    std::vector<uint32_t*> E(P);
    for (uint32_t k = 0; k < P; ++k) E[k] = acc + (k + 1) * A;
    uint32_t* G0 = acc + (P + 1) * A;
    auto G = [&](uint32_t a, uint32_t b) { return G0 + ((size_t)a * (l - 1) + (b < a ? b : b - 1)) * A; };
    uint32_t* W0 = G0 + (size_t)l * (l - 1) * A;
    const uint32_t* ub = u + c0 * l * B.lw;  // sample j, class a at ub + (j l + a) lw
    auto run = [&]() -> hipError_t {
      hipError_t e = hipSuccess;
      for (uint32_t a = 0; e == hipSuccess && a < l; ++a)
        for (uint32_t b = a + 1; e == hipSuccess && b < l; ++b) {
          e = lin(B, m, d, 1, 1, ub + a * B.lw, l, -1, ub + b * B.lw, l, (u128)(1ull << (P - 1)) * 2 * vi);
          if (e == hipSuccess) e = bits(B, m, P, d, E.data(), y, o);
          if (e == hipSuccess) e = lin(B, m, G(a, b), 1, (int64_t)1 << (P - 3), E[P - 1], 1);
          if (e == hipSuccess) e = lin(B, m, G(b, a), 1, -1, G(a, b), 1, 0, nullptr, 0, s8);
        }
      for (uint32_t a = 0; e == hipSuccess && a < l; ++a) {
        uint32_t* W = W0 + (size_t)a * A;
        std::vector<uint32_t> others;
        for (uint32_t b = 0; b < l; ++b)
          if (b != a) others.push_back(b);
        if (l == 2) {
          e = lin(B, m, W, 1, 2, G(a, others[0]), 1);
          continue;
        }
        e = lin(B, m, acc, 1, 1, G(a, others[0]), 1);
        for (size_t j = 1; e == hipSuccess && j < others.size(); ++j) {
          const bool last = j + 1 == others.size();
          const u128 V = last ? vx : vc;
          e = lin(B, m, y, 1, 1, acc, 1, 1, G(a, others[j]), 1, 3 * vc, true);
          if (e == hipSuccess) e = pbs(B, m, y, o, V);
          if (e == hipSuccess) e = lin(B, m, last ? W : acc, 1, 1, o, 1, 0, nullptr, 0, V);
        }
      }
      // index = sum_a a W_a
      if (e == hipSuccess) e = lin(B, m, out + c0 * B.lw, 1, 0, W0, 1);
      for (uint32_t a = 1; e == hipSuccess && a < l; ++a)
        e = lin(B, m, out + c0 * B.lw, 1, 1, out + c0 * B.lw, 1, a, W0 + (size_t)a * A, 1);
      return e;
    };
    HIP_TRY(timed(c, "argmax", (double)m, st, run));
  }
  return ok();
}

extern "C" hw_status hw_class_sums(hw_ctx* c, const uint32_t* scores, uint64_t n, uint32_t l, uint32_t k0,
                                   uint32_t* sums, hipStream_t st) {
  CHECK(enter(c));
  if (n == 0) return ok();
  if (!scores || !sums) return fail(HW_EINVAL, "null buffer");
  if (l < 1 || k0 < 1) return fail(HW_EINVAL, "l and k0 must be >= 1");
  hw::SumArgs S{};
  S.scores = scores;
  S.sums = sums;
  S.n = n;
  S.l = l;
  S.k0 = k0;
  S.N = c->prm.N;
  S.nq = c->prm.nq;
  HIP_TRY(hw::launch_class_sums(c->tabs, S, st));
  return ok();
}

extern "C" hw_status hw_fm_act(hw_ctx* c, const hw_wisard_shape* sh, const hw_boot_key* key,
                               const uint32_t* pks_key, const uint32_t* model, uint32_t kind, uint64_t param,
                               uint32_t log_p_out, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  Dims d;
  CHECK(check_shape(c, sh, &d));
  CHECK(check_pbs(c, key));
  if (!pks_key || !model || !out) return fail(HW_EINVAL, "null buffer");
  // the activation's argument checks, before anything is allocated or run
  CHECK(activate_core(c, key, nullptr, 0, kind, param, log_p_out, nullptr, st));
  const uint32_t N = c->prm.N;
  const size_t rw = rlwe_words(c), lw = lwe_words(c);
  const uint64_t rows = (uint64_t)d.rows * d.k1;
  {
    const uintptr_t i0 = reinterpret_cast<uintptr_t>(model), i1 = i0 + (uintptr_t)rows * rw * 4;
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(out), o1 = o0 + (uintptr_t)rows * rw * 4;
    if (o0 != i0 && i0 < o1 && o0 < i1) return fail(HW_EINVAL, "out must be model itself or not overlap it");
  }
  // cells of a row: every coefficient a RAM's index can address
  const uint32_t K = d.layout == 2 ? N : 1u << std::min<uint32_t>(d.nbf, (uint32_t)c->logN);
  const uint64_t per = std::max<uint64_t>(1, FM_CHUNK_CELLS / K);  // rows per chunk
  const uint64_t cells = std::min<uint64_t>(per, rows) * K;
  uint32_t* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, 2 * cells * lw * 4));
  uint32_t* ext = buf;
  uint32_t* act = buf + cells * lw;
  hw_status rc = HW_OK;
  for (uint64_t r0 = 0; rc == HW_OK && r0 < rows; r0 += per) {
    const uint64_t m = std::min(per, rows - r0);
    hw::CellArgs A{model + r0 * rw, ext, m, K, N, c->prm.nq};
    const uint64_t words = m * K * lw;
    hipError_t e = timed(c, "extract_cells", (double)(m * K), st, [&] {
      hipLaunchKernelGGL(hw::k_extract_cells, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, c->tabs, A);
      return hipGetLastError();
    });
    if (e != hipSuccess) {
      rc = fail(HW_EDEVICE, "k_extract_cells: %s", hipGetErrorString(e));
      break;
    }
    rc = activate_core(c, key, ext, m * K, kind, param, log_p_out, act, st);
    if (rc == HW_OK) rc = hw_pack_lwe(c, pks_key, act, K, m, out + r0 * rw, st);
  }
  // the chunks' buffers are released once the stream has used them
  const hipError_t es = hipStreamSynchronize(st);
  (void)hipFree(buf);
  if (rc != HW_OK) return rc;
  HIP_TRY(es);
  return ok();
}
