/*
 * oracle.c -- plain, slow CPU oracle for the encrypted WiSARD hot path of
 * "Homomorphic WiSARDs" (arXiv 2403.20190).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU product path
 * neither links nor calls it, and the two share no code, headers or tables.
 *
 * What it computes, in the paper's terms:
 *   ring R_q = Z_q[X]/(X^N+1)                          (Sec. 2.1, Notation)
 *   SecretKeyGen / EncRLWE / EncRGSW / DecRLWE / DecLWE (Sec. 2.5.1)
 *   external product, CMUX, ExtractLWE, BlindRotate     (Sec. 2.5.1)
 *   Vertical Packing                                    (Sec. 2.5.2, Alg. 3)
 *   CDEMUX gate and tree, Inverse Vertical Packing      (Sec. 3.3, Alg. 5)
 *   homomorphic training                                (Sec. 3.4, Alg. 6)
 *   homomorphic inference, PD-act branch                (Sec. 3.6, Alg. 7)
 *   class counter for dataset balancing                 (Sec. 3.7.1)
 * The paper works over a 64-bit torus; this oracle uses residues modulo 30-bit
 * NTT-friendly primes in RNS, a ternary secret, a discrete Gaussian of
 * sigma = 3.2 and an exact RNS gadget of base 2^6 with 5 digits per prime.
 * Every reading taken where the paper is silent or garbled is stated next to
 * the function that takes it.
 *
 * All arithmetic is exact: residues live in uint64_t, products of two residues
 * (< 2^60) are reduced with the C '%' operator, CRT values use unsigned
 * __int128.  Negacyclic products go through a textbook radix-2 NTT (a library
 * step); the tests pin it to schoolbook multiplication.
 *
 * Layouts (all uint32_t residues in [0, q_i), coefficient domain):
 *   polynomial over all primes : [prime][N]
 *   RLWE                       : [poly a=0, b=1][prime][N]
 *   RGSW                       : [row 0..2D)[poly][prime][N], D = digits*nq;
 *                                rows 0..D-1 carry the gadget in b, rows
 *                                D..2D-1 carry it in a; within a side, row
 *                                i*digits + j is prime i, digit j.
 *   LWE                        : [prime][N+1]  (a_0..a_{N-1}, b)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORC_MAXQ 4
#define DOM_KEY 1u
#define DOM_PERM 2u
#define DOM_ENC_A 3u
#define DOM_ENC_E 4u
#define DOM_ENC_A2 5u
#define CDT_TAIL 41

/* ------------------------------------------------------------------------ */
/* modular integer helpers                                                  */
/* ------------------------------------------------------------------------ */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (a * b) % q; }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (a + b) % q; }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return (a + q - b) % q; }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

/* inverse of a modulo the prime q, by Fermat's little theorem */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }

/* primality by trial division; fine for the < 2^32 moduli used here */
int orc_is_prime(uint64_t n) {
  if (n < 2) return 0;
  if (n % 2 == 0) return n == 2;
  for (uint64_t d = 3; d * d <= n; d += 2)
    if (n % d == 0) return 0;
  return 1;
}

/* Parameter rule: the nq largest primes q < 2^30 with q = 1 (mod 2N), in
 * decreasing order.  The paper fixes only a torus modulus (Table 2); the prime
 * choice is this implementation's reading.  Returns 0 on success. */
int orc_find_primes(uint32_t N, uint32_t nq, uint32_t* out) {
  uint64_t m = 2ull * N;
  uint64_t q = ((((1ull << 30) - 1) - 1) / m) * m + 1;
  uint32_t found = 0;
  while (found < nq && q > m) {
    if (orc_is_prime(q)) out[found++] = (uint32_t)q;
    q -= m;
  }
  return found == nq ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the 64-bit draw     */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* Weyl key schedule */
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
  memcpy(out, c, sizeof c);
}

/* Counter-based 64-bit draw number `index` of stream (seed, domain): the key is
 * the seed, the counter is (index/2, domain, 0); even indices take output
 * words 0,1, odd indices words 2,3 (low word first).  The paper does not name
 * a generator; this is the reading used by both implementations. */
uint64_t orc_w64(uint64_t seed, uint32_t domain, uint64_t index) {
  uint64_t blk = index >> 1;
  uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), domain, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  if (index & 1) return (uint64_t)o[2] | ((uint64_t)o[3] << 32);
  return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
}

/* 32-bit draw number `index` of stream (seed, domain): word index mod 4 of
 * block index / 4 (counter (block, domain, 0), key = seed). */
uint32_t orc_w32(uint64_t seed, uint32_t domain, uint64_t index) {
  uint64_t blk = index >> 2;
  uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), domain, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  return o[index & 3];
}

/* Uniform residue mod q of draw x of the encryption stream: the 32-bit word
 * w = w32(seed, ENC_A, x) when w < floor(2^32 / q) q, as w mod q (each
 * residue then has exactly floor(2^32 / q) preimages); otherwise the 64-bit
 * draw w64(seed, ENC_A2, x) mod q (probability (2^32 mod q) / 2^32, about
 * 3e-5 for q near 2^30). */
uint64_t orc_uniform_mod(uint64_t seed, uint64_t x, uint64_t q) {
  uint32_t w = orc_w32(seed, DOM_ENC_A, x);
  uint64_t lim = (((uint64_t)1 << 32) / q) * q;
  if (w < lim) return w % q;
  return orc_w64(seed, DOM_ENC_A2, x) % q;
}

/* ------------------------------------------------------------------------ */
/* discrete Gaussian by cumulative distribution table                        */
/* ------------------------------------------------------------------------ */

/* T[k] = floor(2^63 * P(|X| <= k)) for X the discrete Gaussian of standard
 * deviation sigma cut at |X| <= 41, with rho(x) = exp(-x^2 / (2 sigma^2)).
 * The cumulative sums run over x = 0, 1, 2, ... with weight 1 for x = 0 and
 * 2*rho(x) otherwise, in that order, in double precision; T[41] = 2^63. */
void orc_cdt_table(double sigma, uint64_t* T) {
  double cum[CDT_TAIL + 1];
  double acc = 0.0;
  for (int x = 0; x <= CDT_TAIL; ++x) {
    double w = (x == 0) ? 1.0 : 2.0 * exp(-((double)x * (double)x) / (2.0 * sigma * sigma));
    acc = acc + w;
    cum[x] = acc;
  }
  for (int x = 0; x < CDT_TAIL; ++x) T[x] = (uint64_t)floor(ldexp(cum[x] / cum[CDT_TAIL], 63));
  T[CDT_TAIL] = 1ull << 63;
}

/* magnitude = smallest k with (w >> 1) < T[k]; sign from bit 0 of w; a zero
 * magnitude ignores the sign */
int64_t orc_cdt_sample(const uint64_t* T, uint64_t w) {
  uint64_t r = w >> 1;
  int64_t k = 0;
  while (!(r < T[k])) ++k;
  if (k != 0 && (w & 1)) return -k;
  return k;
}

/* ------------------------------------------------------------------------ */
/* context                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t N, logN, nq, log_base, digits, D;
  uint64_t p;
  uint64_t q[ORC_MAXQ];
  u128 Q, delta;                  /* Q = prod q_i, delta = floor(Q / p) */
  uint64_t delta_mod[ORC_MAXQ];   /* delta mod q_i */
  uint64_t crt_inv[ORC_MAXQ];     /* [(Q/q_i)^{-1}]_{q_i} */
  uint64_t psi[ORC_MAXQ];         /* primitive 2N-th root of unity mod q_i */
  uint64_t* psi_pow[ORC_MAXQ];    /* psi^j, j < N */
  uint64_t* psi_ipow[ORC_MAXQ];   /* psi^{-j}, j < N */
  uint64_t* omega_pow[ORC_MAXQ];  /* omega^j, omega = psi^2, j < N */
  uint64_t* omega_ipow[ORC_MAXQ]; /* omega^{-j} */
  uint64_t n_inv[ORC_MAXQ];
  uint64_t cdt[CDT_TAIL + 1];
  double sigma;
} orc_ctx;

/* smallest x >= 2 such that psi = x^((q-1)/2N) has psi^N = -1 mod q; such a
 * psi has multiplicative order exactly 2N */
static uint64_t find_psi(uint64_t q, uint32_t N) {
  for (uint64_t x = 2; x < q; ++x) {
    uint64_t psi = powmod(x, (q - 1) / (2ull * N), q);
    if (powmod(psi, N, q) == q - 1) return psi;
  }
  return 0;
}

void orc_ctx_free(orc_ctx* c) {
  if (!c) return;
  for (uint32_t i = 0; i < ORC_MAXQ; ++i) {
    free(c->psi_pow[i]);
    free(c->psi_ipow[i]);
    free(c->omega_pow[i]);
    free(c->omega_ipow[i]);
  }
  free(c);
}

/* primes[] == NULL or primes[0] == 0 selects the rule of orc_find_primes */
orc_ctx* orc_ctx_new(uint32_t N, uint32_t nq, const uint32_t* primes, uint32_t log_base,
                     uint32_t digits, uint64_t p, double sigma) {
  if (N < 2 || (N & (N - 1)) || nq < 1 || nq > ORC_MAXQ) return NULL;
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->N = N;
  c->logN = 0;
  while ((1u << c->logN) < N) c->logN++;
  c->nq = nq;
  c->log_base = log_base;
  c->digits = digits;
  c->D = digits * nq;
  c->p = p;
  c->sigma = sigma;
  uint32_t pr[ORC_MAXQ] = {0};
  if (primes && primes[0]) {
    for (uint32_t i = 0; i < nq; ++i) pr[i] = primes[i];
  } else if (orc_find_primes(N, nq, pr) != 0) {
    free(c);
    return NULL;
  }
  c->Q = 1;
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = pr[i];
    if (!orc_is_prime(q) || (q - 1) % (2ull * N) != 0) {
      orc_ctx_free(c);
      return NULL;
    }
    c->q[i] = q;
    c->Q *= q;
  }
  c->delta = c->Q / p;
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    c->delta_mod[i] = (uint64_t)(c->delta % q);
    uint64_t Mi = (uint64_t)((c->Q / q) % q);
    c->crt_inv[i] = invmod(Mi, q);
    c->psi[i] = find_psi(q, N);
    uint64_t psi = c->psi[i], psi_inv = invmod(psi, q);
    uint64_t om = mulmod(psi, psi, q), om_inv = invmod(om, q);
    c->psi_pow[i] = (uint64_t*)malloc(sizeof(uint64_t) * N);
    c->psi_ipow[i] = (uint64_t*)malloc(sizeof(uint64_t) * N);
    c->omega_pow[i] = (uint64_t*)malloc(sizeof(uint64_t) * N);
    c->omega_ipow[i] = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t a = 1, b = 1, d = 1, e = 1;
    for (uint32_t j = 0; j < N; ++j) {
      c->psi_pow[i][j] = a;
      c->psi_ipow[i][j] = b;
      c->omega_pow[i][j] = d;
      c->omega_ipow[i][j] = e;
      a = mulmod(a, psi, q);
      b = mulmod(b, psi_inv, q);
      d = mulmod(d, om, q);
      e = mulmod(e, om_inv, q);
    }
    c->n_inv[i] = invmod(N, q);
  }
  orc_cdt_table(sigma, c->cdt);
  return c;
}

void orc_ctx_info(const orc_ctx* c, uint32_t* primes, uint64_t* delta_mod, uint64_t* q_words,
                  uint64_t* delta_words) {
  for (uint32_t i = 0; i < c->nq; ++i) {
    primes[i] = (uint32_t)c->q[i];
    delta_mod[i] = c->delta_mod[i];
  }
  q_words[0] = (uint64_t)c->Q;
  q_words[1] = (uint64_t)(c->Q >> 64);
  delta_words[0] = (uint64_t)c->delta;
  delta_words[1] = (uint64_t)(c->delta >> 64);
}

void orc_ctx_cdt(const orc_ctx* c, uint64_t* T) { memcpy(T, c->cdt, sizeof c->cdt); }

/* ------------------------------------------------------------------------ */
/* polynomial arithmetic in Z_q[X]/(X^N+1)                                   */
/* ------------------------------------------------------------------------ */

/* negacyclic product by the definition: X^N = -1 (Notation, Sec. 2.1) */
void orc_negmul_schoolbook(uint32_t N, uint64_t q, const uint64_t* a, const uint64_t* b,
                           uint64_t* out) {
  for (uint32_t k = 0; k < N; ++k) out[k] = 0;
  for (uint32_t i = 0; i < N; ++i)
    for (uint32_t j = 0; j < N; ++j) {
      uint64_t t = mulmod(a[i] % q, b[j] % q, q);
      uint32_t k = i + j;
      if (k < N)
        out[k] = addmod(out[k], t, q);
      else
        out[k - N] = submod(out[k - N], t, q);
    }
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

/* textbook iterative radix-2 cyclic NTT, A[k] = sum_j a[j] w^{jk}; `wpow`
 * holds w^j for j < N */
static void cyclic_ntt(uint64_t* a, uint32_t N, uint32_t logN, uint64_t q, const uint64_t* wpow) {
  for (uint32_t i = 0; i < N; ++i) {
    uint32_t r = bitrev(i, logN);
    if (r > i) {
      uint64_t t = a[i];
      a[i] = a[r];
      a[r] = t;
    }
  }
  for (uint32_t len = 2; len <= N; len <<= 1) {
    uint32_t half = len >> 1, step = N / len;
    for (uint32_t s = 0; s < N; s += len)
      for (uint32_t j = 0; j < half; ++j) {
        uint64_t u = a[s + j];
        uint64_t v = mulmod(a[s + j + half], wpow[j * step], q);
        a[s + j] = addmod(u, v, q);
        a[s + j + half] = submod(u, v, q);
      }
  }
}

/* negacyclic product through the psi-twisted cyclic NTT:
 * c = psi^{-j} * INTT( NTT(a psi^j) * NTT(b psi^j) ) */
static void negmul_ntt(const orc_ctx* c, uint32_t i, const uint64_t* a, const uint64_t* b,
                       uint64_t* out) {
  uint32_t N = c->N;
  uint64_t q = c->q[i];
  uint64_t* A = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* B = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t j = 0; j < N; ++j) {
    A[j] = mulmod(a[j] % q, c->psi_pow[i][j], q);
    B[j] = mulmod(b[j] % q, c->psi_pow[i][j], q);
  }
  cyclic_ntt(A, N, c->logN, q, c->omega_pow[i]);
  cyclic_ntt(B, N, c->logN, q, c->omega_pow[i]);
  for (uint32_t j = 0; j < N; ++j) A[j] = mulmod(A[j], B[j], q);
  cyclic_ntt(A, N, c->logN, q, c->omega_ipow[i]);
  for (uint32_t j = 0; j < N; ++j)
    out[j] = mulmod(mulmod(A[j], c->n_inv[i], q), c->psi_ipow[i][j], q);
  free(A);
  free(B);
}

/* exported for the pins: product of two residue polynomials mod q_i */
void orc_negmul(const orc_ctx* c, uint32_t i, const uint64_t* a, const uint64_t* b, uint64_t* out) {
  negmul_ntt(c, i, a, b, out);
}

/* out (+)= poly * (integer polynomial d lifted mod q_i), all for prime i */
static void mul_acc_small(const orc_ctx* c, uint32_t i, const int32_t* d, const uint32_t* poly,
                          uint32_t* acc) {
  uint32_t N = c->N;
  uint64_t q = c->q[i];
  uint64_t* A = (uint64_t*)calloc(N, sizeof(uint64_t));
  uint64_t* B = (uint64_t*)calloc(N, sizeof(uint64_t));
  uint64_t* P = (uint64_t*)calloc(N, sizeof(uint64_t));
  for (uint32_t j = 0; j < N; ++j) {
    int64_t v = d[j];
    A[j] = (uint64_t)(v < 0 ? v + (int64_t)q : v);
    B[j] = poly[j];
  }
  negmul_ntt(c, i, A, B, P);
  for (uint32_t j = 0; j < N; ++j) acc[j] = (uint32_t)addmod(acc[j], P[j], q);
  free(A);
  free(B);
  free(P);
}

/* RLWE helpers; an RLWE holds 2*nq*N words */
static size_t rlwe_words(const orc_ctx* c) { return 2ull * c->nq * c->N; }
static size_t rgsw_words(const orc_ctx* c) { return 2ull * c->D * rlwe_words(c); }

static void rlwe_add(const orc_ctx* c, const uint32_t* x, const uint32_t* y, uint32_t* out) {
  for (uint32_t p = 0; p < 2; ++p)
    for (uint32_t i = 0; i < c->nq; ++i)
      for (uint32_t k = 0; k < c->N; ++k) {
        size_t o = ((size_t)p * c->nq + i) * c->N + k;
        out[o] = (uint32_t)addmod(x[o], y[o], c->q[i]);
      }
}

static void rlwe_sub(const orc_ctx* c, const uint32_t* x, const uint32_t* y, uint32_t* out) {
  for (uint32_t p = 0; p < 2; ++p)
    for (uint32_t i = 0; i < c->nq; ++i)
      for (uint32_t k = 0; k < c->N; ++k) {
        size_t o = ((size_t)p * c->nq + i) * c->N + k;
        out[o] = (uint32_t)submod(x[o], y[o], c->q[i]);
      }
}

/* Multiplication by the monomial X^e, e any integer (negacyclic: X^N = -1),
 * applied to both polynomials of an RLWE. */
void orc_rlwe_rotate(const orc_ctx* c, const uint32_t* in, int64_t e, uint32_t* out) {
  uint32_t N = c->N;
  int64_t twoN = 2 * (int64_t)N;
  int64_t em = ((e % twoN) + twoN) % twoN;
  for (uint32_t p = 0; p < 2; ++p)
    for (uint32_t i = 0; i < c->nq; ++i) {
      const uint32_t* src = in + ((size_t)p * c->nq + i) * N;
      uint32_t* dst = out + ((size_t)p * c->nq + i) * N;
      uint64_t q = c->q[i];
      for (uint32_t j = 0; j < N; ++j) {
        int64_t t = j + em;
        int neg = 0;
        if (t >= twoN) t -= twoN;
        if (t >= N) {
          t -= N;
          neg = 1;
        }
        dst[t] = neg ? (uint32_t)((q - src[j]) % q) : src[j];
      }
    }
}

/* ------------------------------------------------------------------------ */
/* keys, encryption, decryption (Sec. 2.5.1)                                 */
/* ------------------------------------------------------------------------ */

/* ternary secret s_k = (w64(seed, KEY, k) mod 3) - 1; the paper samples a
 * binary key, the ternary key is this implementation's parameter choice */
void orc_keygen(const orc_ctx* c, uint64_t seed, int32_t* s) {
  for (uint32_t k = 0; k < c->N; ++k) s[k] = (int32_t)(orc_w64(seed, DOM_KEY, k) % 3) - 1;
}

/* The polynomial of prime i whose value at the point psi^(2 brv(k) + 1) is
 * ev[k] for every k < N (brv: bit reversal over log2 N bits).  Evaluation at
 * the N roots psi^(2m+1) of X^N + 1 is a bijection of R_q onto Z_q^N (the
 * ring isomorphism behind NTT multiplication, Sec. 2.1); its inverse is
 * a_j = psi^{-j} N^{-1} sum_m E_m omega^{-m j} with E_m = ev[brv(m)], the
 * value at psi^(2m+1), and omega = psi^2. */
static void from_evaluations(const orc_ctx* c, uint32_t i, const uint64_t* ev, uint64_t* a) {
  uint32_t N = c->N;
  uint64_t q = c->q[i];
  for (uint32_t m = 0; m < N; ++m) a[m] = ev[bitrev(m, c->logN)];
  cyclic_ntt(a, N, c->logN, q, c->omega_ipow[i]);
  for (uint32_t j = 0; j < N; ++j) a[j] = mulmod(mulmod(a[j], c->n_inv[i], q), c->psi_ipow[i][j], q);
}

/* EncRLWE of an integer polynomial mu (coefficients in [0, p)):
 * b = a*s + Delta*mu + e, a uniform in R_q (Sec. 2.5.1).  The draws of row
 * `row` of ciphertext `ct` among `rows` rows per ciphertext are
 *   u_{i,k} = uniform_mod(seed, ((ct*rows + row)*nq + i)*N + k, q_i)
 *   e_k     = CDT(w64(seed, ENC_E, (ct*rows + row)*N + 8 (k mod N/8) + floor(k / (N/8)))),
 * e being one integer polynomial shared by all primes.  With a_eval == 0
 * the u_{i,k} are the coefficients of a mod q_i; with a_eval != 0 they are
 * its values at the points psi_i^(2 brv(k) + 1) (the same uniform
 * distribution on R_q, since evaluation is a bijection).  mu == NULL
 * encrypts 0. */
static void enc_row(const orc_ctx* c, const int32_t* s, const uint64_t* mu, uint64_t seed, uint64_t ct,
                    uint64_t rows, uint64_t row, int a_eval, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t* A = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* S = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * N);
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * N);
  uint64_t rid = ct * rows + row;
  /* coefficient k takes error draw 8 (k mod N/8) + k / (N/8): a bijection
   * of [0, N) (the order in which the draws are consumed is a convention) */
  for (uint32_t k = 0; k < N; ++k) {
    uint32_t pos = 8u * (k % (N / 8u)) + k / (N / 8u);
    e[k] = orc_cdt_sample(c->cdt, orc_w64(seed, DOM_ENC_E, rid * N + pos));
  }
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    for (uint32_t k = 0; k < N; ++k) {
      P[k] = orc_uniform_mod(seed, (rid * nq + i) * N + k, q);
      S[k] = (uint64_t)(s[k] < 0 ? (int64_t)q + s[k] : s[k]);
    }
    if (a_eval)
      from_evaluations(c, i, P, A);
    else
      memcpy(A, P, sizeof(uint64_t) * N);
    negmul_ntt(c, i, A, S, P);
    uint32_t* oa = out + (size_t)i * N;
    uint32_t* ob = out + ((size_t)nq + i) * N;
    for (uint32_t k = 0; k < N; ++k) {
      uint64_t ek = (uint64_t)(e[k] < 0 ? (int64_t)q + e[k] : e[k]);
      uint64_t m = mu ? mulmod(c->delta_mod[i], mu[k] % q, q) : 0;
      oa[k] = (uint32_t)A[k];
      ob[k] = (uint32_t)addmod(addmod(P[k], m, q), ek, q);
    }
  }
  free(A);
  free(S);
  free(P);
  free(e);
}

void orc_enc_rlwe_row(const orc_ctx* c, const int32_t* s, const uint64_t* mu, uint64_t seed,
                      uint64_t ct, uint64_t rows, uint64_t row, uint32_t* out) {
  enc_row(c, s, mu, seed, ct, rows, row, 0, out);
}

/* RLWE ciphertexts draw a by its coefficients */
void orc_enc_rlwe(const orc_ctx* c, const int32_t* s, const uint64_t* mu, uint64_t seed, uint64_t ct,
                  uint32_t* out) {
  enc_row(c, s, mu, seed, ct, 1, 0, 0, out);
}

/* EncRGSW of a bit m: 2D rows, each an encryption of 0, plus m * g_{i,j} on
 * residue i of the b part (rows i*digits+j) or of the a part (rows
 * D + i*digits + j), g_{i,j} = base^j.  The paper's gadget entry carries a
 * stray 1/p factor (Sec. 2.5.1, EncRGSW); the exact gadget base^j is the
 * reading taken here, in its RNS form (one gadget row per prime and digit).
 * Each row draws its a by its values at the evaluation points (enc_row). */
void orc_enc_rgsw(const orc_ctx* c, const int32_t* s, uint32_t m, uint64_t seed, uint64_t ct,
                  uint32_t* out) {
  uint32_t N = c->N, nq = c->nq, D = c->D, rows = 2 * D;
  size_t rw = rlwe_words(c);
  for (uint32_t r = 0; r < rows; ++r) {
    uint32_t* row = out + r * rw;
    enc_row(c, s, NULL, seed, ct, rows, r, 1, row);
    if (m) {
      uint32_t side = r < D ? 1u : 0u; /* b for the first D rows, a after */
      uint32_t rr = r % D, i = rr / c->digits, j = rr % c->digits;
      uint64_t q = c->q[i];
      uint64_t g = powmod(1ull << c->log_base, j, q);
      uint32_t* poly = row + ((size_t)side * nq + i) * N;
      poly[0] = (uint32_t)addmod(poly[0], g, q);
    }
  }
}

/* a noiseless RGSW m*G, used by the pins (a trivial encryption) */
void orc_trivial_rgsw(const orc_ctx* c, uint32_t m, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq, D = c->D;
  size_t rw = rlwe_words(c);
  memset(out, 0, sizeof(uint32_t) * rgsw_words(c));
  if (!m) return;
  for (uint32_t r = 0; r < 2 * D; ++r) {
    uint32_t side = r < D ? 1u : 0u;
    uint32_t rr = r % D, i = rr / c->digits, j = rr % c->digits;
    out[r * rw + ((size_t)side * nq + i) * N] = (uint32_t)powmod(1ull << c->log_base, j, c->q[i]);
  }
}

/* CRT: the unique phi in [0, Q) with phi = x_i mod q_i */
static u128 crt(const orc_ctx* c, const uint64_t* x) {
  u128 phi = 0;
  for (uint32_t i = 0; i < c->nq; ++i) {
    uint64_t q = c->q[i];
    uint64_t y = mulmod(x[i] % q, c->crt_inv[i], q);
    u128 Mi = c->Q / q;
    phi += (u128)y * Mi;
    while (phi >= c->Q) phi -= c->Q;
  }
  return phi;
}

/* decode: mu = floor((p*phi + floor(Q/2)) / Q) mod p, i.e. phi/Delta rounded
 * half up (the paper's rounding of (b - <a,s>)/(q/p), Sec. 2.5.1) */
static uint64_t decode(const orc_ctx* c, u128 phi) {
  u128 num = (u128)c->p * phi + c->Q / 2;
  return (uint64_t)((num / c->Q) % c->p);
}

/* phase b - a*s of an RLWE, per prime, coefficient domain */
static void rlwe_phase(const orc_ctx* c, const int32_t* s, const uint32_t* ct, uint64_t* ph) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t* A = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* S = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    for (uint32_t k = 0; k < N; ++k) {
      A[k] = ct[(size_t)i * N + k];
      S[k] = (uint64_t)(s[k] < 0 ? (int64_t)q + s[k] : s[k]);
    }
    negmul_ntt(c, i, A, S, P);
    for (uint32_t k = 0; k < N; ++k) ph[(size_t)i * N + k] = submod(ct[((size_t)nq + i) * N + k], P[k], q);
  }
  free(A);
  free(S);
  free(P);
}

void orc_dec_rlwe(const orc_ctx* c, const int32_t* s, const uint32_t* ct, uint64_t* mu) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t* ph = (uint64_t*)malloc(sizeof(uint64_t) * nq * N);
  rlwe_phase(c, s, ct, ph);
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t x[ORC_MAXQ];
    for (uint32_t i = 0; i < nq; ++i) x[i] = ph[(size_t)i * N + k];
    mu[k] = decode(c, crt(c, x));
  }
  free(ph);
}

/* signed noise phi - Delta*mu (centered mod Q) per coefficient, as a double;
 * returns the largest magnitude */
double orc_noise_rlwe(const orc_ctx* c, const int32_t* s, const uint32_t* ct, const uint64_t* mu,
                      double* noise_out) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t* ph = (uint64_t*)malloc(sizeof(uint64_t) * nq * N);
  rlwe_phase(c, s, ct, ph);
  double mx = 0;
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t x[ORC_MAXQ];
    for (uint32_t i = 0; i < nq; ++i) x[i] = ph[(size_t)i * N + k];
    u128 phi = crt(c, x);
    u128 dm = (c->delta * (u128)(mu[k] % c->p)) % c->Q;
    u128 d = phi >= dm ? phi - dm : phi + c->Q - dm;
    double v = (d > c->Q / 2) ? -(double)(c->Q - d) : (double)d;
    if (noise_out) noise_out[k] = v;
    if (fabs(v) > mx) mx = fabs(v);
  }
  free(ph);
  return mx;
}

/* DecLWE: phi = b - <a, s> (Sec. 2.5.1) then the same rounding */
void orc_dec_lwe(const orc_ctx* c, const int32_t* s, const uint32_t* lwe, uint64_t* mu) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t x[ORC_MAXQ];
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    const uint32_t* a = lwe + (size_t)i * (N + 1);
    uint64_t acc = 0;
    for (uint32_t k = 0; k < N; ++k) {
      uint64_t sk = (uint64_t)(s[k] < 0 ? (int64_t)q + s[k] : s[k]);
      acc = addmod(acc, mulmod(a[k], sk, q), q);
    }
    x[i] = submod(a[N], acc, q);
  }
  *mu = decode(c, crt(c, x));
}

/* ------------------------------------------------------------------------ */
/* gadget decomposition and the external product                             */
/* ------------------------------------------------------------------------ */

/* Balanced base-2^log_base digits of each residue: v = the residue centered
 * in (-q/2, q/2); for j < digits-1: d = v mod B in [0, B), d -= B if
 * d >= B/2, v = (v - d)/B; the last digit is what remains of v.  Then
 * sum_j d_j B^j = v exactly.  Output digit polynomial (i, j) at
 * out[(i*digits + j)*N + k]. */
void orc_decompose(const orc_ctx* c, const uint32_t* poly, int32_t* out) {
  uint32_t N = c->N;
  int64_t B = 1ll << c->log_base;
  for (uint32_t i = 0; i < c->nq; ++i) {
    int64_t q = (int64_t)c->q[i];
    for (uint32_t k = 0; k < N; ++k) {
      int64_t v = poly[(size_t)i * N + k];
      if (v > (q - 1) / 2) v -= q;
      for (uint32_t j = 0; j + 1 < c->digits; ++j) {
        int64_t d = ((v % B) + B) % B;
        if (d >= B / 2) d -= B;
        out[((size_t)i * c->digits + j) * N + k] = (int32_t)d;
        v = (v - d) / B;
      }
      out[((size_t)i * c->digits + c->digits - 1) * N + k] = (int32_t)v;
    }
  }
}

/* External product C [.] (a, b) = sum_{i,j} dec(b)_{i,j} * C[B(i,j)]
 *                               + sum_{i,j} dec(a)_{i,j} * C[A(i,j)]
 * with B(i,j) = i*digits + j and A(i,j) = D + i*digits + j; each digit
 * polynomial is lifted into every prime (Sec. 2.5.1, multiplication). */
void orc_extprod(const orc_ctx* c, const uint32_t* C, const uint32_t* in, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq, D = c->D;
  size_t rw = rlwe_words(c);
  int32_t* dig = (int32_t*)malloc(sizeof(int32_t) * (size_t)D * N);
  memset(out, 0, sizeof(uint32_t) * rw);
  for (uint32_t side = 0; side < 2; ++side) {
    /* side 0 decomposes b against the B-rows, side 1 decomposes a against the A-rows */
    const uint32_t* src = in + (side == 0 ? (size_t)nq * N : 0);
    uint32_t row0 = side == 0 ? 0 : D;
    orc_decompose(c, src, dig);
    for (uint32_t r = 0; r < D; ++r) {
      const uint32_t* row = C + (size_t)(row0 + r) * rw;
      for (uint32_t ip = 0; ip < nq; ++ip) {
        mul_acc_small(c, ip, dig + (size_t)r * N, row + (size_t)ip * N, out + (size_t)ip * N);
        mul_acc_small(c, ip, dig + (size_t)r * N, row + ((size_t)nq + ip) * N,
                      out + ((size_t)nq + ip) * N);
      }
    }
  }
  free(dig);
}

/* CMUX(C, d1, d0) = d0 + C [.] (d1 - d0): selects d1 when C encrypts 1 */
void orc_cmux(const orc_ctx* c, const uint32_t* C, const uint32_t* d1, const uint32_t* d0,
              uint32_t* out) {
  size_t rw = rlwe_words(c);
  uint32_t* diff = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  uint32_t* h = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  rlwe_sub(c, d1, d0, diff);
  orc_extprod(c, C, diff, h);
  rlwe_add(c, d0, h, out);
  free(diff);
  free(h);
}

/* BlindRotate: for t = 0, 1, ..., k-1: acc <- CMUX(C_t, X^{e_t} acc, acc).
 * With C_t encrypting S_t the result encrypts v * X^{sum_t S_t e_t}; the
 * paper's I_t is -e_t (Sec. 2.5.1). */
static uint32_t ceil_log2_u(uint32_t l) {
  uint32_t L = 0;
  while ((1u << L) < l) ++L;
  return L;
}

void orc_blind_rotate(const orc_ctx* c, const uint32_t* in, const uint32_t* const* C,
                      const int64_t* e, uint32_t k, uint32_t* out) {
  size_t rw = rlwe_words(c);
  uint32_t* rot = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  memcpy(out, in, sizeof(uint32_t) * rw);
  for (uint32_t t = 0; t < k; ++t) {
    orc_rlwe_rotate(c, out, e[t], rot);
    orc_cmux(c, C[t], rot, out, tmp);
    memcpy(out, tmp, sizeof(uint32_t) * rw);
  }
  free(rot);
  free(tmp);
}

/* CDEMUX(C, d) = (d - C [.] d, C [.] d)  (Sec. 3.3.1) */
void orc_cdemux(const orc_ctx* c, const uint32_t* C, const uint32_t* in, uint32_t* out0,
                uint32_t* out1) {
  size_t rw = rlwe_words(c);
  uint32_t* h = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  orc_extprod(c, C, in, h);
  rlwe_sub(c, in, h, out0);
  memcpy(out1, h, sizeof(uint32_t) * rw);
  free(h);
}

/* Inverse Vertical Packing (Alg. 5) on nb bits C[0..nb): nr = min(nb, log2 N)
 * rotation bits C[z..nb) with exponents +2^t, then the CDEMUX tree over
 * C[0..z), level i pairing L_j with L_{j+2^i}.  out receives 2^z RLWE; cell
 * m of the table sits at ciphertext m mod 2^z, coefficient m >> z.  The
 * algorithm's loop bound "0 to n" is read as j in [0, n). */
void orc_ivp(const orc_ctx* c, const uint32_t* const* C, uint32_t nb, const uint32_t* in,
             uint32_t* out) {
  size_t rw = rlwe_words(c);
  uint32_t nr = nb < c->logN ? nb : c->logN;
  uint32_t z = nb - nr;
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * (nr ? nr : 1));
  for (uint32_t t = 0; t < nr; ++t) e[t] = (int64_t)1 << t;
  orc_blind_rotate(c, in, C + z, e, nr, out);
  uint32_t* t0 = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  for (uint32_t i = 0; i < z; ++i) {
    uint32_t n = 1u << i;
    for (uint32_t j = 0; j < n; ++j) {
      orc_cdemux(c, C[i], out + j * rw, t0, out + (j + n) * rw);
      memcpy(out + j * rw, t0, sizeof(uint32_t) * rw);
    }
  }
  free(t0);
  free(e);
}

/* Node u of the CDEMUX tree (after the level that creates it) leads to a
 * cell of a class below l.  Index bits 0..L-1 are the label bits, so the
 * label of every leaf under u is congruent to u mod 2^min(level+1, L); with
 * z >= L the node is live iff (u mod 2^L) < l (for u < 2^L the smallest label
 * under it is u itself); with z < L every leaf receives some class < l,
 * because 2^z <= 2^(L-1) < l. */
static int node_live(uint32_t u, uint32_t z, uint32_t L, uint32_t l) {
  return z < L || (u & ((1u << L) - 1u)) < l;
}

/* IVP (Alg. 5) over the index [label bits (L), tuple bits] that creates only
 * the live tree nodes: a split of L_j whose new branch L_{j+2^i} is not live
 * is skipped, L_j keeping the undivided value (that branch would encrypt 0
 * for every index whose label is below l).  out: 2^z RLWE, the non-live
 * leaves left as zero.  This is the IVP behind the model of Definition 2,
 * whose rows hold only the ciphertexts of classes below l. */
void orc_ivp_pruned(const orc_ctx* c, const uint32_t* const* C, uint32_t nb, uint32_t l,
                    const uint32_t* in, uint32_t* out) {
  size_t rw = rlwe_words(c);
  uint32_t L = ceil_log2_u(l);
  uint32_t nr = nb < c->logN ? nb : c->logN;
  uint32_t z = nb - nr;
  memset(out, 0, sizeof(uint32_t) * rw * ((size_t)1 << z));
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * (nr ? nr : 1));
  for (uint32_t t = 0; t < nr; ++t) e[t] = (int64_t)1 << t;
  orc_blind_rotate(c, in, C + z, e, nr, out);
  uint32_t* t0 = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  for (uint32_t i = 0; i < z; ++i) {
    uint32_t n = 1u << i;
    for (uint32_t j = 0; j < n; ++j) {
      if (!node_live(j, z, L, l) || !node_live(j + n, z, L, l)) continue;
      orc_cdemux(c, C[i], out + j * rw, t0, out + (j + n) * rw);
      memcpy(out + j * rw, t0, sizeof(uint32_t) * rw);
    }
  }
  free(t0);
  free(e);
}

/* Row position of tree leaf d (z tree bits, L label bits) in the model of
 * Definition 2, or -1 for a leaf that holds no class below l.  With z >= L,
 * leaf d = c + 2^L w (class c < l, w < 2^(z-L)) goes to row w l + c, so a row
 * holds l 2^(z-L) = l 2^a / N ciphertexts; with z < L row d = leaf d. */
int32_t orc_leaf_row(uint32_t d, uint32_t z, uint32_t l) {
  uint32_t L = ceil_log2_u(l);
  if (z < L) return (int32_t)d;
  uint32_t cls = d & ((1u << L) - 1u);
  if (cls >= l) return -1;
  return (int32_t)((d >> L) * l + cls);
}

/* ExtractLWE(c, i) (Sec. 2.5.1): the LWE of coefficient i of c's phase under
 * the key's coefficients: a'_k = a_{i-k} for k <= i, a'_k = -a_{N+i-k} for
 * k > i (X^N = -1), b' = b_i */
void orc_extract_lwe(const orc_ctx* c, const uint32_t* in, uint32_t idx, uint32_t* lwe) {
  uint32_t N = c->N, nq = c->nq;
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    const uint32_t* a = in + (size_t)i * N;
    uint32_t* o = lwe + (size_t)i * (N + 1);
    for (uint32_t k = 0; k < N; ++k)
      o[k] = k <= idx ? a[idx - k] : (uint32_t)((q - a[N + idx - k]) % q);
    o[N] = in[((size_t)nq + i) * N + idx];
  }
}

/* ExtractLWE(c, 0): a'_0 = a_0, a'_k = -a_{N-k} (k >= 1), b' = b_0 */
void orc_extract_lwe0(const orc_ctx* c, const uint32_t* in, uint32_t* lwe) {
  uint32_t N = c->N, nq = c->nq;
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t q = c->q[i];
    const uint32_t* a = in + (size_t)i * N;
    uint32_t* o = lwe + (size_t)i * (N + 1);
    o[0] = a[0];
    for (uint32_t k = 1; k < N; ++k) o[k] = (uint32_t)((q - a[N - k]) % q);
    o[N] = in[((size_t)nq + i) * N];
  }
}

/* Vertical Packing (Alg. 3) of one LUT of 2^z RLWE under nb bits, where bit u
 * is either encrypted (C[u] != NULL) or the cleartext clear[u].  Levels run
 * from i = z-1 down to 0, level i pairing T[j] with T[j + 2^i] and taking
 * T[j + 2^i] when bit i is 1 (the inverse of the IVP layout; Alg. 3 as printed
 * pairs its bits in the opposite order, which is not the inverse of Alg. 5).
 * Then the blind rotation by X^{-2^t} over bits z..nb and ExtractLWE(., 0).
 * A cleartext bit is applied as the exact selection a noiseless RGSW of that
 * bit produces. */
static void vp_core(const orc_ctx* c, const uint32_t* const* C, const uint8_t* clear, uint32_t nb,
                    const uint32_t* lut, uint32_t* acc_out, uint32_t* lwe);

void orc_vp(const orc_ctx* c, const uint32_t* const* C, const uint8_t* clear, uint32_t nb,
            const uint32_t* lut, uint32_t* lwe) {
  vp_core(c, C, clear, nb, lut, NULL, lwe);
}

/* the same Vertical Packing, returning the rotated accumulator (RLWE)
 * before extraction */
void orc_vp_rlwe(const orc_ctx* c, const uint32_t* const* C, const uint8_t* clear, uint32_t nb,
                 const uint32_t* lut, uint32_t* acc_out) {
  vp_core(c, C, clear, nb, lut, acc_out, NULL);
}

static void vp_core(const orc_ctx* c, const uint32_t* const* C, const uint8_t* clear, uint32_t nb,
                    const uint32_t* lut, uint32_t* acc_out, uint32_t* lwe) {
  size_t rw = rlwe_words(c);
  uint32_t nr = nb < c->logN ? nb : c->logN;
  uint32_t z = nb - nr;
  uint32_t nt = 1u << z;
  uint32_t* T = (uint32_t*)malloc(sizeof(uint32_t) * rw * nt);
  uint32_t* rot = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  memcpy(T, lut, sizeof(uint32_t) * rw * nt);
  for (int i = (int)z - 1; i >= 0; --i) {
    uint32_t n = 1u << i;
    for (uint32_t j = 0; j < n; ++j) {
      uint32_t* lo = T + j * rw;
      uint32_t* hi = T + (j + n) * rw;
      if (C[i]) {
        orc_cmux(c, C[i], hi, lo, tmp);
        memcpy(lo, tmp, sizeof(uint32_t) * rw);
      } else if (clear[i]) {
        memcpy(lo, hi, sizeof(uint32_t) * rw);
      }
    }
  }
  uint32_t* acc = T;
  for (uint32_t t = 0; t < nr; ++t) {
    uint32_t u = z + t;
    int64_t e = -((int64_t)1 << t);
    if (C[u]) {
      orc_rlwe_rotate(c, acc, e, rot);
      orc_cmux(c, C[u], rot, acc, tmp);
      memcpy(acc, tmp, sizeof(uint32_t) * rw);
    } else if (clear[u]) {
      orc_rlwe_rotate(c, acc, e, rot);
      memcpy(acc, rot, sizeof(uint32_t) * rw);
    }
  }
  if (lwe) orc_extract_lwe0(c, acc, lwe);
  if (acc_out) memcpy(acc_out, acc, sizeof(uint32_t) * rw);
  free(T);
  free(rot);
  free(tmp);
}

/* ------------------------------------------------------------------------ */
/* WiSARD layer (Def. 1-2, Alg. 6, Alg. 7)                                   */
/* ------------------------------------------------------------------------ */

/* pi_r: Fisher-Yates over [0, s): for k = s-1 down to 1, j = w64(seed, PERM,
 * s-1-k) mod (k+1), swap(pi[k], pi[j]).  The permuted input is t[k] =
 * x[pi[k]].  The paper leaves the permutation's generator unspecified. */
void orc_permutation(uint64_t seed, uint32_t s, uint32_t* pi) {
  for (uint32_t k = 0; k < s; ++k) pi[k] = k;
  for (int64_t k = (int64_t)s - 1; k >= 1; --k) {
    uint32_t j = (uint32_t)(orc_w64(seed, DOM_PERM, (uint64_t)((int64_t)s - 1 - k)) % (uint64_t)(k + 1));
    uint32_t t = pi[k];
    pi[k] = pi[j];
    pi[j] = t;
  }
}

/* geometry of RAM j: a_j tuple bits, nb = L + a_j, z = nb - min(nb, log2 N) */
static void ram_geometry(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, uint32_t j,
                         uint32_t* aj, uint32_t* nb, uint32_t* z) {
  uint32_t L = ceil_log2_u(l);
  uint32_t rem = s - j * a;
  *aj = rem < a ? rem : a;
  *nb = L + *aj;
  uint32_t nr = *nb < c->logN ? *nb : c->logN;
  *z = *nb - nr;
}

/* rows of RAM row of H for a RAM with z tree bits: the live leaves */
static uint32_t live_leaves(uint32_t z, uint32_t l) {
  uint32_t L = ceil_log2_u(l);
  return z >= L ? l << (z - L) : 1u << z;
}

/* k1 of Definition 2, ceil(l 2^a / N): the live leaves of a full RAM, l
 * 2^(z-L) when z >= L (equal to the printed value); when z < L the IVP
 * layout needs all 2^z (the printed value then undercounts). */
uint32_t orc_k1(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a) {
  uint32_t aj, nb, z;
  ram_geometry(c, s, l, a, 0, &aj, &nb, &z);
  (void)aj;
  (void)nb;
  return live_leaves(z, l);
}

/* Class-packed layout (the horizontal packing the paper lists among its
 * further improvements: one evaluation serves the RAMs of every
 * discriminator).  The IVP index is [tuple bits, label bits] with the label
 * bits on top, so cell (c, addr) of RAM j is m = addr + 2^a_j c: tree leaf
 * m mod 2^z, coefficient (addr >> z) + c 2^(a_j - z).  A row holds all 2^z
 * leaves, each with every class of its cells; one VP over the tuple bits
 * brings the cells of all classes to coefficients c 2^(a_j - z). */
uint32_t orc_k1_layout(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, uint32_t layout) {
  if (layout == 0) return orc_k1(c, s, l, a);
  /* layouts 1 and 2: every tree leaf.  They need the tree to hold tuple bits
   * only, z <= a_j, i.e. L <= log2 N; 0 marks the shape as invalid for them */
  if (ceil_log2_u(l) > c->logN) return 0;
  uint32_t aj, nb, z;
  ram_geometry(c, s, l, a, 0, &aj, &nb, &z);
  (void)aj;
  (void)nb;
  return 1u << z;
}

/* Several small RAMs per RLWE (layout 2, the other half of horizontal
 * packing): with nb = L + a index bits and 2^nb < N, r = N / 2^nb RAMs share
 * a model row, RAM j at coefficient offset (j mod r) 2^nb of row j / r.
 * Built from the class-packed rows H1 (one RLWE per RAM, since z = 0) as
 * row R = sum_t X^(t 2^nb) H1[R r + t] over the RAMs of the row.  Rotation
 * by a monomial and addition are exact, so the packed rows of a model
 * trained sample by sample equal the packed rows of its sum. */
uint32_t orc_rams_per_row(const orc_ctx* c, uint32_t l, uint32_t a) {
  uint32_t nb = ceil_log2_u(l) + a;
  return nb < c->logN ? 1u << (c->logN - nb) : 1u;
}

uint32_t orc_model_rows(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, uint32_t layout) {
  uint32_t k0 = (s + a - 1) / a;
  if (layout != 2) return k0;
  uint32_t r = orc_rams_per_row(c, l, a);
  return (k0 + r - 1) / r;
}

void orc_pack_rams(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, const uint32_t* H1, uint32_t* Hp) {
  size_t rw = rlwe_words(c);
  uint32_t k0 = (s + a - 1) / a;
  uint32_t k1 = orc_k1_layout(c, s, l, a, 1);
  uint32_t r = orc_rams_per_row(c, l, a);
  uint32_t rows = orc_model_rows(c, s, l, a, 2);
  int64_t stride = (int64_t)1 << (ceil_log2_u(l) + a);
  if (r == 1) {
    memcpy(Hp, H1, sizeof(uint32_t) * rw * k1 * k0);
    return;
  }
  uint32_t* rot = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  for (uint32_t R = 0; R < rows; ++R) {
    uint32_t* dst = Hp + (size_t)R * rw;
    memset(dst, 0, sizeof(uint32_t) * rw);
    for (uint32_t t = 0; t < r && R * r + t < k0; ++t) {
      orc_rlwe_rotate(c, H1 + (size_t)(R * r + t) * rw, (int64_t)t * stride, rot);
      rlwe_add(c, dst, rot, dst);
    }
  }
  free(rot);
}

/* Homomorphic training (Alg. 6) restricted to RAMs [ram_lo, ram_hi):
 * for each sample i in order and each RAM j: b = [Y_i bits 0..L), X_i[pi[j a
 * + t]] for t < a_j]; h = IVP(b, (0, Delta)) with the live tree nodes only;
 * H[j][row(d)] += h[d] for every live leaf d.  The input of the IVP, "(0,1)"
 * in the paper, is read as the trivial RLWE (0, Delta).  The tuple of RAM j
 * is t_{ja} .. t_{ja+a-1} (the printed t_j .. t_{j+a-1} overlaps tuples).
 * x_ptr[i*s + k] points at the RGSW of input bit k of sample i, y_ptr[i*L +
 * u] at label bit u (LSB first); H is [k0][k1] RLWE. */
void orc_train(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, const uint32_t* pi,
               const uint32_t* const* x_ptr, const uint32_t* const* y_ptr, uint64_t n,
               uint32_t ram_lo, uint32_t ram_hi, uint32_t layout, uint32_t* H) {
  size_t rw = rlwe_words(c);
  uint32_t L = ceil_log2_u(l);
  uint32_t k1 = orc_k1_layout(c, s, l, a, layout);
  const uint32_t** bits = (const uint32_t**)malloc(sizeof(uint32_t*) * (L + a + 1));
  uint32_t* in = (uint32_t*)calloc(rw, sizeof(uint32_t));
  uint32_t aj0, nb0, z0;
  ram_geometry(c, s, l, a, 0, &aj0, &nb0, &z0);
  uint32_t* h = (uint32_t*)malloc(sizeof(uint32_t) * rw * ((size_t)1 << z0));
  for (uint32_t i = 0; i < c->nq; ++i) in[((size_t)c->nq + i) * c->N] = (uint32_t)c->delta_mod[i];
  for (uint64_t smp = 0; smp < n; ++smp) {
    for (uint32_t j = ram_lo; j < ram_hi; ++j) {
      uint32_t aj, nb, z;
      ram_geometry(c, s, l, a, j, &aj, &nb, &z);
      if (layout == 0) {
        for (uint32_t u = 0; u < L; ++u) bits[u] = y_ptr[smp * L + u];
        for (uint32_t t = 0; t < aj; ++t) bits[L + t] = x_ptr[smp * s + pi[j * a + t]];
        orc_ivp_pruned(c, bits, nb, l, in, h);
      } else {  /* class-packed: [tuple bits, label bits], every leaf kept */
        for (uint32_t t = 0; t < aj; ++t) bits[t] = x_ptr[smp * s + pi[j * a + t]];
        for (uint32_t u = 0; u < L; ++u) bits[aj + u] = y_ptr[smp * L + u];
        orc_ivp(c, bits, nb, in, h);
      }
      for (uint32_t d = 0; d < (1u << z); ++d) {
        int32_t row = layout == 0 ? orc_leaf_row(d, z, l) : (int32_t)d;
        if (row < 0) continue;
        uint32_t* dst = H + ((size_t)j * k1 + (uint32_t)row) * rw;
        rlwe_add(c, dst, h + (size_t)d * rw, dst);
      }
    }
  }
  free(bits);
  free(in);
  free(h);
}

/* class counter for balancing (Sec. 3.7.1): cnt += BlindRotate((0, Delta),
 * Y_i bits, +2^u) for every sample, i.e. Delta at coefficient y_i */
void orc_class_count(const orc_ctx* c, uint32_t l, const uint32_t* const* y_ptr, uint64_t n,
                     uint32_t* cnt) {
  size_t rw = rlwe_words(c);
  uint32_t L = ceil_log2_u(l);
  uint32_t* in = (uint32_t*)calloc(rw, sizeof(uint32_t));
  uint32_t* h = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * (L ? L : 1));
  for (uint32_t i = 0; i < c->nq; ++i) in[((size_t)c->nq + i) * c->N] = (uint32_t)c->delta_mod[i];
  for (uint32_t u = 0; u < L; ++u) e[u] = (int64_t)1 << u;
  for (uint64_t smp = 0; smp < n; ++smp) {
    orc_blind_rotate(c, in, y_ptr + smp * L, e, L, h);
    rlwe_add(c, cnt, h, cnt);
  }
  free(in);
  free(h);
  free(e);
}

/* Homomorphic inference, PD-act branch (Alg. 7) for one sample, RAM j and
 * label c: b = [bits of c (cleartext), X[pi[j a + t]]], u = VP(b, H[j]) over
 * the row's leaves in tree order.
 * x_ptr[k] points at the RGSW of input bit k of the sample. */
void orc_infer_one(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, const uint32_t* pi,
                   const uint32_t* H, const uint32_t* const* x_ptr, uint32_t j, uint32_t label,
                   uint32_t* lwe) {
  size_t rw = rlwe_words(c);
  uint32_t L = ceil_log2_u(l);
  uint32_t k1 = orc_k1(c, s, l, a);
  uint32_t aj, nb, z;
  ram_geometry(c, s, l, a, j, &aj, &nb, &z);
  const uint32_t** bits = (const uint32_t**)calloc(nb + 1, sizeof(uint32_t*));
  uint8_t* clear = (uint8_t*)calloc(nb + 1, 1);
  for (uint32_t u = 0; u < L; ++u) clear[u] = (uint8_t)((label >> u) & 1u);
  for (uint32_t t = 0; t < aj; ++t) bits[L + t] = x_ptr[pi[j * a + t]];
  /* the row's live leaves in tree order; a leaf of no class below l is zero
   * (the clear label bits never select it) */
  uint32_t* lut = (uint32_t*)calloc(rw * ((size_t)1 << z), sizeof(uint32_t));
  for (uint32_t d = 0; d < (1u << z); ++d) {
    int32_t row = orc_leaf_row(d, z, l);
    if (row >= 0) memcpy(lut + (size_t)d * rw, H + ((size_t)j * k1 + (uint32_t)row) * rw, sizeof(uint32_t) * rw);
  }
  orc_vp(c, bits, clear, nb, lut, lwe);
  free(lut);
  free(bits);
  free(clear);
}

/* Homomorphic inference over the class-packed layout: for one sample and
 * RAM j, one VP over the tuple bits (encrypted) of row H[j] with the label
 * bits left out; the cell of class c then sits at coefficient c 2^(a_j - z)
 * and out[c] = ExtractLWE(acc, c 2^(a_j - z)) for c < l (the scores Alg. 7
 * computes per label, all from one evaluation).  out: [l] LWE. */
void orc_infer_packed(const orc_ctx* c, uint32_t s, uint32_t l, uint32_t a, const uint32_t* pi,
                      const uint32_t* H, const uint32_t* const* x_ptr, uint32_t j, uint32_t layout,
                      uint32_t* out) {
  size_t rw = rlwe_words(c);
  uint32_t k1 = orc_k1_layout(c, s, l, a, 1);
  if (k1 == 0) return; /* L > log2 N: no class-packed layout (the wrapper rejects it first) */
  /* layout 2: RAM j is the (j mod r)-th block of 2^(L + a) coefficients of
   * row j / r; the VP's rotations move only within it */
  uint32_t r = layout == 2 ? orc_rams_per_row(c, l, a) : 1u;
  uint32_t row = j / r;
  uint32_t off = (j % r) << (ceil_log2_u(l) + a);
  uint32_t aj, nb, z;
  ram_geometry(c, s, l, a, j, &aj, &nb, &z);
  /* the VP over all nb index bits with the label bits as cleartext zeros: z
   * <= a_j (L <= log2 N), so the tree takes tuple bits only and the label
   * bits leave the accumulator where the tuple bits put it */
  const uint32_t** bits = (const uint32_t**)calloc(nb + 1, sizeof(uint32_t*));
  uint8_t* clear = (uint8_t*)calloc(nb + 1, 1);
  for (uint32_t t = 0; t < aj; ++t) bits[t] = x_ptr[pi[j * a + t]];
  uint32_t* acc = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  orc_vp_rlwe(c, bits, clear, nb, H + (size_t)row * k1 * rw, acc);
  uint32_t stride = 1u << (aj - z);
  for (uint32_t cl = 0; cl < l; ++cl)
    orc_extract_lwe(c, acc, off + cl * stride, out + (size_t)cl * c->nq * (c->N + 1));
  free(acc);
  free(bits);
  free(clear);
}

/* Merge of Integer WiSARD models trained apart (Sec. 3.7.2: the federated
 * entities' models are merged by adding their RAMs): out = x + y for count
 * RLWE ciphertexts (model rows or class counters), residue by residue */
void orc_rlwe_add_n(const orc_ctx* c, const uint32_t* x, const uint32_t* y, uint64_t count, uint32_t* out) {
  size_t rw = rlwe_words(c);
  for (uint64_t k = 0; k < count; ++k) rlwe_add(c, x + k * rw, y + k * rw, out + k * rw);
}

/* LWE addition, used for the per-class sums u_c = sum_j u[c][j] */
void orc_lwe_add(const orc_ctx* c, const uint32_t* x, const uint32_t* y, uint32_t* out) {
  for (uint32_t i = 0; i < c->nq; ++i)
    for (uint32_t k = 0; k <= c->N; ++k) {
      size_t o = (size_t)i * (c->N + 1) + k;
      out[o] = (uint32_t)addmod(x[o], y[o], c->q[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* PackingKeySwitching (Sec. 2.5.1; the PD-act return value of Alg. 7)        */
/* ------------------------------------------------------------------------ */
/* k LWE ciphertexts (a^(i), b^(i)), phase_i = b^(i) - sum_j a^(i)_j s_j under
 * the RLWE key's coefficients (the key ExtractLWE leaves them under), become
 * one RLWE whose phase is sum_i phase_i X^i (plus key-switching noise).
 * Key: K[j][r] = RLWE_s(s_j G_r) for j < N and the RNS gadget rows r < D
 * (G_r = base^t in residue g for r = g digits + t, 0 in the others), each a
 * row drawn like an RGSW row (seed, ciphertext j, D rows, a by its
 * evaluations).  Packing: with P_{j,r}(X) = sum_i d_r(a^(i)_j) X^i (d_r: the
 * balanced digit of the external product's decomposition),
 *   out = (0, sum_i b^(i) X^i) - sum_{j,r} P_{j,r} K[j][r],
 * whose phase is sum_i X^i (b^(i) - sum_j (sum_r d_r(a^(i)_j) G_r) s_j). */

/* the balanced base-2^log_base digits of one centered residue (as orc_decompose) */
static void value_digits(const orc_ctx* c, int64_t v, int64_t q, int32_t* d) {
  int64_t B = 1ll << c->log_base;
  if (v > (q - 1) / 2) v -= q;
  for (uint32_t t = 0; t + 1 < c->digits; ++t) {
    int64_t x = ((v % B) + B) % B;
    if (x >= B / 2) x -= B;
    d[t] = (int32_t)x;
    v = (v - x) / B;
  }
  d[c->digits - 1] = (int32_t)v;
}

/* rows j_lo <= j < j_hi of the key (K holds all N x D rows) */
void orc_pks_keygen(const orc_ctx* c, const int32_t* s, uint64_t seed, uint32_t j_lo, uint32_t j_hi, uint32_t* K) {
  uint32_t N = c->N, nq = c->nq, D = c->D;
  size_t rw = rlwe_words(c);
  for (uint32_t j = j_lo; j < j_hi; ++j)
    for (uint32_t r = 0; r < D; ++r) {
      uint32_t* row = K + ((size_t)j * D + r) * rw;
      enc_row(c, s, NULL, seed, j, D, r, 1, row);
      uint32_t g = r / c->digits, t = r % c->digits;
      uint64_t q = c->q[g];
      uint64_t G = powmod(1ull << c->log_base, t, q);
      uint64_t m = s[j] == 0 ? 0 : (s[j] > 0 ? G : q - G);
      uint32_t* b0 = row + ((size_t)nq + g) * N;
      b0[0] = (uint32_t)addmod(b0[0], m, q);
    }
}

/* acc (+)= sum_{j in [j_lo, j_hi), r} P_{j,r} K[j][r]; lwe: [k][nq][N+1] */
void orc_pks_partial(const orc_ctx* c, const uint32_t* K, const uint32_t* lwe, uint32_t k, uint32_t j_lo,
                     uint32_t j_hi, uint32_t* acc) {
  uint32_t N = c->N, nq = c->nq, D = c->D;
  size_t rw = rlwe_words(c);
  int32_t* P = (int32_t*)calloc((size_t)c->digits * N, sizeof(int32_t));
  int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * c->digits);
  for (uint32_t j = j_lo; j < j_hi; ++j)
    for (uint32_t g = 0; g < nq; ++g) {
      for (uint32_t i = 0; i < k; ++i) {
        value_digits(c, lwe[((size_t)i * nq + g) * (N + 1) + j], (int64_t)c->q[g], dg);
        for (uint32_t t = 0; t < c->digits; ++t) P[(size_t)t * N + i] = dg[t];
      }
      for (uint32_t t = 0; t < c->digits; ++t) {
        const uint32_t* row = K + ((size_t)j * D + g * c->digits + t) * rw;
        for (uint32_t part = 0; part < 2; ++part)
          for (uint32_t ip = 0; ip < nq; ++ip)
            mul_acc_small(c, ip, P + (size_t)t * N, row + ((size_t)part * nq + ip) * N,
                          acc + ((size_t)part * nq + ip) * N);
      }
    }
  free(P);
  free(dg);
}

/* out = (0, sum_i b^(i) X^i) - acc */
void orc_pks_finish(const orc_ctx* c, const uint32_t* lwe, uint32_t k, const uint32_t* acc, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq;
  for (uint32_t ip = 0; ip < nq; ++ip) {
    uint64_t q = c->q[ip];
    for (uint32_t x = 0; x < N; ++x) {
      uint64_t b = x < k ? lwe[((size_t)x * nq + ip) * (N + 1) + N] : 0;
      out[(size_t)ip * N + x] = (uint32_t)submod(0, acc[(size_t)ip * N + x], q);
      out[((size_t)nq + ip) * N + x] = (uint32_t)submod(b, acc[((size_t)nq + ip) * N + x], q);
    }
  }
}

/* exported sizes for the Python wrapper */
/* ------------------------------------------------------------------------ */
/* programmable bootstrapping of LWE ciphertexts (Sec. 2.5.3, Sec. 3.5.2)    */
/* ------------------------------------------------------------------------ */

/* Modulus switch Q -> 2N of an LWE ciphertext [prime][N+1] whose mask is
 * zero past its first n coefficients: each a_k (k < n) and the body b, read
 * as integers in [0, Q) through the CRT, becomes round(2N x / Q) mod 2N,
 * i.e. floor((2N x + floor(Q/2)) / Q) mod 2N (Q is odd, so no value rounds
 * from exactly one half).  out[0..n) = the mask, out[n] = the body. */
void orc_modswitch(const orc_ctx* c, const uint32_t* lwe, uint32_t n, int64_t* out) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t x[ORC_MAXQ];
  for (uint32_t k = 0; k <= n; ++k) {
    uint32_t idx = k < n ? k : N;
    for (uint32_t i = 0; i < nq; ++i) x[i] = lwe[(size_t)i * (N + 1) + idx];
    u128 v = crt(c, x);
    u128 r = (v * (u128)(2 * N) + c->Q / 2) / c->Q;
    out[k] = (int64_t)(r % (2 * N));
  }
}

/* Programmable bootstrap with a constant test polynomial V (v[i] = V mod
 * q_i) of an LWE ciphertext whose mask is zero past its first n
 * coefficients, with the bootstrapping key bsk[2k] = RGSW([s_k = 1]),
 * bsk[2k+1] = RGSW([s_k = -1]) (k < n, RGSW under the ring key s):
 *   (a~, b~) = modulus switch to 2N;
 *   ACC = the trivial RLWE (0, X^{-b~} TV), TV = V (1 + X + ... + X^{N-1});
 *   for k < n: ACC <- CMUX(bsk[2k], X^{a~_k} ACC, ACC),
 *              ACC <- CMUX(bsk[2k+1], X^{-a~_k} ACC, ACC)
 *     (at most one of the two bits is 1, so the pair multiplies ACC by
 *      X^{a~_k s_k}), which leaves ACC encrypting X^{-phi~} TV with
 *      phi~ = b~ - sum_k a~_k s_k mod 2N;
 *   out = ExtractLWE(ACC, 0): coefficient 0 of X^{-phi~} TV is TV[phi~] = V
 *     when phi~ < N and -TV[phi~ - N] = -V otherwise (X^N = -1), plus the
 *     noise of 2n external products. */
void orc_pbs(const orc_ctx* c, const uint32_t* const* bsk, const uint32_t* lwe, uint32_t n, const uint64_t* v,
             uint32_t* out) {
  uint32_t N = c->N, nq = c->nq;
  size_t rw = rlwe_words(c);
  int64_t* ms = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  int64_t* ex = (int64_t*)malloc(sizeof(int64_t) * (2 * (size_t)n + 1));
  uint32_t* acc = (uint32_t*)calloc(rw, sizeof(uint32_t));
  uint32_t* res = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  orc_modswitch(c, lwe, n, ms);
  /* the test polynomial TV = V (1 + X + ... + X^{N-1}), rotated by X^{-b~} */
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t vi = v[i] % c->q[i];
    uint32_t* b = res + ((size_t)nq + i) * N;
    memset(res + (size_t)i * N, 0, sizeof(uint32_t) * N);
    for (uint32_t j = 0; j < N; ++j) b[j] = (uint32_t)vi;
  }
  orc_rlwe_rotate(c, res, -ms[n], acc);
  for (uint32_t k = 0; k < n; ++k) {
    ex[2 * k] = ms[k];
    ex[2 * k + 1] = -ms[k];
  }
  orc_blind_rotate(c, acc, bsk, ex, 2 * n, res);
  orc_extract_lwe0(c, res, out);
  free(ms);
  free(ex);
  free(acc);
  free(res);
}

uint64_t orc_rlwe_words(const orc_ctx* c) { return rlwe_words(c); }
uint64_t orc_rgsw_words(const orc_ctx* c) { return rgsw_words(c); }
uint32_t orc_logN(const orc_ctx* c) { return c->logN; }

/* ------------------------------------------------------------------------ */
/* bootstrapping through a key switch to a binary LWE key (Sec. 2.5.3: the  */
/* TFHE setting keeps an LWE key in B^n beside the ring key)                 */
/* ------------------------------------------------------------------------ */

/* The key switch works at modulus 2^32 with a gadget of KS_DIGITS balanced
 * digits of KS_LOG_BASE bits taken from the top of each coefficient; the
 * key-switching key's errors are 2^13 c + u, c a discrete Gaussian sample of
 * the context's table, u uniform in [-2^12, 2^12).  These parameters are
 * this implementation's (the paper leaves the bootstrap to other work). */
#define DOM_LWE_KEY 7u
#define DOM_KSK_A 8u
#define DOM_KSK_E 9u
#define KS_LOG_BASE 4
#define KS_DIGITS 6

/* s1_i = bit 0 of w64(seed, LWE_KEY, i), i < n */
void orc_lwe_keygen(uint64_t seed, uint32_t n, uint8_t* s1) {
  for (uint32_t i = 0; i < n; ++i) s1[i] = (uint8_t)(orc_w64(seed, DOM_LWE_KEY, i) & 1u);
}

/* round(2^32 x / Q) mod 2^32 (half up) of the integer x in [0, Q) whose
 * residues are r */
static uint32_t switch_2_32(const orc_ctx* c, const uint64_t* r) {
  u128 v = crt(c, r);
  u128 w = ((v << 32) + c->Q / 2) / c->Q;
  return (uint32_t)w;
}

/* Balanced base-16 digits of the top 24 bits of a (rounded): t = round(a /
 * 2^8) mod 2^24, then from the lowest digit up d = (t mod 16) + carry,
 * d >= 8 -> d - 16 with a carry of 1; the carry out of the top digit is
 * dropped (weight 2^32).  a = sum_j d_j 2^(28 - 4j) + (a - 2^8 t) mod 2^32,
 * d_j in [-8, 8). */
static void ks_digits(uint32_t a, int32_t* d) {
  uint32_t t = (uint32_t)((((uint64_t)a + 128u) >> 8) & 0xFFFFFFu);
  int32_t carry = 0;
  for (int j = KS_DIGITS - 1; j >= 0; --j) {
    int32_t x = (int32_t)(t & 15u) + carry;
    t >>= 4;
    if (x >= 8) {
      x -= 16;
      carry = 1;
    } else {
      carry = 0;
    }
    d[j] = x;
  }
}

/* Key-switching key rows r = k KS_DIGITS + j for k in [k_lo, k_hi): an LWE
 * under s1 at modulus 2^32 of s_k 2^(28 - 4j):
 *   A_r[i] = w32(seed, KSK_A, r n + i),
 *   e_r = 2^13 cdt(w64(seed, KSK_E, 2r)) + (w64(seed, KSK_E, 2r + 1) >> 51) - 2^12,
 *   B_r = sum_i A_r[i] s1_i + e_r + s_k 2^(28 - 4j)  mod 2^32.
 * ksk: [N KS_DIGITS][n + 1] (A_r, then B_r). */
void orc_ksk_gen(const orc_ctx* c, const int32_t* s, const uint8_t* s1, uint32_t n, uint64_t seed,
                 uint32_t k_lo, uint32_t k_hi, uint32_t* ksk) {
  for (uint32_t k = k_lo; k < k_hi; ++k)
    for (uint32_t j = 0; j < KS_DIGITS; ++j) {
      uint64_t r = (uint64_t)k * KS_DIGITS + j;
      uint32_t* row = ksk + r * (n + 1);
      uint32_t b = 0;
      for (uint32_t i = 0; i < n; ++i) {
        uint32_t a = orc_w32(seed, DOM_KSK_A, r * n + i);
        row[i] = a;
        if (s1[i]) b += a;
      }
      int64_t e = orc_cdt_sample(c->cdt, orc_w64(seed, DOM_KSK_E, 2 * r)) * 8192 +
                  (int64_t)(orc_w64(seed, DOM_KSK_E, 2 * r + 1) >> 51) - 4096;
      b += (uint32_t)e;
      b += (uint32_t)((int64_t)s[k] * ((int64_t)1 << (28 - 4 * j)));
      row[n] = b;
    }
}

/* Key switch of an LWE ciphertext under the ring key (modulus Q, mask
 * length N) to s1 at modulus 2^32: every mask coefficient and the body
 * switched to 2^32 (round(2^32 x / Q)), then
 *   out = (0, b') - sum_k sum_j d_j(a'_k) KSK[k KS_DIGITS + j]  mod 2^32,
 * so that out decrypts under s1 to the switched phase of the input plus the
 * rounding of the digits and the key's errors times the digits. */
void orc_key_switch(const orc_ctx* c, const uint32_t* ksk, uint32_t n, const uint32_t* lwe, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq;
  uint64_t x[ORC_MAXQ];
  int32_t d[KS_DIGITS];
  for (uint32_t i = 0; i < nq; ++i) x[i] = lwe[(size_t)i * (N + 1) + N];
  memset(out, 0, sizeof(uint32_t) * (n + 1));
  out[n] = switch_2_32(c, x);
  for (uint32_t k = 0; k < N; ++k) {
    for (uint32_t i = 0; i < nq; ++i) x[i] = lwe[(size_t)i * (N + 1) + k];
    ks_digits(switch_2_32(c, x), d);
    for (uint32_t j = 0; j < KS_DIGITS; ++j) {
      if (!d[j]) continue;
      const uint32_t* row = ksk + ((size_t)k * KS_DIGITS + j) * (n + 1);
      for (uint32_t i = 0; i <= n; ++i) out[i] -= (uint32_t)d[j] * row[i];
    }
  }
}

/* Programmable bootstrap through the key switch: ks = orc_key_switch(lwe);
 * (a~, b~) = round(2N ks / 2^32) mod 2N; ACC = (0, X^{-b~} TV) with
 * TV = V (1 + X + ... + X^{N-1}); for i < n: ACC <- CMUX(bsk[i],
 * X^{a~_i} ACC, ACC) with bsk[i] = RGSW(s1_i) under the ring key, which
 * multiplies ACC by X^{a~_i s1_i}; out = ExtractLWE(ACC, 0): V when the
 * switched phase b~ - sum_i a~_i s1_i mod 2N lies in [0, N), -V otherwise. */
void orc_pbs_ks(const orc_ctx* c, const uint32_t* const* bsk, const uint32_t* ksk, uint32_t n,
                const uint32_t* lwe, const uint64_t* v, uint32_t* out) {
  uint32_t N = c->N, nq = c->nq;
  size_t rw = rlwe_words(c);
  uint32_t* ks = (uint32_t*)malloc(sizeof(uint32_t) * (n + 1));
  int64_t* ex = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  uint32_t* acc = (uint32_t*)calloc(rw, sizeof(uint32_t));
  uint32_t* res = (uint32_t*)malloc(sizeof(uint32_t) * rw);
  orc_key_switch(c, ksk, n, lwe, ks);
  const uint32_t sh = 32 - (c->logN + 1);
  for (uint32_t i = 0; i <= n; ++i)
    ex[i] = (int64_t)((((uint64_t)ks[i] + ((uint64_t)1 << (sh - 1))) >> sh) % (2 * (uint64_t)N));
  for (uint32_t i = 0; i < nq; ++i) {
    uint64_t vi = v[i] % c->q[i];
    uint32_t* b = res + ((size_t)nq + i) * N;
    memset(res + (size_t)i * N, 0, sizeof(uint32_t) * N);
    for (uint32_t j = 0; j < N; ++j) b[j] = (uint32_t)vi;
  }
  orc_rlwe_rotate(c, res, -ex[n], acc);
  orc_blind_rotate(c, acc, bsk, ex, n, res);
  orc_extract_lwe0(c, res, out);
  free(ks);
  free(ex);
  free(acc);
  free(res);
}
