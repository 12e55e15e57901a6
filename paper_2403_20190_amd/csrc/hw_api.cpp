// hw_api.cpp -- host side of the C ABI in include/hwisard.h: parameter
// derivation (primes, roots of unity, NTT twiddles, Delta, CRT constants,
// Gaussian table), argument checks, workspace management and the
// orchestration of the kernels in hw_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hwisard.h"
#include "hw_ctx.h"
#include "hw_internal.h"


// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

hw_status fail(hw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

hw_status ok() {
  g_err.clear();
  return HW_OK;
}


extern "C" const char* hw_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// number theory on the host
// ---------------------------------------------------------------------------

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

static uint64_t powm(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  for (; e; e >>= 1, b = mulm(b, b, m))
    if (e & 1) r = mulm(r, b, m);
  return r;
}

// deterministic Miller-Rabin for n < 2^32 (witnesses 2, 7, 61)
static bool is_prime32(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 61ull})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int r = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++r;
  }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    uint64_t x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; ++i) {
      x = mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1u);
  return r;
}

// Shoup companion floor(w * 2^32 / q)
static uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

// ---------------------------------------------------------------------------
// Philox4x32-10 on the host (for the permutation) and the Gaussian table
// ---------------------------------------------------------------------------

static void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1, n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

static uint64_t draw64(uint64_t seed, uint32_t domain, uint64_t index) {
  const uint64_t blk = index >> 1;
  uint32_t c[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), domain, 0u};
  philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return (index & 1) ? ((uint64_t)c[2] | ((uint64_t)c[3] << 32)) : ((uint64_t)c[0] | ((uint64_t)c[1] << 32));
}

uint64_t lib_draw64(uint64_t seed, uint32_t domain, uint64_t index) { return draw64(seed, domain, index); }

// T[k] = floor(2^63 P(|X| <= k)), X ~ discrete Gaussian(sigma) cut at 41; the
// cumulative weights 1, 2 rho(1), 2 rho(2), ... are summed in increasing order
static void build_cdt(double sigma, uint64_t T[42]) {
  double cum[42], acc = 0.0;
  for (int x = 0; x < 42; ++x) {
    const double w = x == 0 ? 1.0 : 2.0 * std::exp(-((double)x * (double)x) / (2.0 * sigma * sigma));
    acc = acc + w;
    cum[x] = acc;
  }
  for (int x = 0; x < 41; ++x) T[x] = (uint64_t)std::floor(std::ldexp(cum[x] / cum[41], 63));
  T[41] = 1ull << 63;
}

// The guide of the CDT search (hw::Cdt::guide): entry b counts the T[j]
// (j <= 40) at or below the first draw of bucket b, plus CDT_GUIDE_WIDE when
// more than two T[j] fall inside the bucket, where two comparisons from that
// count would not finish the search.
static void build_cdt_guide(const uint64_t T[42], uint8_t G[hw::CDT_GUIDE_SIZE]) {
  const int sh = 63 - (int)hw::CDT_GUIDE_BITS;
  for (uint32_t b = 0; b < hw::CDT_GUIDE_SIZE; ++b) {
    const uint64_t lo = (uint64_t)b << sh, hi = lo + ((1ull << sh) - 1);
    uint32_t below = 0, inside = 0;
    for (int j = 0; j <= 40; ++j) {
      if (T[j] <= lo)
        ++below;
      else if (T[j] <= hi)
        ++inside;
    }
    G[b] = (uint8_t)(below | (inside > 2 ? hw::CDT_GUIDE_WIDE : 0u));
  }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------


extern "C" hw_status hw_ctx_create(const hw_params* params, int device, hw_ctx** out) {
  if (!params || !out) return fail(HW_EINVAL, "null argument");
  *out = nullptr;
  hw_params P = *params;
  int logN = 0;
  while ((1u << logN) < P.N) ++logN;
  if ((1u << logN) != P.N || logN < 10 || logN > 12)
    return fail(HW_EUNSUPPORTED, "N = %u: supported ring degrees are 1024, 2048, 4096", P.N);
  if (P.nq < 1 || P.nq > 3) return fail(HW_EUNSUPPORTED, "nq = %u: 1..3 primes supported", P.nq);
  if (!(P.log_base == 6 && P.digits == 5) && !(P.log_base == 15 && P.digits == 2 && P.nq >= 2))
    return fail(HW_EUNSUPPORTED,
                "gadget base 2^%u with %u digits: the kernels are built for base 2^6 with 5 digits, and for base "
                "2^15 with 2 digits on rings of two or more primes", P.log_base, P.digits);
  if (!(P.sigma > 0.0 && P.sigma < 16.0)) return fail(HW_EINVAL, "sigma = %g out of range (0, 16)", P.sigma);
  if (P.plain_mod < 2 || P.plain_mod > (1ull << 20) || (P.plain_mod & (P.plain_mod - 1)))
    return fail(HW_EINVAL, "plain_mod = %llu: a power of two in [2, 2^20] is required",
                (unsigned long long)P.plain_mod);
  const uint64_t m = 2ull * P.N;
  if (P.primes[0] == 0) {
    uint64_t q = ((((1ull << 30) - 2)) / m) * m + 1;
    uint32_t found = 0;
    for (; found < P.nq && q > m; q -= m)
      if (is_prime32(q)) P.primes[found++] = (uint32_t)q;
    if (found != P.nq) return fail(HW_EINVAL, "not enough primes");
  }
  for (uint32_t i = 0; i < P.nq; ++i) {
    const uint32_t q = P.primes[i];
    if (q >= (1u << 30) || !is_prime32(q) || (q - 1) % m)
      return fail(HW_EINVAL, "prime %u: need a prime < 2^30 with q = 1 mod 2N", q);
    for (uint32_t j = 0; j < i; ++j)
      if (P.primes[j] == q) return fail(HW_EINVAL, "primes must be distinct");
  }
  for (uint32_t i = P.nq; i < 4; ++i) P.primes[i] = 0;

  HIP_TRY(hipSetDevice(device));
  hw_ctx* c = new hw_ctx();
  c->prm = P;
  c->device = device;
  c->logN = logN;
  const uint32_t N = P.N;
  c->Q = 1;
  for (uint32_t i = 0; i < P.nq; ++i) c->Q *= P.primes[i];
  const u128 delta = c->Q / P.plain_mod;
  if (delta < 2) {
    delete c;
    return fail(HW_EINVAL, "plain_mod too large for Q");
  }

  // tables: for each prime fwd[N], inv[N] and evx[N] of (w, Shoup); the
  // forward table holds -w mod 2^32 in place of w (its butterflies form the
  // negated product directly)
  std::vector<uint2> host((size_t)3 * P.nq * N);
  for (uint32_t i = 0; i < P.nq; ++i) {
    const uint32_t q = P.primes[i];
    uint64_t g = 2;  // smallest quadratic non-residue: psi = g^((q-1)/2N) has order 2N
    while (powm(g, (q - 1) / 2, q) != q - 1) ++g;
    const uint64_t psi = powm(g, (q - 1) / m, q);
    const uint64_t psi_inv = powm(psi, q - 2, q);
    uint2* fw = host.data() + (size_t)3 * i * N;
    uint2* iv = fw + N;
    uint2* ev = iv + N;
    for (uint32_t k = 0; k < N; ++k) {
      const uint32_t w = (uint32_t)powm(psi, brv(k, logN), q);
      const uint32_t wi = (uint32_t)powm(psi_inv, brv(k, logN), q);
      // the forward transform's output k is the evaluation at psi^(2 brv(k) + 1): for X, that point
      const uint32_t x = (uint32_t)powm(psi, 2ull * brv(k, logN) + 1, q);
      fw[k] = make_uint2(0u - w, shoup(w, q));
      iv[k] = make_uint2(wi, shoup(wi, q));
      ev[k] = make_uint2(x, shoup(x, q));
    }
    hw::PrimeTab& pt = c->tabs.pt[i];
    pt.q = q;
    pt.two_q = 2 * q;
    pt.ninv = (uint32_t)powm(N, q - 2, q);
    pt.ninv_sh = shoup(pt.ninv, q);
    pt.r32 = (uint32_t)((1ull << 32) % q);
    pt.r32_sh = shoup(pt.r32, q);
    pt.one_sh = (uint32_t)((1ull << 32) / q);
    pt.delta = (uint32_t)(delta % q);
    const u128 Mi = c->Q / q;
    c->crt.M_lo[i] = (uint64_t)Mi;
    c->crt.M_hi[i] = (uint64_t)(Mi >> 64);
    c->crt.inv[i] = (uint32_t)powm((uint64_t)(Mi % q), q - 2, q);
  }
  c->crt.Q_lo = (uint64_t)c->Q;
  c->crt.Q_hi = (uint64_t)(c->Q >> 64);
  c->crt.half_lo = (uint64_t)(c->Q / 2);
  c->crt.half_hi = (uint64_t)((c->Q / 2) >> 64);
  c->crt.p = P.plain_mod;
  build_cdt(P.sigma, c->cdt.T);
  uint8_t guide[hw::CDT_GUIDE_SIZE];
  build_cdt_guide(c->cdt.T, guide);

  // the twiddle tables, then the CDT guide (at a 16-byte aligned offset: 3 nq N uint2)
  const size_t tw_bytes = host.size() * sizeof(uint2);
  hipError_t e = hipMalloc(&c->d_tables, tw_bytes + hw::CDT_GUIDE_SIZE);
  if (e == hipSuccess) e = hipMemcpy(c->d_tables, host.data(), tw_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(static_cast<char*>(c->d_tables) + tw_bytes, guide, hw::CDT_GUIDE_SIZE, hipMemcpyHostToDevice);
  c->cdt.guide = reinterpret_cast<const uint8_t*>(static_cast<char*>(c->d_tables) + tw_bytes);
  if (e == hipSuccess) e = hipMalloc(&c->d_skhat, sizeof(uint32_t) * sk_hat_words(c));
  if (e != hipSuccess) {
    hw_ctx_destroy(c);
    return fail(e == hipErrorOutOfMemory ? HW_ENOMEM : HW_EDEVICE, "table upload: %s", hipGetErrorString(e));
  }
  for (uint32_t i = 0; i < P.nq; ++i) {
    c->tabs.fwd[i] = reinterpret_cast<const uint2*>(c->d_tables) + (size_t)3 * i * N;
    c->tabs.inv[i] = c->tabs.fwd[i] + N;
    c->tabs.evx[i] = c->tabs.fwd[i] + 2 * N;
  }
  const char* wb = getenv("HWISARD_WS_BYTES");
  c->ws_budget = wb ? (size_t)strtoull(wb, nullptr, 10) : ((size_t)16 << 30);
  const char* tn = getenv("HWISARD_TUNE");
  c->tune_off = tn && strcmp(tn, "0") == 0;
  *out = c;
  return ok();
}

extern "C" void hw_ctx_destroy(hw_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  if (c->d_tables) hipFree(c->d_tables);
  if (c->d_skhat) hipFree(c->d_skhat);
  if (c->d_ws) hipFree(c->d_ws);
  for (auto& kv : c->perms) hipFree(kv.second);
  if (c->h_btab) hipHostFree(c->h_btab);
  if (c->d_btab) hipFree(c->d_btab);
  if (c->h_itab) hipHostFree(c->h_itab);
  if (c->d_itab) hipFree(c->d_itab);
  if (c->d_counter) hipFree(c->d_counter);
  for (auto& kv : c->tune)
    for (auto& p : kv.second.pend) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  delete c;
}

extern "C" hw_status hw_ctx_params(const hw_ctx* c, hw_params* out) {
  if (!c || !out) return fail(HW_EINVAL, "null argument");
  *out = c->prm;
  return ok();
}

extern "C" hw_status hw_sizes(const hw_ctx* c, uint64_t* sk, uint64_t* rlwe, uint64_t* rgsw, uint64_t* lwe) {
  if (!c) return fail(HW_EINVAL, "null context");
  if (sk) *sk = 4ull * c->prm.N;
  if (rlwe) *rlwe = 4 * rlwe_words(c);
  if (rgsw) *rgsw = 4 * rgsw_words(c);
  if (lwe) *lwe = 4 * lwe_words(c);
  return ok();
}

static uint32_t ceil_log2(uint32_t l) {
  uint32_t L = 0;
  while ((1u << L) < l) ++L;
  return L;
}


// rows of a model RAM with z tree bits, L label bits and l classes: the
// leaves of the IVP tree that hold a class below l (Definition 2's k1 when
// z >= L; all 2^z leaves when z < L)
uint32_t live_rows(uint32_t z, uint32_t L, uint32_t l) { return z >= L ? l << (z - L) : 1u << z; }

// external products of one IVP over nb index bits: the rotation chain and
// the live tree nodes (one split per live leaf beyond the first)
// live splits of tree level lev (< z) of an IVP: nodes j < 2^lev that lead to
// a class below l and whose new branch j + 2^lev does too (node_live of the
// kernels; with L = 0 every node is live)
uint32_t live_splits(uint32_t lev, uint32_t z, uint32_t L, uint32_t l) {
  if (lev >= z) return 0;
  auto live = [&](uint32_t u) { return z < L || (u & ((1u << L) - 1u)) < l; };
  const uint32_t n = 1u << lev;
  uint32_t c = 0;
  for (uint32_t j = 0; j < n; ++j) c += live(j) && live(j + n);
  return c;
}

uint32_t ivp_xp(uint32_t nb, int logN, uint32_t L, uint32_t l) {
  const uint32_t nr = std::min(nb, (uint32_t)logN);
  return nr + live_rows(nb - nr, L, l) - 1;
}

hw_status check_shape(const hw_ctx* c, const hw_wisard_shape* sh, Dims* d) {
  if (!sh) return fail(HW_EINVAL, "null shape");
  if (sh->layout > 2) return fail(HW_EINVAL, "shape.layout = %u: must be 0, 1 or 2", sh->layout);
  if (sh->s < 1 || sh->s > (1u << 24)) return fail(HW_EINVAL, "s = %u out of range [1, 2^24]", sh->s);
  if (sh->l < 1 || sh->l > 256) return fail(HW_EINVAL, "l = %u out of range [1, 256]", sh->l);
  if (sh->a < 1 || sh->a > 20) return fail(HW_EINVAL, "a = %u out of range [1, 20]", sh->a);
  d->L = ceil_log2(sh->l);
  // class-packed rows need the tree to hold tuple bits only (z <= a_j): L <= log2 N,
  // which the supported rings (N >= 1024) and l <= 256 always meet
  if (sh->layout && d->L > (uint32_t)c->logN)
    return fail(HW_EINVAL, "layout %u needs ceil(log2 l) <= log2 N", sh->layout);
  d->k0 = (sh->s + sh->a - 1) / sh->a;
  const uint32_t nb = d->L + sh->a;
  const uint32_t nr = nb < (uint32_t)c->logN ? nb : (uint32_t)c->logN;
  d->z = nb - nr;
  d->kt = 1u << d->z;
  d->layout = sh->layout;
  d->pL = sh->layout ? 0u : d->L;
  d->pl = sh->layout ? 1u : sh->l;
  d->k1 = live_rows(d->z, d->pL, d->pl);
  d->nbf = nb;
  d->rpr = sh->layout == 2 && nb < (uint32_t)c->logN ? 1u << (c->logN - nb) : 1u;
  d->rows = (d->k0 + d->rpr - 1) / d->rpr;
  return HW_OK;
}

// CMUX-tree temporaries of one inference VP: the outputs of its widest
// encrypted level
uint32_t infer_slots(const Dims& d) { return d.z > d.pL + 1 ? (1u << (d.z - d.pL - 1)) : 1u; }

// external products of the inference of one sample: per VP the encrypted
// tree levels and the encrypted positions of the rotation chain; layout 0
// runs one VP per (RAM, label), layout 1 one per RAM
double infer_xp_per_sample(const hw_ctx* c, const hw_wisard_shape* sh, const Dims& d) {
  double xp = 0;
  for (uint32_t j = 0; j < d.k0; ++j) {
    const uint32_t aj = std::min(sh->a, sh->s - j * sh->a);
    const uint32_t nb = d.L + aj;
    const uint32_t nr = std::min(nb, (uint32_t)c->logN), z = nb - nr;
    const uint32_t tree = z > d.pL ? (1u << (z - d.pL)) - 1 : 0;
    if (d.layout) {
      xp += tree + (aj - z);  // the chain's tuple bits; the label bits on top stay clear zeros
    } else {
      const uint32_t chain = z >= d.L ? nr : (nr > d.L - z ? nr - (d.L - z) : 0);
      xp += (double)sh->l * (tree + chain);
    }
  }
  return xp;
}

extern "C" hw_status hw_wisard_dims(const hw_ctx* c, const hw_wisard_shape* sh, uint32_t* k0, uint32_t* k1,
                                    uint64_t* model_bytes) {
  if (!c) return fail(HW_EINVAL, "null context");
  Dims d;
  hw_status st = check_shape(c, sh, &d);
  if (st) return st;
  if (k0) *k0 = d.k0;
  if (k1) *k1 = d.k1;
  if (model_bytes) *model_bytes = (uint64_t)d.rows * d.k1 * 4 * rlwe_words(c);
  return ok();
}

extern "C" hw_status hw_wisard_model_rows(const hw_ctx* c, const hw_wisard_shape* sh, uint32_t* rows,
                                          uint32_t* rams_per_row) {
  if (!c) return fail(HW_EINVAL, "null context");
  Dims d;
  hw_status st = check_shape(c, sh, &d);
  if (st) return st;
  if (rows) *rows = d.rows;
  if (rams_per_row) *rams_per_row = d.rpr;
  return ok();
}

static void make_perm(uint32_t s, uint64_t seed, uint32_t* pi) {
  for (uint32_t k = 0; k < s; ++k) pi[k] = k;
  for (int64_t k = (int64_t)s - 1; k >= 1; --k) {
    const uint64_t j = draw64(seed, 2u, (uint64_t)((int64_t)s - 1 - k)) % (uint64_t)(k + 1);
    std::swap(pi[k], pi[j]);
  }
}

extern "C" hw_status hw_permutation(const hw_wisard_shape* sh, uint32_t* perm_host) {
  if (!sh || !perm_host) return fail(HW_EINVAL, "null argument");
  if (sh->s < 1 || sh->s > (1u << 24)) return fail(HW_EINVAL, "s out of range");
  make_perm(sh->s, sh->perm_seed, perm_host);
  return ok();
}

hw_status ensure_ws(hw_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return HW_OK;
  if (c->d_ws) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(c->d_ws));
    c->d_ws = nullptr;
    c->ws_bytes = 0;
  }
  HIP_TRY(hipMalloc(&c->d_ws, bytes));
  c->ws_bytes = bytes;
  return HW_OK;
}

// the device permutation of (s, seed), uploaded once and kept with the context
hw_status perm_for(hw_ctx* c, const hw_wisard_shape* sh, hipStream_t st, const uint32_t** out) {
  const auto key = std::make_pair(sh->s, sh->perm_seed);
  auto it = c->perms.find(key);
  if (it == c->perms.end()) {
    std::vector<uint32_t> h(sh->s);
    make_perm(sh->s, sh->perm_seed, h.data());
    uint32_t* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(uint32_t) * sh->s));
    HIP_TRY(hipMemcpyAsync(d, h.data(), sizeof(uint32_t) * sh->s, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    it = c->perms.emplace(key, d).first;
  }
  *out = it->second;
  return HW_OK;
}

hw_status enter(hw_ctx* c) {
  if (!c) return fail(HW_EINVAL, "null context");
  HIP_TRY(hipSetDevice(c->device));
  return HW_OK;
}


// ---------------------------------------------------------------------------
// client side
// ---------------------------------------------------------------------------

extern "C" hw_status hw_keygen(hw_ctx* c, uint64_t seed, int32_t* sk, hipStream_t st) {
  CHECK(enter(c));
  if (!sk) return fail(HW_EINVAL, "null key buffer");
  HIP_TRY(hw::launch_keygen(c->prm.N, seed, sk, st));
  return ok();
}

static hw_status sk_hat(hw_ctx* c, const int32_t* sk, hipStream_t st) {
  if (!sk) return fail(HW_EINVAL, "null key");
  HIP_TRY(hw::launch_sk_hat(c->logN, c->prm.nq, c->tabs, sk, c->d_skhat, st));
  return HW_OK;
}

extern "C" hw_status hw_encrypt_rgsw_bits(hw_ctx* c, const int32_t* sk, const uint8_t* bits, uint64_t nbits,
                                          uint64_t seed, uint64_t ct0, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  if (nbits == 0) return ok();
  if (!bits || !out) return fail(HW_EINVAL, "null buffer");
  CHECK(sk_hat(c, sk, st));
  hw::EncArgs A{};
  A.sk = sk;
  A.sk_hat = c->d_skhat;
  A.bits = bits;
  A.out = out;
  A.seed = seed;
  A.ct0 = ct0;
  A.log_base = c->prm.log_base;
  const double rows = (double)nbits * 2 * c->prm.digits * c->prm.nq;
  HIP_TRY(timed(c, "encrypt_rgsw", rows, st, [&] {
    return tuned(c, "encrypt_rgsw", rows, st, [&](int v) {
      return hw::launch_enc_rgsw(c->logN, c->prm.nq, c->prm.digits, c->tabs, c->cdt, A, nbits,
                                 enc_rows_per_wg(v), st);
    });
  }));
  return ok();
}

extern "C" hw_status hw_encrypt_rlwe(hw_ctx* c, const int32_t* sk, const uint64_t* msg, uint64_t count,
                                     uint64_t seed, uint64_t ct0, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!out) return fail(HW_EINVAL, "null output");
  CHECK(sk_hat(c, sk, st));
  hw::EncArgs A{};
  A.sk = sk;
  A.sk_hat = c->d_skhat;
  A.msg = msg;
  A.out = out;
  A.seed = seed;
  A.ct0 = ct0;
  A.log_base = c->prm.log_base;
  HIP_TRY(timed(c, "encrypt_rlwe", (double)count, st,
                [&] { return hw::launch_enc_rlwe(c->logN, c->prm.nq, c->tabs, c->cdt, A, count, st); }));
  return ok();
}

extern "C" hw_status hw_decrypt_rlwe(hw_ctx* c, const int32_t* sk, const uint32_t* ct, uint64_t count,
                                     uint64_t* msg, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!ct || !msg) return fail(HW_EINVAL, "null buffer");
  CHECK(sk_hat(c, sk, st));
  HIP_TRY(timed(c, "decrypt_rlwe", (double)count, st, [&] {
    return hw::launch_dec_rlwe(c->logN, c->prm.nq, c->tabs, c->crt, c->d_skhat, ct, count, msg, st);
  }));
  return ok();
}

extern "C" hw_status hw_decrypt_lwe(hw_ctx* c, const int32_t* sk, const uint32_t* lwe, uint64_t count,
                                    uint64_t* msg, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!sk || !lwe || !msg) return fail(HW_EINVAL, "null buffer");
  HIP_TRY(timed(c, "decrypt_lwe", (double)count, st,
                [&] { return hw::launch_dec_lwe(c->logN, c->prm.nq, c->tabs, c->crt, sk, lwe, count, msg, st); }));
  return ok();
}

extern "C" hw_status hw_rgsw_export_canonical(hw_ctx* c, const uint32_t* rgsw, uint64_t count, uint32_t* out,
                                              hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!rgsw || !out) return fail(HW_EINVAL, "null buffer");
  if (rgsw == out) return fail(HW_EINVAL, "output must not alias input");
  HIP_TRY(hw::launch_rgsw_export(c->logN, c->prm.nq, c->prm.digits, c->tabs, rgsw, count, out, st));
  return ok();
}

extern "C" hw_status hw_ntt(hw_ctx* c, uint32_t* polys, uint64_t count, int inverse, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!polys) return fail(HW_EINVAL, "null buffer");
  if (inverse != 0 && inverse != 1) return fail(HW_EINVAL, "inverse must be 0 or 1");
  const double work = (double)count * c->prm.nq;
  HIP_TRY(timed(c, "ntt", work, st, [&] {
    return tuned(c, inverse ? "ntt_inverse" : "ntt", work, st, [&](int v) {
      return hw::launch_ntt(c->logN, c->prm.nq, c->tabs, polys, count, inverse, 1u << v, st);
    });
  }));
  return ok();
}

extern "C" hw_status hw_external_product(hw_ctx* c, const uint32_t* rgsw, const uint32_t* in, uint64_t count,
                                         uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!rgsw || !in || !out) return fail(HW_EINVAL, "null buffer");
  if (in == out) return fail(HW_EINVAL, "output must not alias input");
  HIP_TRY(timed(c, "xp", (double)count, st,
                [&] { return hw::launch_xp(c->logN, c->prm.nq, c->prm.digits, c->tabs, rgsw, in, count, out, st); }));
  return ok();
}

// ---------------------------------------------------------------------------
// server side
// ---------------------------------------------------------------------------

size_t train_ws_per_sample(const hw_ctx* c, const Dims& d) {
  return (size_t)(d.k0 + 1) * (d.kt + 1) * rlwe_words(c) * 4;  // the tree's 2^z leaves + input slot per RAM
}

size_t infer_ws_per_sample(const hw_ctx* c, const hw_wisard_shape* sh, const Dims& d) {
  const uint32_t nlab = d.layout ? 1u : sh->l;
  return (size_t)nlab * d.k0 * (infer_slots(d) + 1) * rlwe_words(c) * 4;  // + input slot
}

hw_status train_core(hw_ctx* c, const hw_wisard_shape* sh, const Dims& d, const uint32_t* perm,
                     const uint32_t* x_rgsw, const uint32_t* y_rgsw, uint64_t n, uint32_t* model,
                     uint32_t* class_count, uint32_t* ws, size_t ws_bytes, hipStream_t st, bool timing,
                     bool tune) {
  const size_t rw = rlwe_words(c);
  uint64_t n_sub = ws_bytes / train_ws_per_sample(c, d);
  if (n_sub < 1) return fail(HW_ENOMEM, "training workspace smaller than one sample");
  const uint32_t nram = d.k0 + (class_count ? 1 : 0);
  if (n_sub > n) n_sub = n;
  n_sub = std::min<uint64_t>(n_sub, std::min<uint64_t>(65535, (1u << 22) / nram));
  if (n_sub < 1) return fail(HW_EINVAL, "too many RAMs for one launch");
  hw::TrainArgs A{};
  A.x_rgsw = x_rgsw;
  A.y_rgsw = y_rgsw;
  A.perm = perm;
  A.out = ws;
  A.rgsw_words = rgsw_words(c);
  A.s = sh->s;
  A.a = sh->a;
  A.L = d.L;
  A.k0 = d.k0;
  A.k1 = d.k1;
  A.kt = d.kt;
  A.l = sh->l;
  A.layout = d.layout;
  hw::ReduceArgs R{};
  R.out = A.out;
  R.model = model;
  R.cnt = class_count;
  R.s = sh->s;
  R.a = sh->a;
  R.L = d.L;
  R.k0 = d.k0;
  R.k1 = d.k1;
  R.kt = d.kt;
  R.l = sh->l;
  R.layout = d.layout;
  R.logN = c->logN;
  R.N = c->prm.N;
  R.nq = c->prm.nq;
  A.nram = nram;
  // external products per sample: the rotation chain and the live CDEMUX tree of every RAM
  double xp_per_sample = 0;
  // per tree level: the most live splits any RAM has there (z <= L + a - 10 < 32
  // levels; a fixed array, so that the no-allocation entry point allocates nothing)
  uint32_t smax[32] = {}, levels = 0, widest = 0, seen[3] = {0, 0, 0}, nseen = 0;
  for (uint32_t j = 0; j < nram; ++j) {
    const uint32_t nb = j < d.k0 ? d.L + std::min(sh->a, sh->s - j * sh->a) : d.L;
    xp_per_sample += ivp_xp(nb, c->logN, d.pL, d.pl);
    // RAMs have at most three index widths: full tuples, the last tuple, the counter
    if (std::find(seen, seen + nseen, nb + 1) != seen + nseen) continue;
    if (nseen < 3) seen[nseen++] = nb + 1;
    const uint32_t z = std::min<uint32_t>(nb - std::min(nb, (uint32_t)c->logN), 32);
    levels = std::max(levels, z);
    for (uint32_t lev = 0; lev < z; ++lev) {
      smax[lev] = std::max(smax[lev], live_splits(lev, z, d.pL, d.pl));
      widest = std::max(widest, smax[lev]);
    }
  }
  // staging the levels launches (splits of the widest level) x samples x RAMs workgroups
  const bool can_stage = widest <= 4096;
  const bool tm = timing && c->prof;
  for (uint64_t i0 = 0; i0 < n; i0 += n_sub) {
    const uint64_t m = n - i0 < n_sub ? n - i0 : n_sub;
    A.i0 = i0;
    A.nsub = (uint32_t)m;
    const double xp = (double)m * xp_per_sample;
    // variant v: bit 0 grid order, bit 1 tree levels staged (one launch per
    // level after the chains), bit 2 occupancy target 4
    auto run = [&](int v) {
      A.map = (uint32_t)(v & 1);
      const int occ = v & 4 ? 4 : 3;
      A.tree = (v & 2) && can_stage ? 0u : 1u;
      hipError_t e = hw::launch_train(c->logN, c->prm.nq, c->prm.digits, c->tabs, A, occ, st);
      for (uint32_t lev = 0; e == hipSuccess && !A.tree && lev < levels; ++lev) {
        A.lev = lev;
        A.smax = smax[lev];
        e = hw::launch_train_level(c->logN, c->prm.nq, c->prm.digits, c->tabs, A, occ, st);
      }
      return e;
    };
    auto lt = [&] { return tune ? tuned(c, "train", xp, st, run) : run(settled_variant(c, "train")); };
    HIP_TRY(tm ? timed(c, "train", xp, st, lt) : lt());
    R.n_sub = m;
    hw::RowPackArgs P{};
    const bool rowpack = d.rpr > 1;  // layout 2 with several RAMs per row (then z = 0)
    if (rowpack) {  // one leaf per RAM: slot 0 of each block, rotated into its row
      P.src = ws;
      P.rstride = (uint64_t)(d.kt + 1) * rw;
      P.sstride = (uint64_t)(d.k0 + 1) * P.rstride;
      P.nsmp = m;
      P.dst = model;
      P.cnt = class_count;
      P.k0 = d.k0;
      P.rpr = d.rpr;
      P.nbf = d.nbf;
      P.rows = d.rows;
      P.N = c->prm.N;
      P.nq = c->prm.nq;
    }
    auto lr = [&] {
      return rowpack ? hw::launch_row_pack(c->tabs, P, st) : hw::launch_reduce_model(c->tabs, R, st);
    };
    HIP_TRY(tm ? timed(c, "reduce", (double)d.rows * d.k1 * rw, st, lr) : lr());
  }
  return HW_OK;
}

extern "C" hw_status hw_wisard_train_encrypted(hw_ctx* c, const hw_wisard_shape* sh, const uint32_t* x_rgsw,
                                               const uint32_t* y_rgsw, uint64_t n, uint32_t* model,
                                               uint32_t* class_count, hipStream_t st) {
  CHECK(enter(c));
  Dims d;
  CHECK(check_shape(c, sh, &d));
  if (n == 0) return ok();
  if (!x_rgsw || !model) return fail(HW_EINVAL, "null buffer");
  if (d.L > 0 && !y_rgsw) return fail(HW_EINVAL, "null label ciphertexts");
  const size_t per_sample = train_ws_per_sample(c, d);
  uint64_t n_sub = std::max<uint64_t>(1, c->ws_budget / per_sample);
  n_sub = std::min<uint64_t>(std::min<uint64_t>(n_sub, n), 65535);
  CHECK(ensure_ws(c, n_sub * per_sample));
  const uint32_t* perm = nullptr;
  CHECK(perm_for(c, sh, st, &perm));
  CHECK(train_core(c, sh, d, perm, x_rgsw, y_rgsw, n, model, class_count, static_cast<uint32_t*>(c->d_ws),
                   n_sub * per_sample, st, true));
  return ok();
}

hw_status infer_core(hw_ctx* c, const hw_wisard_shape* sh, const Dims& d, const uint32_t* perm,
                     const uint32_t* model, const uint32_t* x_rgsw, uint64_t n, uint32_t* ram_scores,
                     uint32_t* class_scores, uint32_t* ws, size_t ws_bytes, hipStream_t st, bool timing) {
  uint64_t n_sub = ws_bytes / infer_ws_per_sample(c, sh, d);
  if (n_sub < 1) return fail(HW_ENOMEM, "inference workspace smaller than one sample");
  if (n_sub > n) n_sub = n;
  const uint32_t nlab = d.layout ? 1u : sh->l;
  n_sub = std::min<uint64_t>(n_sub, std::min<uint64_t>(65535, (1u << 22) / ((uint64_t)d.k0 * nlab)));
  if (n_sub < 1) return fail(HW_EINVAL, "too many (RAM, label) pairs for one launch");
  const uint32_t slots = infer_slots(d);
  const double xp_per_sample = infer_xp_per_sample(c, sh, d);
  hw::InferArgs A{};
  A.model = model;
  A.x_rgsw = x_rgsw;
  A.perm = perm;
  A.scores = ram_scores;
  A.scratch = ws;
  A.rgsw_words = rgsw_words(c);
  A.s = sh->s;
  A.a = sh->a;
  A.L = d.L;
  A.l = sh->l;
  A.k0 = d.k0;
  A.k1 = d.k1;
  A.slots = slots;
  A.layout = d.layout;
  A.nlab = nlab;
  A.rpr = d.rpr;
  A.nbf = d.layout == 2 ? d.nbf : 0u;
  const bool tm = timing && c->prof;
  for (uint64_t i0 = 0; i0 < n; i0 += n_sub) {
    const uint64_t m = n - i0 < n_sub ? n - i0 : n_sub;
    A.i0 = i0;
    A.nsub = (uint32_t)m;
    const double xp = (double)m * xp_per_sample;
    auto li = [&] {
      return tuned(c, "infer", xp, st, [&](int v) {
        A.map = (uint32_t)(v & 1);
        return hw::launch_infer(c->logN, c->prm.nq, c->prm.digits, c->tabs, A, v & 2 ? 4 : 3, st);
      });
    };
    HIP_TRY(tm ? timed(c, "infer", xp, st, li) : li());
  }
  if (class_scores) {
    hw::SumArgs S{};
    S.scores = ram_scores;
    S.sums = class_scores;
    S.n = n;
    S.l = sh->l;
    S.k0 = d.k0;
    S.N = c->prm.N;
    S.nq = c->prm.nq;
    auto ls = [&] { return hw::launch_class_sums(c->tabs, S, st); };
    HIP_TRY(tm ? timed(c, "class_sums", (double)n * sh->l * lwe_words(c), st, ls) : ls());
  }
  return HW_OK;
}

extern "C" hw_status hw_wisard_infer_encrypted(hw_ctx* c, const hw_wisard_shape* sh, const uint32_t* model,
                                               const uint32_t* x_rgsw, uint64_t n, uint32_t* ram_scores,
                                               uint32_t* class_scores, hipStream_t st) {
  CHECK(enter(c));
  Dims d;
  CHECK(check_shape(c, sh, &d));
  if (n == 0) return ok();
  if (!model || !x_rgsw || !ram_scores) return fail(HW_EINVAL, "null buffer");
  const size_t per_sample = infer_ws_per_sample(c, sh, d);
  uint64_t n_sub = std::max<uint64_t>(1, c->ws_budget / per_sample);
  n_sub = std::min<uint64_t>(std::min<uint64_t>(n_sub, n), 65535);
  CHECK(ensure_ws(c, n_sub * per_sample));
  const uint32_t* perm = nullptr;
  CHECK(perm_for(c, sh, st, &perm));
  CHECK(infer_core(c, sh, d, perm, model, x_rgsw, n, ram_scores, class_scores, static_cast<uint32_t*>(c->d_ws),
                   n_sub * per_sample, st, true));
  return ok();
}

// ---------------------------------------------------------------------------
// PackingKeySwitching
// ---------------------------------------------------------------------------

extern "C" hw_status hw_pks_keygen(hw_ctx* c, const int32_t* sk, uint64_t seed, uint32_t* key, hipStream_t st) {
  CHECK(enter(c));
  if (!sk || !key) return fail(HW_EINVAL, "null buffer");
  CHECK(sk_hat(c, sk, st));
  hw::EncArgs A{};
  A.sk = sk;
  A.sk_hat = c->d_skhat;
  A.out = key;
  A.seed = seed;
  A.log_base = 6;  // PackingKeySwitching's own gadget: 5 digits of 6 bits per prime on every context
  HIP_TRY(timed(c, "encrypt_pks", (double)c->prm.N * 5 * c->prm.nq, st,
                [&] { return hw::launch_enc_pks(c->logN, c->prm.nq, c->tabs, c->cdt, A, st); }));
  return ok();
}

extern "C" hw_status hw_pks_key_export_canonical(hw_ctx* c, const uint32_t* key, uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  if (!key || !out) return fail(HW_EINVAL, "null buffer");
  if (key == out) return fail(HW_EINVAL, "output must not alias input");
  // N x D rows have the row layout of N / 2 RGSW ciphertexts (2 D rows each)
  HIP_TRY(hw::launch_rgsw_export(c->logN, c->prm.nq, 5, c->tabs, key, c->prm.N / 2, out, st));
  return ok();
}

extern "C" hw_status hw_pack_lwe(hw_ctx* c, const uint32_t* key, const uint32_t* lwe, uint32_t k, uint64_t count,
                                 uint32_t* out, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!key || !lwe || !out) return fail(HW_EINVAL, "null buffer");
  if (k < 1 || k > c->prm.N) return fail(HW_EINVAL, "k = %u out of range [1, N = %u]", k, c->prm.N);
  const uint32_t nblk = hw::pks_blocks(c->logN);
  const size_t per_group = (size_t)c->prm.nq * nblk * 2 * c->prm.N * 4;
  uint64_t n_sub = std::max<uint64_t>(1, c->ws_budget / per_group);
  n_sub = std::min<uint64_t>(std::min<uint64_t>(n_sub, count), 65535);
  CHECK(ensure_ws(c, n_sub * per_group));
  for (uint64_t c0 = 0; c0 < count; c0 += n_sub) {
    const uint64_t m = std::min<uint64_t>(n_sub, count - c0);
    hw::PksArgs A{};
    A.key = key;
    A.lwe = lwe + c0 * k * lwe_words(c);
    A.part = static_cast<uint32_t*>(c->d_ws);
    A.out = out + c0 * rlwe_words(c);
    A.k = k;
    HIP_TRY(timed(c, "pack_lwe", (double)m, st,
                  [&] { return hw::launch_pks(c->logN, c->prm.nq, c->tabs, A, (uint32_t)m, st); }));
  }
  return ok();
}

extern "C" hw_status hw_rlwe_add(hw_ctx* c, uint32_t* dst, const uint32_t* src, uint64_t count, hipStream_t st) {
  CHECK(enter(c));
  if (count == 0) return ok();
  if (!dst || !src) return fail(HW_EINVAL, "null buffer");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15)
    return fail(HW_EINVAL, "buffers must be 16-byte aligned");
  const uint64_t words = count * rlwe_words(c);
  HIP_TRY(timed(c, "rlwe_add", (double)words, st,
                [&] { return hw::launch_rlwe_add(c->tabs, dst, src, words, c->prm.N, c->prm.nq, st); }));
  return ok();
}

extern "C" hw_status hw_wisard_pack_rams(hw_ctx* c, const hw_wisard_shape* sh, const uint32_t* model_in,
                                         uint32_t* model_out, hipStream_t st) {
  CHECK(enter(c));
  Dims d;
  CHECK(check_shape(c, sh, &d));
  if (d.layout != 2) return fail(HW_EINVAL, "shape.layout must be 2 (the layout of model_out)");
  if (!model_in || !model_out) return fail(HW_EINVAL, "null buffer");
  const size_t rw = rlwe_words(c);
  const uintptr_t i0 = reinterpret_cast<uintptr_t>(model_in), i1 = i0 + (uintptr_t)d.k0 * d.k1 * rw * 4;
  const uintptr_t o0 = reinterpret_cast<uintptr_t>(model_out), o1 = o0 + (uintptr_t)d.rows * d.k1 * rw * 4;
  if (i0 < o1 && o0 < i1) return fail(HW_EINVAL, "model_out must not overlap model_in");
  if (d.rpr == 1) {  // one RAM per row: the rows are the class-packed rows
    HIP_TRY(hipMemcpyAsync(model_out, model_in, (size_t)d.k0 * d.k1 * rw * 4, hipMemcpyDeviceToDevice, st));
    return ok();
  }
  hw::RowPackArgs P{};
  P.src = model_in;
  P.rstride = (uint64_t)d.k1 * rw;
  P.sstride = 0;
  P.nsmp = 1;
  P.dst = model_out;
  P.k0 = d.k0;
  P.rpr = d.rpr;
  P.nbf = d.nbf;
  P.rows = d.rows;
  P.N = c->prm.N;
  P.nq = c->prm.nq;
  P.store = 1;
  HIP_TRY(timed(c, "pack_rams", (double)d.rows * rw, st, [&] { return hw::launch_row_pack(c->tabs, P, st); }));
  return ok();
}

// ---------------------------------------------------------------------------
// batched training
// ---------------------------------------------------------------------------


namespace {
// one persistent launch: the jobs, the queue of (job, RAM, piece) items
// (longest first) and the workspace it needs
struct BPlan {
  std::vector<hw::BJob> jobs;
  std::vector<hw::BItem> items;
  uint64_t words = 0;          // model (+ counter) words the reduction writes
  uint64_t acc_words = 0;      // accumulators of pieces >= 1
  uint64_t scratch_words = 0;  // per persistent workgroup
  uint32_t grid = 0;           // persistent workgroups: the larger of grid_occ[]
  uint32_t grid_occ[2] = {0, 0};  // for occupancy targets 3 and 4 (0: variant absent)
  uint32_t max_pieces = 0;
  double xp = 0;               // external products of the batch
  size_t ws_words() const { return (size_t)grid * scratch_words + acc_words; }
};
}  // namespace

// Validate the jobs, resolve their permutations and cut every (job, RAM)
// into pieces of consecutive samples.  A piece is aimed at 1/8 of one
// workgroup's share of the batch (load balance of the longest-first queue);
// pieces are made longer, down to one piece per RAM, until their
// accumulators and the workgroups' scratch fit the workspace budget.
static hw_status plan_batch(hw_ctx* c, const hw_train_job* jobs, uint32_t njobs, hipStream_t st, BPlan& B) {
  B = BPlan();
  if (njobs && !jobs) return fail(HW_EINVAL, "null job list");
  std::vector<Dims> dims(njobs);
  std::vector<const uint32_t*> perms(njobs, nullptr);
  for (uint32_t j = 0; j < njobs; ++j) {
    const hw_train_job& J = jobs[j];
    hw_status e = check_shape(c, &J.shape, &dims[j]);
    if (e) return fail(e, "job %u: %s", j, hw_last_error());
    if (J.n == 0) continue;
    if (J.shape.layout == 2)
      return fail(HW_EINVAL, "job %u: layout 2 rows are shared by several RAMs; batch-train layout 1 and pack", j);
    if (!J.x_rgsw_dev || !J.model_dev) return fail(HW_EINVAL, "job %u: null buffer", j);
    if (dims[j].L > 0 && !J.y_rgsw_dev) return fail(HW_EINVAL, "job %u: null label ciphertexts", j);
    if (J.n > 0xFFFFFFFFull) return fail(HW_EINVAL, "job %u: too many samples", j);
    for (uint32_t i = 0; i < j; ++i)
      if (jobs[i].n && (jobs[i].model_dev == J.model_dev ||
                        (J.class_count_dev && jobs[i].class_count_dev == J.class_count_dev)))
        return fail(HW_EINVAL, "jobs %u and %u share an output buffer", i, j);
  }
  for (uint32_t j = 0; j < njobs; ++j)
    if (jobs[j].n) CHECK(perm_for(c, &jobs[j].shape, st, &perms[j]));
  for (int v = 0; v < tune_variants(c, "train_batch"); ++v)
    HIP_TRY(hw::batch_grid(c->logN, c->prm.nq, c->prm.digits, v ? 4 : 3, &B.grid_occ[v]));
  B.grid = std::max(B.grid_occ[0], B.grid_occ[1]);
  const size_t rw = rlwe_words(c);
  // per job: RAMs, external products per (sample, RAM) and per sample
  std::vector<uint32_t> nram(njobs, 0), xp_max(njobs, 0);
  std::vector<double> xp_smp(njobs, 0);
  double W = 0;
  uint32_t k1max = 0;
  for (uint32_t j = 0; j < njobs; ++j) {
    if (!jobs[j].n) continue;
    const Dims& d = dims[j];
    nram[j] = d.k0 + (jobs[j].class_count_dev ? 1 : 0);
    for (uint32_t r = 0; r < nram[j]; ++r) {
      const uint32_t nb = r < d.k0 ? d.L + std::min(jobs[j].shape.a, jobs[j].shape.s - r * jobs[j].shape.a) : d.L;
      const uint32_t xp = ivp_xp(nb, c->logN, d.pL, d.pl);
      xp_max[j] = std::max(xp_max[j], xp);
      xp_smp[j] += xp;
    }
    W += xp_smp[j] * (double)jobs[j].n;
    k1max = std::max(k1max, d.kt);
  }
  if (W == 0) return HW_OK;
  B.scratch_words = (uint64_t)(k1max + 1) * rw;
  std::vector<uint32_t> per(njobs, 1), pieces(njobs, 0);
  double target = std::max(1.0, W / (8.0 * B.grid));
  for (;;) {
    B.acc_words = 0;
    bool single = true;
    for (uint32_t j = 0; j < njobs; ++j) {
      if (!jobs[j].n) continue;
      const uint64_t n = jobs[j].n;
      per[j] = (uint32_t)std::min<uint64_t>(n, std::max<uint64_t>(1, (uint64_t)(target / xp_max[j])));
      pieces[j] = (uint32_t)((n + per[j] - 1) / per[j]);
      B.acc_words += (uint64_t)(pieces[j] - 1) * nram[j] * dims[j].k1 * rw;
      single &= pieces[j] == 1;
    }
    if (single || 4 * B.ws_words() <= c->ws_budget) break;
    target *= 2;
  }
  uint64_t acc0 = 0;
  for (uint32_t j = 0; j < njobs; ++j) {
    if (!jobs[j].n) continue;
    const hw_train_job& J = jobs[j];
    const Dims& d = dims[j];
    hw::BJob b{};
    b.x = J.x_rgsw_dev;
    b.y = J.y_rgsw_dev;
    b.perm = perms[j];
    b.model = J.model_dev;
    b.cnt = J.class_count_dev;
    b.acc0 = acc0;
    b.words0 = B.words;
    b.s = J.shape.s;
    b.a = J.shape.a;
    b.L = d.L;
    b.k0 = d.k0;
    b.k1 = d.k1;
    b.kt = d.kt;
    b.l = J.shape.l;
    b.nsmp = (uint32_t)J.n;
    b.nram = nram[j];
    b.per = per[j];
    b.pieces = pieces[j];
    b.layout = d.layout;
    acc0 += (uint64_t)(pieces[j] - 1) * nram[j] * d.k1 * rw;
    if (pieces[j] > 1) B.words += (uint64_t)d.k0 * d.k1 * rw + (J.class_count_dev ? rw : 0);
    B.max_pieces = std::max(B.max_pieces, pieces[j]);
    const uint32_t jb = (uint32_t)B.jobs.size();
    // piece-major: the RAMs of one piece (one run of samples) are adjacent in
    // the queue, so workgroups running at the same time share the samples'
    // label ciphertexts in L2
    for (uint32_t p = 0; p < pieces[j]; ++p) {
      const uint64_t cnt = std::min<uint64_t>(per[j], J.n - (uint64_t)p * per[j]);
      for (uint32_t r = 0; r < nram[j]; ++r) {
        const uint32_t nb = r < d.k0 ? d.L + std::min(J.shape.a, J.shape.s - r * J.shape.a) : d.L;
        const uint64_t ixp = cnt * ivp_xp(nb, c->logN, d.pL, d.pl);
        B.items.push_back(hw::BItem{jb, r, p, (uint32_t)std::min<uint64_t>(ixp, 0xFFFFFFFFull)});
        B.xp += (double)ixp;
      }
    }
    B.jobs.push_back(b);
  }
  if (B.items.size() > 0xFFFFFFFFull) return fail(HW_EINVAL, "too many work items");
  // longest items first: the queue then ends with short ones
  std::stable_sort(B.items.begin(), B.items.end(),
                   [](const hw::BItem& x, const hw::BItem& y) { return x.xp > y.xp; });
  return HW_OK;
}

// enqueue the persistent launch and the reduction of the accumulators
static hw_status run_batch(hw_ctx* c, const BPlan& B, const hw::BJob* djobs, const hw::BItem* ditems,
                           uint32_t* counter, uint32_t* ws, hipStream_t st, bool timing) {
  hw::BatchArgs A{};
  A.jobs = djobs;
  A.items = ditems;
  A.nitems = (uint32_t)B.items.size();
  A.counter = counter;
  A.ws = ws;
  A.scratch_words = B.scratch_words;
  A.acc = ws + (size_t)B.grid * B.scratch_words;
  A.rgsw_words = rgsw_words(c);
  const bool tm = timing && c->prof;
  auto lt = [&] {
    return tuned(c, "train_batch", B.xp, st, [&](int v) {
      return hw::launch_train_batch(c->logN, c->prm.nq, c->prm.digits, c->tabs, A, B.grid_occ[v], v ? 4 : 3, st);
    });
  };
  HIP_TRY(tm ? timed(c, "train_batch", B.xp, st, lt) : lt());
  if (B.words) {
    auto lr = [&] {
      return hw::launch_reduce_batch(c->tabs, djobs, (uint32_t)B.jobs.size(), B.words, c->logN, c->prm.N,
                                     c->prm.nq, A.acc, st);
    };
    HIP_TRY(tm ? timed(c, "reduce_batch", (double)B.words, st, lr) : lr());
  }
  return HW_OK;
}

extern "C" hw_status hw_batch_train(hw_ctx* c, const hw_train_job* jobs, uint32_t njobs, hipStream_t st) {
  CHECK(enter(c));
  if (njobs == 0) return ok();
  BPlan B;
  CHECK(plan_batch(c, jobs, njobs, st, B));
  if (B.items.empty()) return ok();
  if (!c->d_counter) HIP_TRY(hipMalloc(&c->d_counter, 64));
  CHECK(ensure_ws(c, 4 * B.ws_words()));
  const size_t jb = B.jobs.size() * sizeof(hw::BJob), io = (jb + 255) / 256 * 256;
  const size_t need = io + B.items.size() * sizeof(hw::BItem);
  HIP_TRY(hipStreamSynchronize(st));  // an earlier batch on this stream has released the tables
  if (need > c->btab_bytes) {
    if (c->h_btab) HIP_TRY(hipHostFree(c->h_btab));
    if (c->d_btab) HIP_TRY(hipFree(c->d_btab));
    c->h_btab = c->d_btab = nullptr;
    c->btab_bytes = 0;
    HIP_TRY(hipHostMalloc(&c->h_btab, need));
    HIP_TRY(hipMalloc(&c->d_btab, need));
    c->btab_bytes = need;
  }
  char* h = static_cast<char*>(c->h_btab);
  memcpy(h, B.jobs.data(), jb);
  memcpy(h + io, B.items.data(), B.items.size() * sizeof(hw::BItem));
  HIP_TRY(hipMemcpyAsync(c->d_btab, c->h_btab, need, hipMemcpyHostToDevice, st));
  char* d = static_cast<char*>(c->d_btab);
  CHECK(run_batch(c, B, reinterpret_cast<const hw::BJob*>(d), reinterpret_cast<const hw::BItem*>(d + io),
                  c->d_counter, static_cast<uint32_t*>(c->d_ws), st, true));
  return ok();
}

// ---------------------------------------------------------------------------
// batch plans: the same queue computed once, tables uploaded once, launches
// captured into a HIP graph
// ---------------------------------------------------------------------------

struct hw_batch_plan {
  hw_ctx* ctx = nullptr;
  int device = 0;
  void* d_tab = nullptr;
  uint32_t* d_ws = nullptr;
  uint32_t* d_counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t items = 0;
  uint32_t max_pieces = 0;
  double xp = 0;
  size_t ws_bytes = 0;
};

static void free_plan(hw_batch_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->d_tab) (void)hipFree(P->d_tab);
  if (P->d_ws) (void)hipFree(P->d_ws);
  if (P->d_counter) (void)hipFree(P->d_counter);
  delete P;
}

static hw_status build_plan(hw_ctx* c, const hw_train_job* jobs, uint32_t njobs, hipStream_t cs, hw_batch_plan* P) {
  BPlan B;
  CHECK(plan_batch(c, jobs, njobs, cs, B));
  P->items = B.items.size();
  P->max_pieces = B.max_pieces;
  P->xp = B.xp;
  P->ws_bytes = 4 * B.ws_words();
  HIP_TRY(hipMalloc(&P->d_counter, 64));
  const size_t jb = B.jobs.size() * sizeof(hw::BJob), io = (jb + 255) / 256 * 256;
  const size_t tab_bytes = io + B.items.size() * sizeof(hw::BItem);
  if (!B.items.empty()) {
    std::vector<char> h(tab_bytes, 0);
    memcpy(h.data(), B.jobs.data(), jb);
    memcpy(h.data() + io, B.items.data(), B.items.size() * sizeof(hw::BItem));
    HIP_TRY(hipMalloc(&P->d_tab, tab_bytes));
    HIP_TRY(hipMemcpy(P->d_tab, h.data(), tab_bytes, hipMemcpyHostToDevice));
  }
  if (P->ws_bytes) HIP_TRY(hipMalloc(&P->d_ws, P->ws_bytes));
  // capture: kernel launches only (the queue counter is cleared by a kernel)
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hw_status st = HW_OK;
  if (!B.items.empty()) {
    char* d = static_cast<char*>(P->d_tab);
    st = run_batch(c, B, reinterpret_cast<const hw::BJob*>(d), reinterpret_cast<const hw::BItem*>(d + io),
                   P->d_counter, P->d_ws, cs, false);
  }
  const hipError_t ec = hipStreamEndCapture(cs, &P->graph);
  if (st != HW_OK) return st;
  HIP_TRY(ec);
  HIP_TRY(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
  return HW_OK;
}

extern "C" hw_status hw_batch_plan_create(hw_ctx* c, const hw_train_job* jobs, uint32_t njobs,
                                          hw_batch_plan** out) {
  CHECK(enter(c));
  if (!out) return fail(HW_EINVAL, "null output");
  *out = nullptr;
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hw_batch_plan* P = new hw_batch_plan();
  P->ctx = c;
  P->device = c->device;
  const hw_status st = build_plan(c, jobs, njobs, cs, P);
  (void)hipStreamDestroy(cs);
  if (st != HW_OK) {
    free_plan(P);
    return st;
  }
  *out = P;
  return ok();
}

extern "C" hw_status hw_batch_plan_launch(hw_batch_plan* P, hipStream_t st) {
  if (!P) return fail(HW_EINVAL, "null plan");
  hw_ctx* c = P->ctx;
  CHECK(enter(c));
  HIP_TRY(timed(c, "batch_plan", P->xp, st, [&] { return hipGraphLaunch(P->exec, st); }));
  return ok();
}

extern "C" hw_status hw_batch_plan_info(const hw_batch_plan* P, uint64_t* items, uint32_t* max_pieces, double* xp,
                                        uint64_t* ws_bytes) {
  if (!P) return fail(HW_EINVAL, "null plan");
  if (items) *items = P->items;
  if (max_pieces) *max_pieces = P->max_pieces;
  if (xp) *xp = P->xp;
  if (ws_bytes) *ws_bytes = P->ws_bytes;
  return ok();
}

extern "C" void hw_batch_plan_destroy(hw_batch_plan* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();  // a launch still in flight reads the plan's buffers
  free_plan(P);
}

// ---------------------------------------------------------------------------
// schedule tuning
// ---------------------------------------------------------------------------

namespace {
struct TuneKernel {
  const char* kernel;
  double min_work;  // launches with less work (too few workgroups to fill the chip) are not timed
  std::vector<const char*> variants;
};
// variants past the first four of "train", the first two of "infer" and the
// first of "train_batch" (occupancy target 4) exist for N = 4096 only
const std::vector<TuneKernel>& tune_table() {
  static const std::vector<TuneKernel> t = {
      {"train", 5e4, {"ram-major 2-D grid", "xcd-grouped 1-D grid", "ram-major 2-D grid, tree levels staged",
                      "xcd-grouped 1-D grid, tree levels staged", "ram-major 2-D grid, 4 waves/SIMD",
                      "xcd-grouped 1-D grid, 4 waves/SIMD", "ram-major 2-D grid, tree levels staged, 4 waves/SIMD",
                      "xcd-grouped 1-D grid, tree levels staged, 4 waves/SIMD"}},
      {"infer", 5e4, {"ram-major 3-D grid", "labels-adjacent xcd-grouped 1-D grid",
                      "ram-major 3-D grid, 4 waves/SIMD", "labels-adjacent xcd-grouped 1-D grid, 4 waves/SIMD"}},
      {"train_batch", 5e4, {"persistent, 3 waves/SIMD", "persistent, 4 waves/SIMD"}},
      {"infer_batch", 5e4, {"persistent, 3 waves/SIMD", "persistent, 4 waves/SIMD"}},
      {"ntt", 16384, {"1 polynomial/workgroup", "2 polynomials/workgroup", "4 polynomials/workgroup",
                      "8 polynomials/workgroup"}},
      {"ntt_inverse", 16384, {"1 polynomial/workgroup", "2 polynomials/workgroup", "4 polynomials/workgroup",
                              "8 polynomials/workgroup"}},
      {"encrypt_rgsw", 2e4, {"1 row/workgroup", "2 rows/workgroup", "5 rows/workgroup"}},
  };
  return t;
}
}  // namespace

int enc_rows_per_wg(int v) { return v == 2 ? 5 : v + 1; }

static int table_variants(const char* kernel) {
  for (const auto& k : tune_table())
    if (!strcmp(k.kernel, kernel)) return (int)k.variants.size();
  return 0;
}

int tune_variants(const hw_ctx* c, const char* kernel) {
  const int n = table_variants(kernel);
  if (!strcmp(kernel, "encrypt_rgsw") && c->prm.digits == 2) return 2;  // 5 rows per workgroup divide no 4 nq
  if (c->logN == 12) return n;
  if (!strcmp(kernel, "train")) return 4;
  if (!strcmp(kernel, "infer")) return 2;
  if (!strcmp(kernel, "train_batch") || !strcmp(kernel, "infer_batch")) return 1;
  return n;
}

double tune_min_work(const char* kernel) {
  for (const auto& k : tune_table())
    if (!strcmp(k.kernel, kernel)) return k.min_work;
  return 0;
}

const char* tune_variant_name(const char* kernel, int v) {
  for (const auto& k : tune_table())
    if (!strcmp(k.kernel, kernel)) return v >= 0 && v < (int)k.variants.size() ? k.variants[v] : nullptr;
  return nullptr;
}

void tune_settle(TuneState& S) {
  for (size_t i = 0; i < S.pend.size();) {
    TuneState::Pend& p = S.pend[i];
    const hipError_t q = hipEventQuery(p.b);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    float ms = 0;
    if (q == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess && p.work > 0) {
      S.best[p.v] = std::min(S.best[p.v], (double)ms / p.work);
      S.runs[p.v] += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
    S.pend.erase(S.pend.begin() + i);
  }
  if (S.chosen >= 0 || S.runs.empty()) return;
  for (int r : S.runs)
    if (r < TUNE_RUNS) return;
  int best = 0;
  for (int v = 1; v < (int)S.best.size(); ++v)
    if (S.best[v] < S.best[best]) best = v;
  S.chosen = best;
}

extern "C" hw_status hw_tune_set(hw_ctx* c, const char* kernel, int variant) {
  if (!c || !kernel) return fail(HW_EINVAL, "null argument");
  const int n = tune_variants(c, kernel);
  if (n == 0) return fail(HW_EINVAL, "no tunable kernel named '%s'", kernel);
  if (variant < -1 || variant >= n) return fail(HW_EINVAL, "variant %d out of range [-1, %d)", variant, n);
  CHECK(enter(c));
  TuneState& S = c->tune[kernel];
  for (auto& p : S.pend) {  // drop timings in flight
    (void)hipEventSynchronize(p.b);
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  S = TuneState();
  S.forced = variant;
  return ok();
}

extern "C" hw_status hw_tune_get(hw_ctx* c, const char* kernel, int* variant, int* timings, int* count) {
  if (!c || !kernel) return fail(HW_EINVAL, "null argument");
  const int n = tune_variants(c, kernel);
  if (n == 0) return fail(HW_EINVAL, "no tunable kernel named '%s'", kernel);
  CHECK(enter(c));
  TuneState& S = c->tune[kernel];
  if ((int)S.runs.size() != n) {
    S.runs.assign(n, 0);
    S.best.assign(n, 1e300);
  }
  if (S.chosen < 0 && S.forced < 0 && (c->tune_off || n == 1)) S.chosen = 0;
  tune_settle(S);
  int t = 0;
  for (int r : S.runs) t += r;
  if (variant) *variant = S.forced >= 0 ? S.forced : S.chosen;
  if (timings) *timings = t;
  if (count) *count = n;
  return ok();
}

extern "C" const char* hw_tune_variant_name(const char* kernel, int variant) {
  return kernel ? tune_variant_name(kernel, variant) : nullptr;
}

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------

extern "C" hw_status hw_profile_enable(hw_ctx* c, int enable) {
  if (!c) return fail(HW_EINVAL, "null context");
  c->prof = enable != 0;
  return ok();
}

static hw_status drain(hw_ctx* c) {
  for (auto& r : c->pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    auto& a = c->acc[r.name];
    a.ms += ms;
    a.work += r.work;
    a.launches += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->pending.clear();
  return HW_OK;
}

extern "C" hw_status hw_profile_read(hw_ctx* c, const char* name, double* total_ms, uint64_t* launches,
                                     double* work) {
  if (!c || !name) return fail(HW_EINVAL, "null argument");
  CHECK(enter(c));
  CHECK(drain(c));
  auto it = c->acc.find(name);
  const hw_ctx::Acc a = it == c->acc.end() ? hw_ctx::Acc{} : it->second;
  if (total_ms) *total_ms = a.ms;
  if (launches) *launches = a.launches;
  if (work) *work = a.work;
  return ok();
}

extern "C" hw_status hw_profile_reset(hw_ctx* c) {
  if (!c) return fail(HW_EINVAL, "null context");
  CHECK(enter(c));
  CHECK(drain(c));
  c->acc.clear();
  return ok();
}
