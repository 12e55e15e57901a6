/*
 * hwisard.h -- C ABI of the MI355X (gfx950) hot path of encrypted WiSARD
 * training and inference (Homomorphic WiSARDs, arXiv 2403.20190).
 *
 * Conventions shared by every call
 * --------------------------------
 * Status.      Every call returns hw_status (0 = HW_OK).  Arguments are checked
 *              on the host before anything is enqueued, so a call that fails
 *              its checks has written nothing.  Errors raised by the device
 *              runtime while enqueueing are returned as HW_EDEVICE; faults of
 *              work already enqueued surface at the next synchronisation of
 *              the caller's stream.  hw_last_error() gives a message for the
 *              last failing call of the calling thread.
 * Ownership.   The caller owns every buffer it passes; device pointers ("_dev")
 *              must stay valid until the work on `stream` has completed.  The
 *              library owns only the context, its tables and its workspace.
 * Streams.     Device work is enqueued on the caller's `stream` (NULL = the
 *              default stream) and returns without waiting for it.  Calls on
 *              one context must be serialised by the caller (they share its
 *              workspace); distinct contexts are independent.
 * Residues.    Ciphertext words are uint32 residues in [0, q_i).  Coefficient
 *              order: a polynomial over all primes is [prime][N]; an RLWE
 *              ciphertext is [poly a=0, b=1][prime][N]; an LWE ciphertext is
 *              [prime][N+1] (a_0..a_{N-1}, b); RGSW ciphertexts use a device
 *              layout (NTT domain, internal coefficient order) of
 *              hw_sizes().rgsw bytes each, exported to the coefficient domain
 *              by hw_rgsw_export_canonical.
 * Secret key.  int32[N] with entries in {-1, 0, 1}.
 */
#ifndef HWISARD_H
#define HWISARD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HW_OK = 0,
  HW_EINVAL = -1,        /* invalid argument or shape */
  HW_ENOMEM = -2,        /* device allocation failed */
  HW_EDEVICE = -3,       /* HIP runtime error */
  HW_EUNSUPPORTED = -4,  /* parameter set outside the compiled kernels */
  HW_EBUSY = -5,         /* serving engine: request refused for lack of memory */
  HW_ECANCELLED = -6     /* serving engine: request cancelled */
} hw_status;

/* One RLWE parameter set (Setup, Sec. 2.5.1).  The paper fixes a 64-bit torus
 * modulus (Table 2); this library uses residues modulo 30-bit NTT-friendly
 * primes instead.  The RGSW gadget (log_base, digits) is (6, 5) or, on rings
 * of two or more primes, (15, 2): the digit size of the paper's HE1 TFHE set
 * (Sec. 4), with 2.5x fewer rows per RGSW and fewer forward transforms per
 * external product; other pairs give HW_EUNSUPPORTED.  The gadget shapes
 * RGSW only: keys, RLWE and LWE ciphertexts are the same under both, so two
 * contexts of one ring with different gadgets share them.
 * PackingKeySwitching keeps 5 digits of 6 bits per prime on every context. */
typedef struct {
  uint32_t N;          /* ring degree: 1024, 2048 or 4096 */
  uint32_t nq;         /* number of primes: 1, 2 or 3 */
  uint32_t primes[4];  /* distinct primes q < 2^30, q = 1 mod 2N; primes[0] == 0
                          selects the nq largest such primes, decreasing */
  uint32_t log_base;   /* gadget base 2^log_base: 6, or 15 when nq >= 2 */
  uint32_t digits;     /* gadget digits per prime: 5 with base 2^6, 2 with base 2^15 */
  double sigma;        /* standard deviation of the discrete Gaussian error */
  uint64_t plain_mod;  /* plaintext modulus p: a power of two, 2 <= p <= 2^20 */
} hw_params;

/* WiSARD shape (Def. 1-2): s input bits, l classes, tuple (address) size a,
 * seed of the pseudo-random input permutation pi_r, and the layout of the
 * encrypted model:
 *   0  label-pruned rows (Def. 2): the IVP index is [label bits, tuple bits];
 *      a row holds only the tree leaves of classes below l; inference runs
 *      one VP per (RAM, label).
 *   1  class-packed rows (the horizontal packing of the paper's further
 *      improvements, Sec. 5.1): the index is [tuple bits, label bits], so the
 *      cell (class c, address m) of RAM j sits in row (m + 2^a_j c) mod 2^z
 *      at coefficient (m + 2^a_j c) >> z; every tree leaf is a row
 *      (k1 = 2^z); one VP per RAM over the tuple bits brings the cell of
 *      every class to coefficient c 2^(a_j - z) and inference extracts all l
 *      scores from it.  Same scores, fewer external products at inference,
 *      more at training when l < 2^L.
 *   2  class-packed rows with several RAMs per row: when 2^(L+a) < N, the
 *      r = N / 2^(L+a) RAMs j = R r + t share model row R, RAM j's layout-1
 *      row rotated by X^(t 2^(L+a)); the model is [ceil(k0 / r)][1] RLWE
 *      (hw_wisard_model_rows).  Same scores and external products as
 *      layout 1, r times less model memory.  With r = 1 it is layout 1.
 *      Batched training rejects it (its rows are written in place per RAM);
 *      batch-train layout 1 and convert with hw_wisard_pack_rams.
 * Other values are rejected (HW_EINVAL). */
typedef struct {
  uint32_t s;
  uint32_t l;
  uint32_t a;
  uint32_t layout;     /* model layout: 0, 1 or 2, see above */
  uint64_t perm_seed;
} hw_wisard_shape;

typedef struct hw_ctx hw_ctx;

/* Create a context for `params` on HIP device `device`: validates the
 * parameters, derives the primes, NTT twiddle tables, Delta = floor(Q/p) and
 * CRT constants, and uploads them.  On success *out owns them. */
hw_status hw_ctx_create(const hw_params* params, int device, hw_ctx** out);

/* Release a context and its device memory; waits for the device first. */
void hw_ctx_destroy(hw_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* hw_last_error(void);

/* The resolved parameter set (primes filled in). */
hw_status hw_ctx_params(const hw_ctx* ctx, hw_params* out);

/* Bytes of the secret key (int32[N]), of one RLWE, one RGSW (device layout)
 * and one LWE ciphertext.  Any output pointer may be NULL. */
hw_status hw_sizes(const hw_ctx* ctx, uint64_t* sk_bytes, uint64_t* rlwe_bytes, uint64_t* rgsw_bytes,
                   uint64_t* lwe_bytes);

/* Model geometry of Def. 2: k0 = ceil(s/a) RAMs and k1 RLWE per RAM.  With
 * L = ceil(log2 l) label bits and z = L + a - min(L + a, log2 N) tree bits:
 * layout 0 keeps the ciphertexts that hold a class below l (leaf
 * d = c + 2^L w holds class c and goes to row w l + c), so
 * k1 = l 2^(z-L) = ceil(l 2^a / N) when z >= L, and k1 = 2^z otherwise;
 * layouts 1 and 2 keep all k1 = 2^z leaves.
 * model_bytes is the size of H = [rows][k1] RLWE (rows = k0 except for
 * layout 2, see hw_wisard_model_rows). */
hw_status hw_wisard_dims(const hw_ctx* ctx, const hw_wisard_shape* shape, uint32_t* k0,
                         uint32_t* k1, uint64_t* model_bytes);

/* Rows of the model and RAMs per row: (k0, 1) for layouts 0 and 1;
 * (ceil(k0 / r), r) for layout 2 with r = N / 2^(L+a) when 2^(L+a) < N. */
hw_status hw_wisard_model_rows(const hw_ctx* ctx, const hw_wisard_shape* shape, uint32_t* rows,
                               uint32_t* rams_per_row);

/* Layout-2 model from the class-packed rows of the same WiSARD (the
 * horizontal packing of several RAMs into one RLWE, Sec. 5.1): row R of
 * model_out = sum over t < r, R r + t < k0 of X^(t 2^(L+a)) model_in[R r + t].
 * shape: the layout-2 shape; model_in: [k0][k1] RLWE trained with layout 1
 * (same s, l, a, perm_seed); model_out: [rows][k1] RLWE, overwritten, not
 * overlapping model_in.  Exact: training into layout 2 directly gives the
 * same bits.  Models of layout 2 merge with hw_rlwe_add like any other. */
hw_status hw_wisard_pack_rams(hw_ctx* ctx, const hw_wisard_shape* shape, const uint32_t* model_in,
                              uint32_t* model_out, hipStream_t stream);

/* The permutation pi_r of Def. 1 for `shape` (host output, s entries):
 * Fisher-Yates driven by the library's counter-based generator; the permuted
 * input is t[k] = x[pi[k]]. */
hw_status hw_permutation(const hw_wisard_shape* shape, uint32_t* perm_host);

/* ---- client side (Sec. 2.5.1), run on the device for throughput ---------- */

/* SecretKeyGen: ternary RLWE key s_k = (w64(seed, KEY, k) mod 3) - 1.
 * sk_dev: int32[N]. */
hw_status hw_keygen(hw_ctx* ctx, uint64_t seed, int32_t* sk_dev, hipStream_t stream);

/* EncRGSW of nbits bits (bits_dev: uint8 0/1, nbits entries); ciphertext
 * number ct_index0 + k encrypts bit k and is written at
 * rgsw_dev + k * rgsw_bytes.  Rows: 2D = 2 * digits * nq encryptions of 0,
 * the first D carrying bit * base^j on residue i of b, the next D on residue
 * i of a (row i*digits + j within a half).  Randomness: draw streams of the
 * library's generator keyed by `seed`, a function of (ciphertext, row) only. */
hw_status hw_encrypt_rgsw_bits(hw_ctx* ctx, const int32_t* sk_dev, const uint8_t* bits_dev,
                               uint64_t nbits, uint64_t seed, uint64_t ct_index0,
                               uint32_t* rgsw_dev, hipStream_t stream);

/* EncRLWE of `count` plaintext polynomials msg_dev[count][N] (uint64 in
 * [0, p); NULL encrypts zeros): b = a s + Delta msg + e.  Output
 * rlwe_dev[count] in the coefficient domain. */
hw_status hw_encrypt_rlwe(hw_ctx* ctx, const int32_t* sk_dev, const uint64_t* msg_dev,
                          uint64_t count, uint64_t seed, uint64_t ct_index0, uint32_t* rlwe_dev,
                          hipStream_t stream);

/* DecRLWE: msg_dev[count][N] = round(p (b - a s) / Q) mod p, the phase taken
 * through the CRT (round half up). */
hw_status hw_decrypt_rlwe(hw_ctx* ctx, const int32_t* sk_dev, const uint32_t* rlwe_dev,
                          uint64_t count, uint64_t* msg_dev, hipStream_t stream);

/* DecLWE: msg_dev[count] = round(p (b - <a, s>) / Q) mod p. */
hw_status hw_decrypt_lwe(hw_ctx* ctx, const int32_t* sk_dev, const uint32_t* lwe_dev,
                         uint64_t count, uint64_t* msg_dev, hipStream_t stream);

/* Copy `count` device-layout RGSW ciphertexts to the coefficient domain,
 * out_dev[count][2D][2][nq][N] (for checks against other implementations). */
hw_status hw_rgsw_export_canonical(hw_ctx* ctx, const uint32_t* rgsw_dev, uint64_t count,
                                   uint32_t* out_dev, hipStream_t stream);

/* ---- ring and ciphertext kernels ----------------------------------------- */

/* In-place negacyclic NTT of `count` polynomials polys_dev[count][nq][N]
 * (every residue transformed modulo its own prime).  inverse = 0: coefficient
 * domain -> evaluation domain in the library's internal order; inverse = 1:
 * back (including the 1/N factor).  Pointwise products in the evaluation
 * domain followed by the inverse give negacyclic products (Sec. 2.1). */
hw_status hw_ntt(hw_ctx* ctx, uint32_t* polys_dev, uint64_t count, int inverse,
                 hipStream_t stream);

/* External product (Sec. 2.5.1): out[k] = rgsw[k] [.] in[k] for k < count,
 * i.e. sum_{i,j} dec(b)_{i,j} C[i*digits+j] + sum_{i,j} dec(a)_{i,j}
 * C[D+i*digits+j] with the balanced base-2^log_base digits of the centered
 * residues (the last digit takes what is left above the others).
 * in_dev/out_dev: RLWE[count]; rgsw_dev: RGSW[count] in device layout.
 * out must not alias in. */
hw_status hw_external_product(hw_ctx* ctx, const uint32_t* rgsw_dev, const uint32_t* in_dev,
                              uint64_t count, uint32_t* out_dev, hipStream_t stream);

/* ---- server side: the hot path -------------------------------------------- */

/* Homomorphic training (Alg. 6) of n samples, accumulated into the model in
 * place.  Capacity: every sample adds Delta to one cell per RAM and to the
 * class counter, so the model decrypts correctly while it holds at most
 * p - 1 samples in total; the caller tracks that count for this call (the
 * serving engine tracks it for its models and refuses requests past it).  x_rgsw_dev: RGSW[n][s] of the unpermuted input bits; y_rgsw_dev:
 * RGSW[n][L] of the label bits, LSB first (L = ceil(log2 l)).  For sample i
 * and RAM j the IVP (Alg. 5) runs with input (0, Delta) on b = [label bits,
 * x[pi[j a + t]] for t < a_j] (a_j = min(a, s - j a)), creating only the
 * CDEMUX tree nodes that lead to a class below l (layout 0), or on
 * b = [x[pi[j a + t]] for t < a_j, label bits] with every node (layout 1);
 * each kept leaf is added to its row of model_dev[j] (RLWE[k0][k1],
 * coefficient domain; see hw_wisard_dims).
 * class_count_dev (one RLWE, may be NULL) receives the balancing counter
 * (Sec. 3.7.1): the IVP of the label bits alone.  Results are exact:
 * independent of chunking, sample order and launch configuration. */
hw_status hw_wisard_train_encrypted(hw_ctx* ctx, const hw_wisard_shape* shape,
                                    const uint32_t* x_rgsw_dev, const uint32_t* y_rgsw_dev,
                                    uint64_t n, uint32_t* model_dev, uint32_t* class_count_dev,
                                    hipStream_t stream);

/* Bytes of the fixed device scratch behind hw_wisard_train_encrypted_noalloc. */
#define HW_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * training as hw_wisard_train_encrypted, same arguments and same bits, but
 * the call allocates nothing.  Its workspace (the per-sample IVP leaf blocks)
 * and the device permutation live in a fixed device array of
 * HW_NOALLOC_SCRATCH_BYTES bytes, which each GPU holds from the first call on
 * it until the process ends; samples run in sub-batches that fit it.  The
 * kernels run their settled schedules (forced with hw_tune_set, or chosen by
 * earlier tuned calls; else the default) and no timing events are recorded.
 * HW_EINVAL when one sample's workspace plus the permutation exceeds the
 * array ((k0 + 1)(2^z + 1) RLWE per sample: the tiny, Wisconsin- and
 * MNIST-shaped sets fit, the HAM-shaped one does not).  Every call on one GPU
 * shares that GPU's array, so calls whose work overlaps on one GPU race: the
 * caller serialises them (one stream, or a wait between streams). */
hw_status hw_wisard_train_encrypted_noalloc(hw_ctx* ctx, const hw_wisard_shape* shape,
                                            const uint32_t* x_rgsw_dev, const uint32_t* y_rgsw_dev,
                                            uint64_t n, uint32_t* model_dev, uint32_t* class_count_dev,
                                            hipStream_t stream);

/* Homomorphic inference, PD-act branch (Alg. 7).  Layout 0: for each
 * sample, RAM j and label c < l, the Vertical Packing (Alg. 3, read as the
 * inverse of the IVP layout) of model row j with the label bits of c in the
 * clear and the sample's permuted tuple bits encrypted, then
 * ExtractLWE(., 0).  Layout 1: for each sample and RAM j one Vertical Packing
 * over the tuple bits (label bits clear zeros), then ExtractLWE(., c
 * 2^(a_j - z)) for every c < l (Sec. 2.5.1).  Either way
 * ram_scores_dev: LWE[n][l][k0], decrypting to the cell of class c addressed
 * by the sample in RAM j; class_scores_dev (may be NULL): LWE[n][l], the sums
 * over j.  model_dev is read only. */
hw_status hw_wisard_infer_encrypted(hw_ctx* ctx, const hw_wisard_shape* shape,
                                    const uint32_t* model_dev, const uint32_t* x_rgsw_dev,
                                    uint64_t n, uint32_t* ram_scores_dev,
                                    uint32_t* class_scores_dev, hipStream_t stream);

/* PackingKeySwitching (Sec. 2.5.1; Alg. 7 returns the PD-act scores packed
 * by it): k LWE ciphertexts (a^(i), b^(i)) under the RLWE key's coefficients
 * (as ExtractLWE leaves them) become one RLWE whose phase is sum_i phase_i X^i,
 * so it decrypts (hw_decrypt_rlwe) to the k messages in coefficients 0..k-1
 * and zeros after.
 * Key: K[j][r] = RLWE_s(s_j G_r) for j < N and the D = 5 nq RNS gadget rows
 * (G_r = 64^t in residue g for r = 5 g + t, 0 in the others).  Row (j, r) is
 * drawn like row r of RGSW ciphertext j with D rows (a by its evaluations,
 * see hw_encrypt_rgsw_bits) from `seed`.  Device layout [N][D][2][nq][N]
 * uint32 in the evaluation domain: N D 8 nq N bytes (640 MiB at N = 2048,
 * nq = 2), caller-owned.  hw_pks_key_export_canonical writes the same rows in
 * the coefficient domain (tests).
 * Packing: out = (0, sum_i b^(i) X^i) - sum_{j,r} P_{j,r} K[j][r], where
 * P_{j,r} = sum_i d_r(a^(i)_j) X^i collects the balanced base-64 digits (5 per
 * residue, on every context: the paper gives PackingKeySwitching
 * decomposition parameters of its own, Sec. 4).  lwe_dev: [count][k] LWE; out_dev: [count]
 * RLWE (coefficient domain); 1 <= k <= N (HW_EINVAL otherwise). */
hw_status hw_pks_keygen(hw_ctx* ctx, const int32_t* sk_dev, uint64_t seed, uint32_t* key_dev,
                        hipStream_t stream);
hw_status hw_pks_key_export_canonical(hw_ctx* ctx, const uint32_t* key_dev, uint32_t* out_dev,
                                      hipStream_t stream);
hw_status hw_pack_lwe(hw_ctx* ctx, const uint32_t* key_dev, const uint32_t* lwe_dev, uint32_t k,
                      uint64_t count, uint32_t* out_dev, hipStream_t stream);

/* ---- programmable bootstrapping: Activate and EncryptedArgMax (OTF-act) --------- */

/* The paper evaluates the activation of the inference scores (OTF-act,
 * Sec. 3.5.2) and the final ArgMax (Alg. 7) with the programmable
 * bootstrapping, taken as a black box (Sec. 2.5.3).  Here the bootstrap
 * decides one sign at a time, and the functions are circuits of such
 * bootstraps and exact linear operations on LWE ciphertexts, all under the
 * ring key s (LWE [prime][N+1] as ExtractLWE leaves them), modulus Q.
 *
 * Bootstrapping key (hw_pbs_keygen): for the first n key coefficients,
 * bsk[2k] = RGSW([s_k = 1]) and bsk[2k+1] = RGSW([s_k = -1]), ciphertexts 2k
 * and 2k+1 of hw_encrypt_rgsw_bits' stream `seed`; [2n] RGSW in device
 * layout, caller-owned (2n hw_sizes().rgsw bytes: 2.7 GB at N = 2048, nq = 2,
 * n = N).  1 <= n <= N. */
hw_status hw_pbs_keygen(hw_ctx* ctx, const int32_t* sk_dev, uint64_t seed, uint32_t n, uint32_t* bsk_dev,
                        hipStream_t stream);

/* Bootstrapping through a key switch (the TFHE setting of Sec. 2.5.3 keeps an
 * LWE key S0 in B^n beside the ring key): the LWE ciphertext (ring key,
 * modulus Q) is switched to modulus 2^32 (round(2^32 x / Q)), key-switched
 * to a binary key s1 of n coefficients, switched to 2N, and blind-rotated
 * with one CMUX per coefficient of s1 (n external products instead of the
 * ring key's 2n per coefficient); the output is an LWE under the ring key as
 * before.  Key switch: each switched mask coefficient a'_k is rounded to its
 * top 24 bits and cut into 6 balanced base-16 digits d_j (weight 2^(28-4j));
 * out = (0, b') - sum_{k,j} d_j(a'_k) KSK[6k + j] mod 2^32, with KSK[6k + j]
 * an LWE under s1 at modulus 2^32 of s_k 2^(28-4j) whose error is 2^13 c + u
 * (c the Gaussian sample, u uniform in [-2^12, 2^12)).  The sum over the 6N
 * digits runs as a contraction of signed bytes on the matrix cores (the
 * 32-bit key words cut into four signed bytes), exact mod 2^32.
 * hw_pbs_ks_keygen: s1_i = bit 0 of draw i of stream (seed, domain 7)
 * into lwe_key_dev (uint8 [n], device); bsk_dev = RGSW(s1_i) as ciphertexts
 * 0..n-1 of hw_encrypt_rgsw_bits' stream `seed`.  On one prime they use the
 * context's gadget (hw_sizes().rgsw bytes each).  On two or more primes they
 * use 2 balanced digits of 15 bits per prime: 2 x 2 nq RLWE rows per RGSW
 * (row d < 2 nq adds m 2^(15 (d % 2)) to the constant term of residue d / 2
 * of b, row 2 nq + d to that of a), drawn like hw_encrypt_rgsw_bits' rows of
 * a ciphertext with 2 x 2 nq rows, in the device layout
 * (hw_rgsw_export_canonical exports them as rows); the blind rotation's
 * noise stays near 2^27 at N = 2048 with 16 forward NTTs per product
 * instead of 40.  ksk_dev = the key in the
 * contraction's layout, signed bytes [cols][6N], row l (n + 1) + i holding
 * byte l of word i of every KSK row (A_r then B_r at i = n; A_r[i] = 32-bit
 * draw r n + i of (seed, 8), the error from 64-bit draws 2r and 2r + 1 of
 * (seed, 9)), cols = 4 (n + 1) rounded up to 64, the padding rows zero.
 * Sizes from hw_pbs_ks_sizes.  1 <= n <= 8192. */
hw_status hw_pbs_ks_sizes(const hw_ctx* ctx, uint32_t n, uint64_t* bsk_bytes, uint64_t* ksk_bytes);
hw_status hw_pbs_ks_keygen(hw_ctx* ctx, const int32_t* sk_dev, uint64_t seed, uint32_t n, uint8_t* lwe_key_dev,
                           uint32_t* bsk_dev, int8_t* ksk_dev, hipStream_t stream);

/* The key every bootstrapping call takes: ksk == NULL for the ring-key
 * bootstrap (bsk from hw_pbs_keygen, 2n RGSW, n <= N ring coefficients),
 * otherwise the key-switched one (bsk and ksk from hw_pbs_ks_keygen, n the
 * LWE key's length). */
typedef struct {
  const uint32_t* bsk;  /* device */
  const int8_t* ksk;    /* device or NULL */
  uint32_t n;
  uint32_t reserved;    /* 0 */
} hw_boot_key;

/* Bootstrap with the constant test polynomial V (v: its nq residues, host)
 * of `count` LWE ciphertexts whose mask is zero past its first n
 * coefficients (n = N for ExtractLWE outputs; bsk from hw_pbs_keygen with at
 * least n coefficients): the mask and body switched to round(2N x / Q) mod 2N
 * (x read through the CRT, half up), ACC = (0, X^{-b~} V (1 + X + ... +
 * X^{N-1})), then for k < n ACC <- CMUX(bsk[2k], X^{a~_k} ACC, ACC) and
 * ACC <- CMUX(bsk[2k+1], X^{-a~_k} ACC, ACC), out = ExtractLWE(ACC, 0): an
 * LWE of V when the switched phase lies in [0, N), of -V otherwise.  With a
 * key-switched key (key->ksk set) the input may have a full mask; its switch
 * to 2N is the one of hw_pbs_ks_keygen's key switch and the blind rotation
 * is ACC <- CMUX(bsk[i], X^{a~_i} ACC, ACC) for i < key->n.
 * lwe_dev, out_dev: [count] LWE, not overlapping. */
hw_status hw_pbs(hw_ctx* ctx, const hw_boot_key* key, const uint32_t* lwe_dev, uint64_t count,
                 const uint32_t* v_host, uint32_t* out_dev, hipStream_t stream);

/* Activate with the threshold activation (bin of PD-act with thr = T - 1):
 * out[j] encrypts [m_j >= T] for the message m_j in [0, p) of lwe[j] (phase
 * ~ floor(Q/p) m_j, p = the context's plaintext modulus, p >= 8,
 * 1 <= T <= p), with phase ~ 2 V_o [m_j >= T], V_o = floor(floor(Q / p_o) / 2),
 * p_o = 2^log_p_out (decrypt with plaintext modulus p_o).  Steps (P = log2 p,
 * V_b = floor(floor(Q/p) / 2), V_c = floor(Q/16), all on every ciphertext):
 *   bits, k = 0..P-1: y = 2^(P-1-k) x + floor(Q/4); E_k = V_b - PBS(y, V_b);
 *     x = x - 2^k E_k  (E_k ~ 2 V_b bit_k of m, least significant first);
 *   carry of m + (p - T), t = p - T, c = 0, k = 0..P-1:
 *     z = 2^(P-3) E_k + c - (V_c if bit k of t else 3 V_c);
 *     c = PBS(z, V) + V with V = V_o for k = P-1, else V_c.
 * Each bootstrap decides a sign with a margin of N/8 switched positions or
 * more.  2P bootstraps per ciphertext; lwe_dev, out_dev: [count] LWE. */
hw_status hw_activate_ge(hw_ctx* ctx, const hw_boot_key* key, const uint32_t* lwe_dev, uint64_t count,
                         uint64_t T, uint32_t log_p_out, uint32_t* out_dev, hipStream_t stream);

/* The activations of Sec. 2.4.2 that the paper's models use (its parameter
 * table: bin with a threshold, log, b-log), as bootstrapped circuits over
 * `count` LWE (phase ~ floor(Q/p) m, m in [0, p), p >= 8), output phase
 * ~ 2 V_o f(m), V_o = floor(floor(Q / 2^log_p_out) / 2), 1 <= log_p_out <= 60:
 *   HW_ACT_GE   f(m) = [m >= param], 1 <= param <= p (hw_activate_ge; bin
 *               with thr = param - 1), 2P bootstraps;
 *   HW_ACT_LOG  f(m) = floor(log2(m + 1)) (param ignored), 2P bootstraps;
 *   HW_ACT_BLOG f(m) = min(floor(log2(m + 1)), param), param >= 1 (param >= P
 *               is log), 2P - 1 bootstraps for param < P - 1.
 * log and b-log need log_p_out >= 3.  They read x' = x + (0, floor(Q/p)),
 * which encrypts m' = m + 1 mod p (0 only for m = p - 1); E = the bits of m'
 * (as in hw_activate_ge); with o_i = [m' >= 2^i] = the OR of bits i..P-1,
 * f = sum_{i=1}^{c} o_i + c (1 - o_0), c = P (log, the sum up to P - 1) or
 * the cap.  The ORs run from the top: chain value o = 2^(P-3) E_(P-1) (scale
 * ~Q/8); for i = P-2 .. 0, z_i = 2^(P-3) E_i + o - V_c, w_i = PBS(z_i, V_o) +
 * V_o (o_i at the output scale) and, for i >= 1, o = 2^(log_p_out - 3) w_i
 * (back at ~Q/8); o_(P-1), when the sum needs it, is PBS(2^(P-3) E_(P-1) -
 * V_c, V_o) + V_o.  lwe_dev, out_dev: [count] LWE.  HW_EINVAL for a kind,
 * param or log_p_out out of range, before anything runs. */
#define HW_ACT_GE 0u
#define HW_ACT_LOG 1u
#define HW_ACT_BLOG 2u
hw_status hw_activate(hw_ctx* ctx, const hw_boot_key* key, const uint32_t* lwe_dev, uint64_t count,
                      uint32_t kind, uint64_t param, uint32_t log_p_out, uint32_t* out_dev, hipStream_t stream);

/* EncryptedArgMax (Alg. 7): for each of `count` samples, the l class scores
 * u[j][c] (phase ~ 2 V_i s_c, V_i = floor(floor(Q / p_in) / 2),
 * p_in = 2^log_p_in >= 8, every s_c < p_in / 2) give out[j], an LWE of the
 * index of the largest score, ties to the lowest index, with phase
 * ~ 2 V_x index, V_x = floor(floor(Q / 2^(L+1)) / 2), L = ceil(log2 l)
 * (decrypt with plaintext modulus 2^(L+1)).  Steps (P = log_p_in): for
 * a < b, D = u_a - u_b + (p_in/2) 2 V_i, E = the bits of D (as in
 * hw_activate_ge, at p_in), G(a, b) = 2^(P-3) E_(P-1) (= [s_a >= s_b]),
 * G(b, a) = 2^(P-3) 2 V_i - G(a, b); W_a = 2 G(a, b) for l = 2, else the
 * AND of G(a, b) over b != a in order (acc = G(a, b_1); acc = PBS(acc +
 * G(a, b_j) - 3 V_c, V) + V with V = V_x for the last b_j, else V_c);
 * index = sum_a a W_a.  u_dev: [count][l] LWE; out_dev: [count] LWE.
 * 2 <= l <= 64, 3 <= log_p_in <= 20. */
hw_status hw_encrypted_argmax(hw_ctx* ctx, const hw_boot_key* key, const uint32_t* u_dev,
                              uint64_t count, uint32_t l, uint32_t log_p_in, uint32_t* out_dev,
                              hipStream_t stream);

/* Per-class sums of per-RAM LWE scores (Alg. 2's sum over RAMs, on
 * ciphertexts): sums[j][c] = sum over r < k0 of scores[j][c][r], residue by
 * residue, e.g. of hw_activate_ge outputs before hw_encrypted_argmax.
 * scores_dev: [n][l][k0] LWE; sums_dev: [n][l] LWE. */
hw_status hw_class_sums(hw_ctx* ctx, const uint32_t* scores_dev, uint64_t n, uint32_t l, uint32_t k0,
                        uint32_t* sums_dev, hipStream_t stream);

/* FM-act (Sec. 3.5.3): the activation applied once to every cell of a
 * trained model, so that inference on the result (hw_wisard_infer_encrypted,
 * hw_class_sums, hw_encrypted_argmax: Alg. 7's FM-act branch) needs no
 * bootstrap.  For every model RLWE, coefficients 0..K-1 are taken out as LWE
 * (ExtractLWE at each coefficient), activated as in hw_activate (kind and
 * param, output plaintext modulus 2^log_p_out) and packed back into one RLWE at the
 * same coefficients (hw_pack_lwe with pks_key_dev); coefficients from K on
 * decrypt to 0.  K covers every cell a RAM's index can address: 2^min(L + a,
 * log2 N) for layouts 0 and 1, N for layout 2.  model_dev, out_dev: the
 * model of `shape` (hw_wisard_model_rows x k1 RLWE, coefficient domain,
 * plaintext modulus the context's p); out_dev may be model_dev itself (in
 * place) but must not overlap it otherwise.  K times the activation's
 * bootstraps per RLWE.  The call works through the rows in chunks of about 65,536
 * cells, allocates two LWE buffers of that many cells for the call and
 * waits for the stream before returning.  Errors as hw_activate and
 * hw_pack_lwe, checked before anything runs. */
hw_status hw_fm_act(hw_ctx* ctx, const hw_wisard_shape* shape, const hw_boot_key* key,
                    const uint32_t* pks_key_dev, const uint32_t* model_dev, uint32_t kind, uint64_t param,
                    uint32_t log_p_out, uint32_t* out_dev, hipStream_t stream);

/* Merge of models trained apart (Sec. 3.7.2: Integer WiSARD models of
 * federated entities are merged by adding their RAMs; the merged model is
 * the one centralised training on the union would give, bit for bit, since
 * training adds each sample's contribution mod q_i): dst[k] += src[k] for
 * count RLWE ciphertexts, residue by residue.  Also adds class counters and
 * continues training from a checkpoint.  dst and src: device, [count] RLWE,
 * 16-byte aligned; dst may equal src (doubling); otherwise they must not
 * overlap.  HW_EINVAL for null or misaligned buffers. */
hw_status hw_rlwe_add(hw_ctx* ctx, uint32_t* dst_dev, const uint32_t* src_dev, uint64_t count,
                      hipStream_t stream);

/* ---- batching ----------------------------------------------------------------- */

typedef struct {
  hw_wisard_shape shape;
  const uint32_t* x_rgsw_dev;   /* [n][s] RGSW of the input bits */
  const uint32_t* y_rgsw_dev;   /* [n][L] RGSW of the label bits (may be NULL when L = 0) */
  uint64_t n;                   /* samples */
  uint32_t* model_dev;          /* [k0][k1] RLWE, accumulated in place */
  uint32_t* class_count_dev;    /* one RLWE or NULL */
} hw_train_job;

/* Batched homomorphic training (Alg. 6 for every job).  The jobs share this
 * context's parameter set and may differ in shape and size.  They run as one
 * persistent launch over one queue of (job, RAM, piece) items, longest first:
 * a piece is a run of consecutive samples of the job, whose IVP outputs the
 * workgroup adds into the model row itself (first piece of the RAM) or into
 * a workspace accumulator (further pieces), added into the model by one
 * exact modular reduction afterwards.  Pieces are sized for load balance and
 * lengthened until their accumulators fit the workspace budget, so the
 * workspace does not grow with the number of samples.  The result of each
 * job is bit-identical to hw_wisard_train_encrypted on it.  Jobs must not
 * share model or counter buffers. */
hw_status hw_batch_train(hw_ctx* ctx, const hw_train_job* jobs, uint32_t njobs, hipStream_t stream);

/* A batch plan: the queue and pieces of hw_batch_train for a fixed list of
 * jobs, computed once, with their tables uploaded to the device and the
 * launches (queue reset, persistent training launch, reduction of the
 * accumulators) captured into one HIP graph.  hw_batch_plan_launch replays
 * that graph on `stream`: it reads the jobs' input ciphertexts as they are
 * at replay time and adds their samples into the models, exactly as
 * hw_batch_train on the same jobs would, with no host work.  The plan owns
 * its workspace (hw_batch_plan_info: bytes; also the queue items, the most
 * pieces of any RAM and the external products of one replay) and tables;
 * the job buffers stay caller-owned and must outlive the plan, and so must
 * the context.  Replays of one plan must not overlap (they share the
 * workspace).  Errors: those of hw_batch_train, plus HW_EDEVICE if capture
 * fails. */
typedef struct hw_batch_plan hw_batch_plan;
hw_status hw_batch_plan_create(hw_ctx* ctx, const hw_train_job* jobs, uint32_t njobs,
                               hw_batch_plan** plan);
hw_status hw_batch_plan_launch(hw_batch_plan* plan, hipStream_t stream);
hw_status hw_batch_plan_info(const hw_batch_plan* plan, uint64_t* items, uint32_t* max_pieces,
                             double* external_products, uint64_t* workspace_bytes);
/* Waits for the device to finish the plan's replays, then frees it. */
void hw_batch_plan_destroy(hw_batch_plan* plan);

/* One job of hw_batch_run: training (Alg. 6) or inference (Alg. 7, PD-act
 * branch) of n samples under the parameter set ctxs[ctx_index].  The buffers
 * mean what they mean for hw_wisard_train_encrypted (kind 0: x_rgsw, y_rgsw,
 * model accumulated in place, class_count or NULL) and
 * hw_wisard_infer_encrypted (kind 1: model read, x_rgsw, ram_scores,
 * class_scores or NULL); the fields of the other kind are ignored. */
typedef struct {
  uint32_t ctx_index;           /* index into the context list */
  uint32_t kind;                /* 0 = train, 1 = infer */
  hw_wisard_shape shape;
  const uint32_t* x_rgsw_dev;   /* [n][s] RGSW of the input bits */
  const uint32_t* y_rgsw_dev;   /* train: [n][L] RGSW of the label bits (NULL when L = 0) */
  uint64_t n;                   /* samples */
  uint32_t* model_dev;          /* [rows][k1] RLWE: train accumulates into it, infer reads it */
  uint32_t* class_count_dev;    /* train: one RLWE or NULL */
  uint32_t* ram_scores_dev;     /* infer: [n][l][k0] LWE */
  uint32_t* class_scores_dev;   /* infer: [n][l] LWE or NULL */
} hw_job;

/* A batch of training and inference jobs over several parameter sets.  For
 * each context, in the order of `ctxs`: its training jobs run as one
 * persistent launch (exactly hw_batch_train on them), then its inference jobs
 * as one persistent launch over a queue of (job, RAM, label, piece of
 * samples) items, longest first, each workgroup running the Vertical Packing
 * of its item's samples one after another in private slots; per-class sums
 * follow for the jobs that ask for them.  A launch is compiled for one ring
 * degree, prime count and RGSW gadget, so it never spans two contexts: the contexts'
 * launches follow one another on `stream`.  An inference job therefore sees
 * every training job of its context in the same batch.  Every job's result
 * is bit-identical to the single-job call on it.  Training jobs on the same
 * model are rejected (layout 2 is rejected for training as in
 * hw_batch_train), as are jobs whose outputs overlap each other or a model an
 * inference job reads (HW_EINVAL); the checks run before anything is
 * enqueued.  The contexts' calls are serialised as for any call on them. */
hw_status hw_batch_run(hw_ctx* const* ctxs, uint32_t nctx, const hw_job* jobs, uint32_t njobs,
                       hipStream_t stream);

/* ---- serving engine (continuous batching) ------------------------------------- */

/* A request loop on one device: train and infer requests against resident
 * models are cut into chunks of samples; a scheduler thread starts a chunk
 * as soon as a stream slot is free and the chunk's device footprint (input
 * ciphertexts, workspace, scores) fits in the engine's arena.  Requests are
 * served in the configured order (first come, first served, or the least
 * remaining work first): the first request in that order takes every free
 * slot it can use, later ones the slots it cannot.  Requests on one model keep submission
 * order: a training request starts after every earlier request on its model
 * completed (its chunks run one after another), an inference request once
 * every earlier request on its model is an inference (inferences only read
 * the model, so several overlap); requests on different models overlap on
 * the device.  Results depend only on the
 * model state and the request, so each is bit-identical alone and in a mix.
 * For measurement the engine also plays the client: it encrypts request bits
 * on the device with the key it was given and returns decrypted PD-act cells. */
typedef struct hw_engine hw_engine;

typedef struct {
  uint32_t slots;        /* chunks in flight at once, one HIP stream each: 1..16 */
  uint32_t chunk;        /* samples per chunk, >= 1 */
  uint32_t max_s;        /* largest input width served (host staging size) */
  uint32_t max_cells;    /* largest l * k0 served (host staging size) */
  uint64_t arena_bytes;  /* device memory for the chunks in flight */
  uint32_t order;        /* HW_ORDER_FIFO: requests in submission order;
                            HW_ORDER_SHORTEST: the request with the fewest external
                            products left to start first (its unstarted samples times its
                            model's products per sample for its kind), ties in submission order */
  uint32_t reserved;     /* 0 */
} hw_engine_config;
#define HW_ORDER_FIFO 0u
#define HW_ORDER_SHORTEST 1u

typedef struct {
  uint32_t job;                /* id from hw_engine_add_job */
  uint32_t kind;               /* 0 = train, 1 = infer */
  const uint8_t* bits_host;    /* [n][s] input bits; host, read until the request completes */
  const uint8_t* labels_host;  /* train: [n][L] label bits, LSB first; NULL when L = 0 */
  uint64_t n;                  /* samples */
  uint64_t enc_seed;           /* the request's encryption seeds are derived from it
                                  (hw_request_seeds): inputs use seed_x, labels seed_y; ciphertext
                                  index = sample * s + bit (sample * L + bit for labels).  Requests
                                  must not share an enc_seed (their draws would repeat). */
  uint64_t* cells_host;        /* infer: [n][l][k0] decrypted per-RAM scores */
} hw_request;

enum { HW_REQ_QUEUED = 0, HW_REQ_RUNNING = 1, HW_REQ_DONE = 2, HW_REQ_FAILED = 3, HW_REQ_CANCELLED = 4 };

/* Create an engine for `params` on `device` with the client key sk_dev
 * (caller-owned, device, valid until destroy).  Fails with HW_ENOMEM when the
 * arena cannot be allocated. */
hw_status hw_engine_create(const hw_params* params, int device, const int32_t* sk_dev,
                           const hw_engine_config* config, hw_engine** out);

/* Wait for the chunks in flight, stop the scheduler and free the engine. */
void hw_engine_destroy(hw_engine* engine);

/* The two encryption seeds of a request (the engine's client step): the
 * 64-bit draws 0 and 1 of the library's generator (Philox4x32-10, the
 * counter-based generator of every random draw here) in domain 6 keyed by
 * enc_seed.  Input and label streams of one request, and the streams of
 * requests with different enc_seed, are thereby keyed apart: no RLWE draw
 * is reused under the engine's one key (Sec. 2.5 security rests on fresh
 * randomness per ciphertext). */
hw_status hw_request_seeds(uint64_t enc_seed, uint64_t* seed_x, uint64_t* seed_y);

/* Register a resident model (caller-owned device buffers, [k0][k1] RLWE and
 * an optional class counter) of the given shape that already holds `trained`
 * samples (0 for a zeroed model); *job_id names it.  Call before submitting
 * requests that use it.  HW_EINVAL when trained > p - 1. */
hw_status hw_engine_add_job(hw_engine* engine, const hw_wisard_shape* shape, uint32_t* model_dev,
                            uint32_t* class_count_dev, uint64_t trained, uint32_t* job_id);

/* Queue a request.  HW_EBUSY: one chunk of it would not fit in the arena
 * (it could never be admitted); HW_EINVAL: bad job or buffers, or a training
 * request that could take its model past p - 1 samples.  Training adds Delta
 * per sample to one cell of every RAM and to the class counter, so a count
 * of p would wrap to 0 (Sec. 2.5.1 encoding, plaintexts mod p); the engine
 * counts every admitted training request's samples against the model. */
hw_status hw_engine_submit(hw_engine* engine, const hw_request* request, uint64_t* request_id);

/* Samples counted against a model (trained plus admitted training requests)
 * and the capacity p - 1. */
hw_status hw_engine_job_samples(hw_engine* engine, uint32_t job, uint64_t* samples, uint64_t* capacity);

/* State of a request (HW_REQ_*) and, once finished, its latency from submission. */
hw_status hw_engine_poll(hw_engine* engine, uint64_t request_id, int* state, double* latency_ms);

/* Block until the request has finished (done, failed or cancelled). */
hw_status hw_engine_wait(hw_engine* engine, uint64_t request_id, int* state, double* latency_ms);

/* Cancel a request: no further chunks start; chunks in flight complete (a
 * cancelled training request may have updated the model with them). */
hw_status hw_engine_cancel(hw_engine* engine, uint64_t request_id);

/* Counters: chunks started, peak arena bytes in use, peak chunks in flight. */
hw_status hw_engine_stats(hw_engine* engine, uint64_t* chunks, uint64_t* peak_arena_bytes,
                          uint32_t* peak_inflight);

/* ---- schedule tuning ------------------------------------------------------------ */

/* Kernels with more than one launch schedule; every variant computes the
 * same bits, only its speed differs:
 *   "train"        0: 2-D grid, the RAMs of a sample on consecutive workgroups;
 *                  1: 1-D grid, XCD x (workgroup id mod 8) takes the x-th
 *                     eighth of the (sample, RAM) items (label ciphertexts of
 *                     a sample stay in one XCD's L2);
 *                  2, 3 (N = 4096 only): 0 and 1 compiled for 4 waves per
 *                     SIMD instead of 3 (two 512-thread workgroups per CU,
 *                     a few registers spilled)
 *   "infer"        0: 3-D grid (RAM, label, sample); 1: 1-D grid, the labels of
 *                     a (sample, RAM) adjacent, grouped by XCD as above;
 *                  2, 3 (N = 4096 only): as for "train"
 *   "train_batch"  0: 3 waves per SIMD; 1 (N = 4096 only): 4 waves per SIMD
 *   "ntt"          v: 2^v polynomials per workgroup (v < 4), the twiddle table
 *                     copied to LDS once for all of them (forward transforms)
 *   "ntt_inverse"  the same for inverse transforms
 *   "encrypt_rgsw" 0, 1, 2: 1, 2 or 5 rows of an RGSW per workgroup
 * By default each is tuned online per context: its first launches cycle
 * through the variants, timed with HIP events on the launch stream, until
 * each variant has two timings; the variant with the least time per unit of
 * work (external products, polynomials, rows) is then used for the rest of
 * the context's life (by hw_wisard_*, hw_batch_*, hw_ntt and
 * hw_encrypt_rgsw_bits, and by a serving engine's own context).  Only launches large enough to fill the chip are
 * timed (50,000 external products, 16,384 polynomials, 20,000 RGSW rows);
 * smaller ones, and launches under stream capture, use the best variant so
 * far (variant 0 before any timing).  The environment variable HWISARD_TUNE=0 (read at context
 * creation) turns tuning off: variant 0 everywhere. */

/* Force `variant` for `kernel` (-1: forget the timings and tune again).
 * HW_EINVAL for an unknown kernel or a variant out of range. */
hw_status hw_tune_set(hw_ctx* ctx, const char* kernel, int variant);

/* The variant in use (-1 while still tuning), the number of timings taken
 * and the number of variants. */
hw_status hw_tune_get(hw_ctx* ctx, const char* kernel, int* variant, int* timings, int* count);

/* Description of a variant, or NULL for an unknown kernel or variant. */
const char* hw_tune_variant_name(const char* kernel, int variant);

/* ---- device peak probes (measurement) ----------------------------------------- */

/* Measure a peak rate of device `device` on `stream` (waits for it):
 *   "triad"          a = b + k c over three uint32 arrays of `size` bytes each
 *                    (library-allocated, freed before return); *rate = bytes
 *                    moved per second (2 size read + size written), best of 5;
 *   "v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32"
 *                    eight independent chains of that one instruction per
 *                    thread, 8 waves per SIMD on every CU, `size` loop trips
 *                    of 128 instructions (0: 4096); *rate = lane-instructions
 *                    per second (64 per wave instruction), best of 3.
 * *ms (may be NULL): the best launch time.  These are the peaks the hot-path
 * kernels' rooflines are priced against besides the published ones. */
hw_status hw_microbench(int device, const char* kind, uint64_t size, double* rate, double* ms,
                        hipStream_t stream);

/* ---- per-kernel timing ------------------------------------------------------ */

/* While enabled, every kernel launch made by the calls of this context is
 * bracketed by a pair of HIP events recorded on the caller's stream.  Kernel
 * names: "train", "reduce", "train_batch", "reduce_batch", "batch_plan" (a whole
 * plan replay), "infer", "class_sums", "encrypt_rgsw", "encrypt_rlwe",
 * "decrypt_rlwe", "decrypt_lwe", "xp", "ntt", "rlwe_add",
 * "encrypt_pks", "pack_lwe", "pbs", "activate", "argmax", "extract_cells". */
hw_status hw_profile_enable(hw_ctx* ctx, int enable);

/* Waits for the recorded events and returns, for kernel `name`, the summed
 * event time in ms, the number of launches and the algorithmic work those
 * launches did: external products for "train", "infer" and "xp", ciphertext
 * rows for the encryptions, polynomials for "ntt" and the decryptions, model
 * or output words for the reductions.  Unknown names give zeros. */
hw_status hw_profile_read(hw_ctx* ctx, const char* name, double* total_ms, uint64_t* launches,
                          double* work);

/* Drop every accumulated record. */
hw_status hw_profile_reset(hw_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HWISARD_H */
