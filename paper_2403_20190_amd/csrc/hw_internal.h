// hw_internal.h -- argument blocks shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hw_device.h"

namespace hw {

// CRT constants for decryption: phi = sum_i [phi_i * inv_i]_{q_i} * M_i mod Q
struct CrtTab {
  uint64_t Q_lo, Q_hi;          // Q = prod q_i
  uint64_t M_lo[MAXQ], M_hi[MAXQ];  // M_i = Q / q_i
  uint32_t inv[MAXQ];           // (Q/q_i)^{-1} mod q_i
  uint64_t half_lo, half_hi;    // floor(Q / 2)
  uint64_t p;                   // plaintext modulus (power of two)
};

struct Cdt {
  uint64_t T[42];
  // guide of the search (CDT_GUIDE_SIZE bytes, device): entry b, for the
  // draws r with r >> (63 - CDT_GUIDE_BITS) == b, holds the number of
  // T[j] <= b 2^(63 - CDT_GUIDE_BITS) (j <= 40), plus CDT_GUIDE_WIDE when
  // more than two T[j] fall inside that bucket of draws
  const uint8_t* guide;
};
constexpr uint32_t CDT_GUIDE_BITS = 12, CDT_GUIDE_SIZE = 1u << CDT_GUIDE_BITS, CDT_GUIDE_WIDE = 0x80;

struct EncArgs {
  const int32_t* sk;        // [N]
  const uint32_t* sk_hat;   // [NQ][N] evaluation domain (layout P=3), then [NQ][N] Shoup companions
  const uint8_t* bits;      // RGSW: one bit per ciphertext
  const uint64_t* msg;      // RLWE: [count][N] or nullptr
  uint32_t* out;
  uint64_t seed;
  uint64_t ct0;             // ciphertext index of the first output
  uint32_t log_base;
};

struct TrainArgs {
  const uint32_t* x_rgsw;   // [n][s] RGSW
  const uint32_t* y_rgsw;   // [n][L] RGSW
  const uint32_t* perm;     // [s]
  uint32_t* out;            // [n_sub][k0 + 1][kt + 1] RLWE (per-sample IVP leaves + input slot)
  uint64_t rgsw_words;
  uint64_t i0;              // first sample of the sub-batch
  uint32_t s, a, L, k0, k1;
  uint32_t l, kt;           // classes; 2^z leaves of a full RAM's tree (slots per block: kt + 1)
  uint32_t nram, nsub;      // grid: nram RAM items (k0, + 1 for the counter) x nsub samples
  uint32_t map;             // 0: 2-D grid (RAM, sample); 1: 1-D, XCD-grouped
  uint32_t layout;          // model layout: 0 label-pruned rows, 1 class-packed rows
  uint32_t tree;            // k_train: 1 runs the CDEMUX tree in the chain's workgroup, 0 the chain only
  uint32_t lev, smax;       // k_train_level: the tree level and the most live splits a RAM has at it
};

struct ReduceArgs {
  const uint32_t* out;      // as TrainArgs::out
  uint32_t* model;          // [k0][k1] RLWE (live leaves, Def. 2 rows)
  uint32_t* cnt;            // one RLWE or nullptr
  uint64_t n_sub;
  uint32_t s, a, L, k0, k1, logN, N, nq;
  uint32_t l, kt;           // classes; tree leaves per block (block = kt + 1 slots)
  uint32_t layout;          // as TrainArgs::layout
};

struct InferArgs {
  const uint32_t* model;    // [k0][k1] RLWE
  const uint32_t* x_rgsw;   // [n][s] RGSW
  const uint32_t* perm;     // [s]
  uint32_t* scores;         // [n][l][k0] LWE
  uint32_t* scratch;        // [n_sub][nlab][k0][slots + 1] RLWE
  uint64_t rgsw_words;
  uint64_t i0;
  uint32_t s, a, L, l, k0, k1, slots;
  uint32_t nsub;            // samples of this launch
  uint32_t map;             // 0: 3-D grid (RAM, label, sample); 1: 1-D, labels adjacent, XCD-grouped
  uint32_t layout;          // 0: one VP per (RAM, label); 1, 2: class-packed rows, one VP per RAM gives all l
  uint32_t nlab;            // labels in the grid: l for layout 0, 1 otherwise
  uint32_t rpr, nbf;        // layout 2: RAM j in row j / rpr from coefficient (j mod rpr) 2^nbf (else 1, 0)
};

// layout 2 rows from per-RAM rows: dst[R] (+)= sum over samples s < nsmp and
// RAMs j = R rpr + t < k0 of X^(t 2^nbf) src(s, j), src(s, j) = src + s
// sstride + j rstride (one RLWE each); the class counter (cnt) sums
// src(s, k0) unrotated
struct RowPackArgs {
  const uint32_t* src;
  uint64_t sstride, rstride;  // words
  uint64_t nsmp;
  uint32_t* dst;              // [rows] RLWE
  uint32_t* cnt;              // one RLWE or nullptr
  uint32_t k0, rpr, nbf, rows, N, nq;
  uint32_t store;             // 1: dst = sum (cnt is then not written); 0: dst += sum
};

// batched training: one entry per job
struct BJob {
  const uint32_t* x;        // RGSW of the job's first sample: [nsmp][s]
  const uint32_t* y;        // [nsmp][L]
  const uint32_t* perm;     // [s]
  uint32_t* model;          // [k0][k1] RLWE
  uint32_t* cnt;            // class counter or nullptr
  uint64_t acc0;            // word offset of the accumulators of pieces 1.. ([piece-1][nram][k1] RLWE)
  uint64_t words0;          // prefix over the jobs of the model (+ counter) words the reduction writes
  uint32_t s, a, L, k0, k1, nsmp;
  uint32_t l, kt;           // classes; tree leaves of a full RAM (scratch slots beyond the input slot)
  uint32_t nram;            // k0, + 1 with a class counter
  uint32_t per, pieces;     // samples per piece, pieces per RAM
  uint32_t layout;          // as TrainArgs::layout
};

struct BItem {
  uint32_t job, ram, piece, xp;  // xp: external products of the item (queue order)
};

struct BatchArgs {
  const BJob* jobs;
  const BItem* items;
  uint32_t nitems;
  uint32_t* counter;
  uint32_t* ws;             // per persistent workgroup: scratch_words (k1max + 1 RLWE slots)
  uint64_t scratch_words;
  uint32_t* acc;            // accumulators of pieces >= 1
  uint64_t rgsw_words;
};

// batched inference: one entry per job (args.i0, nsub and map unused; args.scratch unused)
struct IJob {
  InferArgs args;           // the job's model, inputs, scores and shape fields
  uint32_t nsmp;            // samples
  uint32_t per;             // samples per piece
};

struct IItem {
  uint32_t job, ram, lab, piece;
};

struct IBatchArgs {
  const IJob* jobs;
  const IItem* items;
  uint32_t nitems;
  uint32_t* counter;
  uint32_t* ws;             // per persistent workgroup: scratch_words (slots + 1 RLWE)
  uint64_t scratch_words;
};

struct PksArgs {
  const uint32_t* key;      // [N][D][2][NQ][N] evaluation domain
  const uint32_t* lwe;      // [count][k] LWE ([NQ][N+1] each)
  uint32_t* part;           // [count][NQ][blocks][2][N] evaluation-domain partial sums
  uint32_t* out;            // [count] RLWE
  uint32_t k;               // LWE per group, <= N
};

struct SumArgs {
  const uint32_t* scores;   // [n][l][k0] LWE
  uint32_t* sums;           // [n][l] LWE
  uint64_t n;
  uint32_t l, k0, N, nq;
};

// launchers (hw_kernels.hip); return hipSuccess or the launch error
hipError_t launch_keygen(uint32_t N, uint64_t seed, int32_t* sk, hipStream_t st);
// the binary LWE key s1[n] and the key-switching key from sk to it, D digits
// per ring coefficient, as signed bytes [4 (n + 1)][N D] (the rows past
// 4 (n + 1) of a padded buffer are left as they are)
hipError_t launch_lwe_keygen(uint32_t n, uint64_t seed, uint8_t* s1, hipStream_t st);
hipError_t launch_ksk_gen(const int32_t* sk, const uint8_t* s1, uint32_t N, uint32_t n, uint64_t seed, uint32_t D,
                          const Cdt& cdt, int8_t* out, hipStream_t st);
// sk_hat: 2 nq N words (the transformed key, then its Shoup companions)
hipError_t launch_sk_hat(int logN, int nq, const Tabs& T, const int32_t* sk, uint32_t* sk_hat, hipStream_t st);
// dig: digits per prime of the RGSW gadget (5 of 6 bits, or 2 of 15 bits on
// rings of two or more primes; A.log_base must match), 2 dig nq rows per RGSW
hipError_t launch_enc_rgsw(int logN, int nq, int dig, const Tabs& T, const Cdt& cdt, const EncArgs& A,
                           uint64_t count, int rows_per_wg, hipStream_t st);
hipError_t launch_enc_rlwe(int logN, int nq, const Tabs& T, const Cdt& cdt, const EncArgs& A, uint64_t count,
                           hipStream_t st);
hipError_t launch_dec_rlwe(int logN, int nq, const Tabs& T, const CrtTab& K, const uint32_t* sk_hat,
                           const uint32_t* ct, uint64_t count, uint64_t* msg, hipStream_t st);
hipError_t launch_dec_lwe(int logN, int nq, const Tabs& T, const CrtTab& K, const int32_t* sk,
                          const uint32_t* lwe, uint64_t count, uint64_t* msg, hipStream_t st);
hipError_t launch_rgsw_export(int logN, int nq, int dig, const Tabs& T, const uint32_t* rgsw, uint64_t count,
                              uint32_t* out, hipStream_t st);
hipError_t launch_ntt(int logN, int nq, const Tabs& T, uint32_t* polys, uint64_t count, int inverse,
                      uint32_t per, hipStream_t st);
hipError_t launch_xp(int logN, int nq, int dig, const Tabs& T, const uint32_t* rgsw, const uint32_t* in,
                     uint64_t count, uint32_t* out, hipStream_t st);
// occ: occupancy target of the external-product kernels, 3 or 4 (4 only for log2 N = 12)
// the permutation of (s, seed) written to pi[0..s) on the device (one thread)
hipError_t launch_perm(uint32_t s, uint64_t seed, uint32_t* pi, hipStream_t st);
hipError_t launch_train(int logN, int nq, int dig, const Tabs& T, const TrainArgs& A, int occ, hipStream_t st);
// one CDEMUX level of every (sample, RAM) of a sub-batch whose chains k_train
// (A.tree = 0) has run: A.nram x A.nsub x A.smax workgroups, one split each
hipError_t launch_train_level(int logN, int nq, int dig, const Tabs& T, const TrainArgs& A, int occ,
                              hipStream_t st);
hipError_t launch_reduce_model(const Tabs& T, const ReduceArgs& A, hipStream_t st);
hipError_t launch_row_pack(const Tabs& T, const RowPackArgs& A, hipStream_t st);
hipError_t batch_grid(int logN, int nq, int dig, int occ, uint32_t* grid);  // persistent workgroups that fit
hipError_t launch_train_batch(int logN, int nq, int dig, const Tabs& T, const BatchArgs& A, uint32_t grid, int occ,
                              hipStream_t st);
hipError_t launch_reduce_batch(const Tabs& T, const BJob* jobs, uint32_t njobs, uint64_t total, uint32_t logN,
                               uint32_t N, uint32_t nq, const uint32_t* acc, hipStream_t st);
hipError_t launch_infer(int logN, int nq, int dig, const Tabs& T, const InferArgs& A, int occ, hipStream_t st);
hipError_t infer_batch_grid(int logN, int nq, int dig, int occ, uint32_t* grid);
hipError_t launch_infer_batch(int logN, int nq, int dig, const Tabs& T, const IBatchArgs& B, uint32_t grid, int occ,
                              hipStream_t st);
hipError_t launch_class_sums(const Tabs& T, const SumArgs& A, hipStream_t st);
hipError_t launch_enc_pks(int logN, int nq, const Tabs& T, const Cdt& cdt, const EncArgs& A, hipStream_t st);
uint32_t pks_blocks(int logN);  // key-coordinate blocks of the packing (partial sums per group and prime)
hipError_t launch_pks(int logN, int nq, const Tabs& T, const PksArgs& A, uint32_t count, hipStream_t st);
hipError_t launch_rlwe_add(const Tabs& T, uint32_t* dst, const uint32_t* src, uint64_t words, uint32_t N, uint32_t nq,
                           hipStream_t st);

}  // namespace hw
