// Shared declarations of the device kernels and their launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "modarith.h"

namespace nshe {

constexpr int MAX_L = 24;            // data primes
constexpr int MAX_ALPHA = 3;         // special primes (data primes per key-switching digit)
constexpr int MAX_PRIMES = 2 * MAX_L + 1 + MAX_ALPHA;

// Device constant tables of a context (all pointers are device memory).
// Prime index convention: data primes q_0..q_{L-1} are 0..L-1, extension
// primes b_0..b_{L} are L..2L, the special primes P_0..P_{alpha-1} are
// 2L+1..2L+alpha (P = P_0 ... P_{alpha-1}).
struct Tables {
  const double* p;           // [K]
  const double* pinv;        // [K] fl(1/p)
  const double* recip;       // [K] fl(1/p), the same values as pinv: no kernel reads it
                             // any more (pinv serves the CRT estimates); kept so that
                             // the struct's layout, and the kernels' registers, stay put
  const double* ninv;        // [K] balanced N^-1
  const double* tw_fwd;      // [K][tw_len] round-0 twiddles (slot 2^k + j)
  const double* tw_inv;      // [K][tw_len]
  int tw_len;
  // rounds >= 1: per index row u the first twiddle of each stage (8 slots,
  // stage k at slot k; a round's rows stored slot-major, slot k of row u at
  // k rows + u), rounds one after the other; the others are that one times
  // a constant per (stage, slot) shared by all rows
  const double* tw_cmp_f;    // [K][tw_cmp_len]
  const double* tw_cmp_i;    // [K][tw_cmp_len]
  int tw_cmp_len;
  const double* tw_cmp_h;    // [K][2][tw_cmp_h_len] (half-limb forward)
  int tw_cmp_h_len;
  const double* tw_cst_f;    // [K][32] slot 2^k + j: omega_k^brv_k(j)
  const double* tw_cst_i;    // [K][32] slot 2^k + j: omega_k^-brv_k(j)
  const double* tw_half;     // [K][2][tw_half_len] round-0 twiddles of each half's sub-transform
  const double* tw_half0;    // [K] psi^(2^14), the stage-0 twiddle
  int tw_half_len;
  // the same for the half-limb inverse sub-transforms (inverse twiddles)
  const double* tw_half_inv; // [K][2][tw_half_len]
  const double* tw_cmp_hi;   // [K][2][tw_cmp_h_len]
  // round 1 of each half's sub-transform in full: [K][2][16 rows][32 slots],
  // slot 2^k + j of row u the twiddle of the round's stage k, block j
  const double* tw_r1_f;
  const double* tw_r1_i;
  // centred lift Q -> B
  const double* q_hat_inv;   // [L]      [(Q/q_i)^-1]_{q_i}
  const double* Q_b;         // [LB]     [Q]_{b_k}
  // scale and round, then B -> Q
  // (the scale-and-round reads inverse-transform output, which carries a
  // factor N: its constants include N^-1)
  // t_qhinv, t_q and c1 hold a second row: the same constants times w,
  // the 2^15-point inverse's last-stage twiddle of the prime (for the upper
  // coefficients after the split inverse)
  const double* t_qhinv;     // [2][L]   [t (Q/q_i)^-1 N^-1]_{q_i}
  const double* t_q;         // [2][L]   [t N^-1]_{q_i}
  const double* c1;          // [2][LB]  [t Q^-1 (B/b_k)^-1 N^-1]_{b_k}
  const double* b_hat_inv;   // [LB]     [(B/b_k)^-1]_{b_k}
  const double* B_q;         // [L]      [B]_{q_i}
  // the three base-conversion matrices, each balanced entry M split for
  // exact FMA accumulation as M = c1 2^24 + c0, stored {c1, c0} (see
  // conv_row), and [2^24]_p, [2^48]_p per prime
  const double* q_hat_b_sp;  // [LB][L][2]  [Q/q_i]_{b_k}
  const double* c2_sp;       // [LB][L][2]  [q_i^-1 (B/b_k)^-1]_{b_k}
  const double* b_hat_q_sp;  // [L][LB][2]  [B/b_k]_{q_i}
  const double* two24;       // [K]
  const double* two48;       // [K]
  // key switching (digits of alpha data primes, alpha special primes; the
  // tables for several primes per digit are at the end of the struct)
  const double* P_inv_q;     // [L]      [P^-1]_{q_i}
  const double* NP_inv_q;    // [2][L]   [N^-1 P^-1]_{q_i}; second row times w_i
  const double* ninv_P;      // [alpha][2] [N^-1]_{P_k}, times w_{P_k} (w: the 2^15-point
                             //          inverse's last-stage twiddle of the prime)
  const double* delta_q;     // [L]      [floor(Q/t)]_{q_i}
  // exact fallback of the Q lift: mixed-radix digits
  const double* mrc_inv;     // [L][L]   [q_j^-1]_{q_i}, canonical, row j
  const double* mrc_half;    // [L]      mixed-radix digits of (Q-1)/2
  // event counters ([MARGIN_COUNT]): exact-lift fallbacks taken, per call
  // site, and B->Q lifts outside their proven range (never)
  unsigned long long* margin;
  // the centred lift's exact fallback is taken when |S - rint(S)| exceeds
  // this (1/2 - 2^-40; 1/4 under the debug switch)
  double lift_edge;
  // residues outside [0, q_i) seen by the input check (debug switch)
  int* bad_input;
  int ks_alpha;              // alpha: 1, 2 or 3
  // alpha > 1: the centred residue mod P = P_0 ... P_{alpha-1} in mixed
  // radix, a_0 + P_0 k_1 + P_0 P_1 k_2 with balanced digits (Garner:
  // k_1 = [(a_1 - a_0) P_0^-1]_{P_1}, k_2 = [((a_2 - a_0) P_0^-1 - k_1) P_1^-1]_{P_2})
  const double* mr_q;        // [alpha-1][L] [(P_0 ... P_{k-1}) P^-1]_{q_i}, k = 1..alpha-1
  double p_inv_p[3];         //          [P_0^-1]_{P_1}, [P_0^-1]_{P_2}, [P_1^-1]_{P_2}, balanced
  // alpha > 1: a digit's value mod target prime i of the key-switching
  // basis from its canonical mixed-radix digits (v_0, ..., v_{alpha-1}):
  // v_0 + [q_{j alpha}]_{p_i} v_1 + [q_{j alpha} q_{j alpha + 1}]_{p_i} v_2
  const double* dig_c;       // [dnum][L + alpha][alpha - 1], balanced
  // N = 2^15, digit transforms by coefficient parity (k_ntt_fwd_par): the
  // 2^14-point transforms of the even and of the odd coefficients (root
  // psi^2) use the full transform's twiddles of stages 0..13, slot 2^s + m
  // of stage s (round 0's row is tw_fwd's); their compact rows of rounds 1
  // and 2, and round 1 in full for the LDS copy (16 rows x 32 slots)
  const double* tw_cmp_par;  // [K][tw_cmp_h_len]
  const double* tw_r1_par;   // [K][512]
  // the full transform's last-stage twiddles psi^brv(2^14 + k) of the
  // key-switching basis, in the order of k_ks_mac_par's threads: entry
  // u 1024 + m holds k = 16 m + u
  const double* tw_last;     // [L + alpha][2^14]
  // set per launch of the scale-and-round: where the relinearization digit
  // source goes (null: in place; see k_scale)
  double* dig_src;
};

// Call sites of the exact-lift fallback (index into Tables::margin).
enum MarginSite {
  MARGIN_LIFT = 0,          // k_lift: a squaring's operand lift, not fused (no split transforms)
  MARGIN_SCALE = 1,         // k_scale: the scale-and-round's lift of [t d]_Q
  MARGIN_SCALE_SPLIT = 2,   // k_scale after the split inverse (N = 2^15)
  MARGIN_MODDOWN_LIFT = 3,  // k_moddown_lift: the next squaring's operand
  MARGIN_SUB_LIFT = 4,      // k_sub_lift: the chain's first operand
  MARGIN_I64_LIFT = 5,      // k_i64_lift: a product's int64 operands
  MARGIN_SITES = 6,
  MARGIN_FAULT = 8,         // B->Q lift outside its range (never)
  MARGIN_COUNT = 9
};

enum { NTT_INPLACE = 0, NTT_DIGIT = 1, INV_TENSOR = 2, INV_TENSOR2 = 3, INV_PLAIN = 4,
       NTT_DIGIT2 = 5, NTT_DIGIT3 = 6 };

struct NttJob {
  double* base;              // first limb of poly 0 (input of in-place kinds)
  double* out;               // output base, same strides (null: in place)
  size_t poly_stride;        // doubles between consecutive polys
  int npoly;                 // polys in the launch
  int nlimb;                 // limbs per poly transformed
  const int* limb_prime;     // [nlimb] prime index of each limb
  int count;                 // npoly * nlimb
  // NTT_DIGIT source: third component's data limbs, canonical residues in
  // [0, q_j) (the digits themselves); with alpha primes per digit, limbs
  // j alpha .. j alpha + alpha - 1 hold digit j's canonical mixed-radix
  // digits (v_0, v_1[, v_2]), D_j = v_0 + q_{j alpha} v_1 (+ q_{j alpha}
  // q_{j alpha + 1} v_2) in [0, Q_j) (NTT_DIGIT2, NTT_DIGIT3), in natural
  // order or (src_split) by coefficient parity, c at (c mod 2) N/2 + c/2; INV_TENSOR: the
  // operands' transforms ([ct][2][W][N], src_b null when squaring)
  const double* src;
  const double* src_b;
  size_t src_ct_stride;      // doubles between ciphertexts in src
  int digits;                // digits per ciphertext (L / alpha)
  int alpha = 1;             // data primes per digit
  int split = 1;             // 2^15-point forward: two workgroups per limb
  // 2^15-point inverse (directions 1 and 3): two workgroups per limb that
  // stop before the last stage, which the consumer (scale-and-round, or
  // mod-down) applies as it loads; see k_ntt_inv_half for the layouts
  int split_inv = 0;
  // 2^15-point digit transforms (direction 2) by coefficient parity, two
  // 2^14-point transforms per limb; the key-switch product applies the last
  // stage (k_ntt_fwd_par, k_ks_mac_par)
  int parity = 0;
  // with parity and three-prime digits: the digit source is stored by
  // coefficient parity (see src)
  int src_split = 0;
};

// run_ntt directions: 0 forward in place, 1 inverse in place, 2 forward of
// relinearization digits, 3 inverse of the tensor product formed on load,
// 4 inverse of tensor components already formed (base) into out, in the
// layout direction 3 writes.

hipError_t run_ntt(int log2n, const NttJob& job, const Tables& tb, int dir, hipStream_t st);
// key-switch product fused with the digit transforms (N = 2^15 only):
// job.npoly = ciphertexts, job.digits = L, job.nlimb = L + 1, job.src /
// src_ct_stride the digits' canonical source limbs, job.limb_prime the
// key-switching basis; writes acc [n_ct][2][L+1][N] (NTT domain)
hipError_t run_ks_fused(const NttJob& job, const double* evk, double* acc, const Tables& tb,
                        hipStream_t st);
int ntt_rounds(int log2n, int* loge, int* r0);

// Per-coefficient and elementwise kernels (rns.hip).
struct CtPtrs;

// A batched wave's ciphertexts: a device table of per-ciphertext pointers
// ([wave][stride] entries) and the wave, a device counter (table null: none)
struct WaveTab {
  const CtPtrs* table = nullptr;
  const int* wave = nullptr;
  int stride = 0;
};

struct Dims {
  int n;        // N
  int L;        // data primes
  int LB;       // extension primes (= L + 1)
  int n_ct;     // ciphertexts in the call
  // launch shape (tunable; results do not depend on it)
  int block = 256;     // threads per workgroup of lift, scale and mod-down
  int ks_chunk = 16;   // ciphertexts per pass over the key in k_ks_mac
  // scale-and-round / mod-down inputs come from the split inverse (2^15
  // points): the last inverse stage is still to be applied on load
  int fused = 0;
  int alpha = 1;       // special primes (data primes per key-switching digit)
  // the digit transforms are by coefficient parity (N = 2^15): the key-switch
  // product applies their last stage (k_ks_mac_par)
  int parity = 0;
  // a batched wave's table: run_sub_lift reads x and y, run_moddown_finish
  // writes out, through it (their pointer arguments are then unused)
  WaveTab tab;
};

hipError_t run_lift(const Dims& d, double* ext, const Tables& tb, hipStream_t st);
// digit_pairs: write the third component as the digits' mixed-radix digits
// (the relinearization digit source with alpha > 1) instead of canonical
// residues.  src (not null): write the third component (the digit source)
// there instead of in place, ciphertext ct at src + ct 2 (L + alpha) N (limbs
// 0..L-1, N apart), coefficient c at (c mod 2) N/2 + c/2, the layout the
// digit transforms by parity read.
hipError_t run_scale(const Dims& d, double* dt, const Tables& tb, hipStream_t st,
                     int digit_pairs = 0, double* src = nullptr);
hipError_t run_ks_mac(const Dims& d, const double* dig, const double* evk, double* acc,
                      const Tables& tb, hipStream_t st);
hipError_t run_moddown(const Dims& d, const double* acc, const double* dt, double* ext,
                       const Tables& tb, hipStream_t st,
                       int accumulate = 0);
// the last level's mod-down written to int64 with the mask's finish,
// (Delta, 0) - z; needs d.fused
hipError_t run_moddown_finish(const Dims& d, const double* acc, const double* dt, int64_t* out,
                              const Tables& tb, hipStream_t st,
                              int finish = 1);
// int64 ciphertexts into ext followed by their lift (a product's operands)
hipError_t run_i64_lift(const Dims& d, const int64_t* in, double* ext, const Tables& tb,
                        hipStream_t st);
// subtraction into ext followed by its lift (the first squaring's operand)
hipError_t run_sub_lift(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                        double* ext, const Tables& tb, hipStream_t st);
// mod-down of the split inverse's output followed by the lift of the result
// (the next squaring's operand), one kernel; needs d.fused
hipError_t run_moddown_lift(const Dims& d, const double* acc, const double* dt, double* ext,
                            const Tables& tb, hipStream_t st);
// conversions at the boundary
hipError_t run_sub_to_ext(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                          double* ext, const Tables& tb, hipStream_t st);
// plaintext products: a slot's basis plaintext, a plaintext's limbs (times
// N^-1), and the pointwise product with the data limbs of transforms
hipError_t run_basis_plain(int n, uint64_t t, uint64_t zinv, uint64_t ninv_t, int64_t* out,
                           hipStream_t st);
hipError_t run_plain_limbs(const Dims& d, int64_t t, const int64_t* pt, double* out,
                           const Tables& tb, hipStream_t st);
hipError_t run_pointwise_plain(const Dims& d, double* fx, const double* pt, const Tables& tb,
                               hipStream_t st);
// comparisons: scalar linear combinations of up to 256 ciphertext arrays
// (J <= 16 outputs, coefficient rows [J][k]), the trivial encryption of 1,
// and differences with optional broadcast and sign
struct BabyPtrs {
  static constexpr int CAP = 256;
  const int64_t* p[CAP];
};
hipError_t run_tensor_mac(const Dims& d, const double* fa, const double* fb, double* acc,
                          int first, const Tables& tb, hipStream_t st);
hipError_t run_lincomb(const Dims& d, int k, const BabyPtrs& b, const double* coef, int J,
                       int64_t* out, size_t out_stride, const Tables& tb, hipStream_t st);
hipError_t run_fill_one(const Dims& d, int64_t* out, const Tables& tb, hipStream_t st);
hipError_t run_diff_i64(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                        int negate, int64_t* out, const Tables& tb, hipStream_t st);
// rotations: automorphism of ext into dt's key-switching layout (the third
// component to src, as in run_scale, when src is not null)
hipError_t run_automorph(const Dims& d, unsigned ginv, const double* ext, double* dt,
                         const Tables& tb, hipStream_t st, double* src = nullptr,
                         size_t src_stride = 0, int src_split = 0);
// alpha primes per digit (alpha > 1): canonical residues of the digit
// source (limbs 0..L-1 of ciphertext ct at src + ct src_stride, any
// coefficient order) into each digit's canonical mixed-radix digits, in place
hipError_t run_digit_mrc(const Dims& d, double* src, size_t src_stride, const Tables& tb,
                         hipStream_t st);
// dt's third component (natural order) into src by coefficient parity (as
// run_scale's src_split)
hipError_t run_digit_split(const Dims& d, const double* dt, double* src, size_t src_stride,
                           hipStream_t st);
// p[0..words) = v, as a kernel (no memset node in a captured graph)
hipError_t run_fill_u64(void* p, size_t words, uint64_t v, hipStream_t st);
// debug input check: sets *tb.bad_input if a residue of [n_poly][L][N] is
// outside [0, q_i)
hipError_t run_check_residues(int n, int L, size_t n_poly, const int64_t* in, const Tables& tb,
                              hipStream_t st);
// out = a + sum_{j < k} b[j * stride] (canonical int64 ciphertexts)
hipError_t run_sum_i64(const Dims& d, const int64_t* a, const int64_t* b, size_t stride, int k,
                       int64_t* out, const Tables& tb, hipStream_t st);
// batched waves (see k_gather_sub): per-ciphertext pointers of a wave
struct CtPtrs {
  const int64_t* x;
  const int64_t* y;
  int64_t* out;
};
hipError_t run_gather_sub(const Dims& d, int stride, const CtPtrs* table, const int* wave,
                          double* ext, const Tables& tb, hipStream_t st);
hipError_t run_scatter_mask(const Dims& d, int stride, const CtPtrs* table, const int* wave,
                            const double* ext, const Tables& tb, hipStream_t st);
// table entries [first, first + n) passed by value (kernel arguments are
// copied at launch, so the host array may be reused at once)
struct TableChunk {
  static constexpr int CAP = 128;
  CtPtrs e[CAP];
  int first;
  int n;
};
hipError_t run_fill_table(const TableChunk& ch, CtPtrs* table, hipStream_t st);
hipError_t run_set_counter(int* counter, int v, hipStream_t st);
hipError_t run_bump_counter(int* counter, int step, hipStream_t st);
hipError_t run_sub_i64(const Dims& d, const int64_t* x, const int64_t* y, int64_t* out,
                       const Tables& tb, hipStream_t st);
// int64 [0, q) -> balanced doubles; polys with index >= canon_from keep the
// canonical value (the relinearization digit source)
hipError_t run_i64_to_polys(const Dims& d, const int64_t* in, int npoly_in, double* out,
                            size_t out_ct_stride, size_t out_poly_stride, int canon_from,
                            const Tables& tb, hipStream_t st);
hipError_t run_polys_to_i64(const Dims& d, const double* in, int npoly, size_t in_ct_stride,
                            size_t in_poly_stride, int64_t* out, int negate_delta,
                            const Tables& tb, hipStream_t st);
hipError_t run_i64_to_dbl_limbs(size_t rows, int n, const int64_t* in, double* out,
                                const int* row_prime, int nprime_rows, const Tables& tb,
                                hipStream_t st);
hipError_t run_ntt_order(int log2n, size_t rows, const double* in, int64_t* out,
                         const int* row_prime, int nprime_rows, int to_natural,
                         const Tables& tb, hipStream_t st);

}  // namespace nshe
