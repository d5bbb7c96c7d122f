/*
 * nshe_probe.h - measurement entry points of libnshe.so (not part of the
 * evaluation path): the ceilings the design is judged against.
 *
 * nshe_probe_modmul  the chip-wide rate of the exact FP64 modular product
 *   the transforms use (six FP64 operations: mul, fma, mul, rndne, fma, add;
 *   van der Hoeven, Lecerf and Quintin 2016), eight independent dependent
 *   chains per thread, 256 x 16 workgroups of 256 threads, `iters` products
 *   per chain; the second of two timed launches is reported.
 *
 * nshe_probe_conversion  one residue-base conversion out_k = sum_i y_i M_ik
 *   (mod m_k), the dense contraction inside the centred lifts and the
 *   scale-and-round (n_in -> n_out primes: 17 -> 18 or 18 -> 17), on n_coef
 *   coefficients of pseudo-random balanced residues and constants, computed
 *   by the library's split-FMA rows (VALU) and by integer MFMA
 *   (v_mfma_i32_32x32x32_i8 on signed base-256 digits); times are the mean
 *   over `reps` launches after one warm-up pass, and `mismatches` counts
 *   outputs where the two differ mod m_k (must be 0).
 *
 * nshe_probe_fp64_overlap  whether FP64 matrix instructions add FP64
 *   throughput to the vector ALU: the same grid (256 x 16 workgroups of 256
 *   threads, `iters` iterations) runs 64 FP64 FMAs per lane and iteration on
 *   the VALU (eight independent chains), or four independent
 *   v_mfma_f64_16x16x4f64 per wave and iteration (the same FMA count), or
 *   both interleaved in every wave; the second of two timed launches of each
 *   is reported.  Independent units would give ms_both near the larger of
 *   ms_valu and ms_mfma; one shared pipeline gives their sum.
 *
 * All allocate and free their own device buffers on `hip_device` and
 * synchronise it.  They return 0, or a negative code with a message from
 * nshe_probe_last_error().
 */
#ifndef NSHE_PROBE_H
#define NSHE_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double ms;              /* one launch */
  double products_per_s;  /* modular products per second, chip-wide */
  double fp64_ops_per_s;  /* 6 FP64 VALU operations per product */
} nshe_modmul_probe;

typedef struct {
  uint64_t coefficients;
  double ms_fma;          /* split-FMA rows, one launch */
  double ms_mfma;         /* integer MFMA, one launch */
  uint64_t mismatches;    /* outputs that differ (mod m_k) */
} nshe_conv_probe;

typedef struct {
  double ms_valu;         /* VALU FMAs only, one launch */
  double ms_mfma;         /* FP64 MFMA only */
  double ms_both;         /* both in every wave */
  double fma_per_s_valu;  /* lane-level FMAs per second, chip-wide */
  double fma_per_s_mfma;
} nshe_overlap_probe;

int nshe_probe_modmul(int hip_device, int iters, nshe_modmul_probe* out_host);
int nshe_probe_fp64_overlap(int hip_device, int iters, nshe_overlap_probe* out_host);
int nshe_probe_conversion(int hip_device, const uint64_t* in_primes_host, int n_in,
                          const uint64_t* out_primes_host, int n_out, size_t n_coef, int reps,
                          nshe_conv_probe* out_host);
const char* nshe_probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NSHE_PROBE_H */
