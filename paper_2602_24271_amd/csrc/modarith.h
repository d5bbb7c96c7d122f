// Exact modular arithmetic on the FP64 pipe of gfx950.
//
// Every residue is an integer held exactly in a double.  Primes p lie in
// [2^48, 2^49), so |x| < 2^53 covers every intermediate below.  A product
// a*b (|a| < 2p, |b| < p) is split exactly into h + l with h = fl(a*b) and
// l = fma(a, b, -h) (the error-free transform of Dekker/Kahan); the quotient
// q = rint(h * pinv) is within 0.875 of a*b/p, so r = (h - q*p) + l is exact
// (both steps stay below 2^53) and |r| < 0.875 p.  This is the FP-FMA
// modular product of van der Hoeven, Lecerf and Quintin ("Modular SIMD
// arithmetic in Mathemagix", 2016), with a rounding quotient so that the
// result is signed and needs no correction branch.
//
// Representations used across kernels:
//   balanced  : |x| < p/2            (the canonical stored form, p odd)
//   lazy      : |x| < 2p             (in-register NTT operands)
// Conversion of any |x| < 2^52 to balanced: x - p * rint(x * pinv), exact
// because x/p is never within 2^-50 of a half-integer (p odd, x integer).
#pragma once
#include <hip/hip_runtime.h>

namespace nshe {

struct Mod {
  double p;
  double pinv;  // fl(1/p)
};

// a*b mod p, |result| < 0.875 p, for |a| < 2p (or |a*b| < 2 p^2) and |b| < p.
__device__ __forceinline__ double mul_lazy(double a, double b, double p, double pinv) {
  double h = a * b;
  double l = __builtin_fma(a, b, -h);
  double q = __builtin_rint(h * pinv);
  return __builtin_fma(-q, p, h) + l;
}

// Balanced representative of x (|x| < 2^52): |result| < p/2.
__device__ __forceinline__ double reduce_bal(double x, double p, double pinv) {
  double q = __builtin_rint(x * pinv);
  return __builtin_fma(-q, p, x);
}

// a*b mod p in balanced form.
__device__ __forceinline__ double mul_bal(double a, double b, double p, double pinv) {
  return reduce_bal(mul_lazy(a, b, p, pinv), p, pinv);
}

// Balanced -> [0, p).
__device__ __forceinline__ double to_canonical(double x, double p) {
  return x < 0.0 ? x + p : x;
}

// [0, p) (as int64) -> balanced double.  Exact: values < 2^49.
__device__ __forceinline__ double from_u64(long long v, double p) {
  double x = (double)v;
  return x > 0.5 * p ? x - p : x;
}

__device__ __forceinline__ long long to_i64(double bal, double p) {
  return (long long)to_canonical(bal, p);
}

}  // namespace nshe

namespace nshe {

// Raw buffer access: one 32-bit VGPR offset per lane plus a scalar offset,
// so per-element addressing of a register-resident limb costs no VGPRs.
// Out-of-range accesses (offset >= bytes) read 0 and drop stores.
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, (v2u)__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, voff, soff, 0);
}

// Read-only table load through the constant address space: uniform
// indices then use scalar loads (SGPRs) instead of one vector load per lane.
// Valid because the tables are never written while a kernel runs.
typedef const __attribute__((address_space(4))) double* const_dptr;
typedef const __attribute__((address_space(4))) int* const_iptr;

__device__ __forceinline__ double cld(const double* p, int i) { return ((const_dptr)p)[i]; }

// A row of a uniform table whose address the compiler cannot see through
// (inline asm on the scalar register), so that its scalar loads are not
// hoisted into earlier loop iterations: a base-conversion loop over 18
// rows of 17 constants would otherwise keep hundreds of constants live in
// SGPRs and spill them into VGPR lanes.
__device__ __forceinline__ const double* opaque_row(const double* p, int off) {
  const double* r = p + off;
  asm volatile("" : "+s"(r));
  return r;
}
__device__ __forceinline__ int cldi(const int* p, int i) { return ((const_iptr)p)[i]; }

// An index the compiler cannot see through (inline asm on a scalar
// register): the scalar loads of an unrolled loop iteration indexed by it
// are neither hoisted above that point nor merged with other iterations'
// into wide loads whose values would be held (and spilled) across the loop.
__device__ __forceinline__ int opaque_idx(int i) {
  asm volatile("" : "+s"(i));
  return i;
}

}  // namespace nshe
