// The split-FMA base-conversion row shared by the per-coefficient kernels
// (and timed against the MFMA form by the conversion probe).
#pragma once
#include "modarith.h"

namespace nshe {

// A base-conversion row sum_j y_j M_j (mod m) over NT <= 25 terms with four
// FMAs per term instead of a modular product.  Each input (a reduced
// residue, |y| <= 2^48) is split once as y = yh 2^24 + yl (|yh| <= 2^24,
// |yl| <= 2^23) and each constant is stored split the same way, M = c1 2^24
// + c0 (|c1| <= 2^24, |c0| <= 2^23).  Then
//   y M = yh c1 2^48 + (yh c0 + yl c1) 2^24 + yl c0,
// so the row is W48 [2^48]_m + W24 [2^24]_m + W0 (mod m) with W48 = sum yh
// c1, W24 = sum yh c0 + yl c1 and W0 = sum yl c0.  Every product is an
// integer of at most 2^48, so exact, and so is every partial sum (|W48|,
// |W24| <= NT 2^48 < 2^53, |W0| <= NT 2^46).  Every prime lies in
// (2^48, 2^49), so [2^24]_m = 2^24 and [2^48]_m = 2^48: T48 = W48 2^48 and
// T24 = W24 2^24 are exact doubles (exponent shifts), and each is reduced
// exactly by one FMA, T - q m with q = rint(T fl(1/m)): the true difference
// is an integer below 1.5 m for NT <= 16 (below 2.5 m for NT <= 25: the
// quotient estimate is within 2 of T / m <= 2^53), so exactly
// representable, and the FMA returns it.  The result is returned
// unreduced, |result| <= (NT / 4 + 7.2) 2^48.
constexpr int CONV_SPLIT_MAX = 25;
constexpr int CONV_CHUNK = 9;

__device__ __forceinline__ void split24(double y, double& yh, double& yl) {
  yh = __builtin_rint(y * 0x1p-24);
  yl = __builtin_fma(-yh, 0x1p24, y);
}

// sp: the row's constants {c1, c0} per term; m in (2^48, 2^49), minv =
// fl(1/m).
template <int NT>
__device__ __forceinline__ double conv_row(const double (&yh)[NT], const double (&yl)[NT],
                                           const double* sp, double m, double minv) {
  static_assert(NT <= CONV_SPLIT_MAX, "partial sums must stay below 2^53");
  double w48 = 0.0, w24a = 0.0, w24b = 0.0, w0 = 0.0;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    // constants are fetched CONV_CHUNK terms at a time: the row pointer is
    // made to depend on the running sums, so later terms' scalar loads are
    // not all hoisted to the row's start (which spills scalar registers)
    if (j && j % CONV_CHUNK == 0) asm volatile("" : "+s"(sp) : "v"(w0));
    const double c1 = cld(sp, 2 * j), c0 = cld(sp, 2 * j + 1);
    w48 = __builtin_fma(yh[j], c1, w48);
    w24a = __builtin_fma(yh[j], c0, w24a);
    w24b = __builtin_fma(yl[j], c1, w24b);
    w0 = __builtin_fma(yl[j], c0, w0);
  }
  // (ldexp: exponents 48 and 24 are inline operands; a 2^48 multiplier
  // would hold a register pair through the row loops)
  const double t48 = __builtin_ldexp(w48, 48), t24 = __builtin_ldexp(w24a + w24b, 24);
  const double r48 = __builtin_fma(-__builtin_rint(t48 * minv), m, t48);
  const double r24 = __builtin_fma(-__builtin_rint(t24 * minv), m, t24);
  return r48 + r24 + w0;
}

}  // namespace nshe
