// Per-coefficient residue-number-system kernels: exact centred lifts between
// the data basis Q = {q_i} and the extension basis B = {b_k}, the BFV
// scale-and-round, key-switch accumulation and mod-down, and the
// conversions at the library boundary.
//
// Exact centred lift (used by the product's operand lift and by the
// scale-and-round): for residues x_i of X in [0, Q), let
// y_i = [x_i (Q/q_i)^-1]_{q_i} (balanced) and S = sum_i y_i / q_i.  Then
// sum_i y_i (Q/q_i) = X + kQ with k = S - X/Q an integer, so the centred
// representative of X is sum_i y_i (Q/q_i) - rint(S) Q.  S is evaluated in
// double precision with absolute error below 2^-45 (L <= 24 terms of
// magnitude < 1/2); when S lies within 2^-40 of a half-integer the rounding
// decision is taken exactly instead: floor(S) = k, and X > (Q-1)/2 is
// decided by comparing mixed-radix digits of X with those of (Q-1)/2
// (Garner's algorithm).  Each such event is counted, per call site
// (MarginSite).  The window is a context setting (tb.lift_edge = 1/2 - 2^-40
// by default); a debug setting widens it to 1/4, which leaves floor(S)
// exact (S is then at least 1/4 from an integer) and sends about half of
// all coefficients through the exact path.
//
// Scale and round (BFV multiply): for d in Q u B (|d| < QB/2), the exact
// r = [t d]_Q (centred) gives y = (t d - r) / Q = round(t d / Q) exactly.
// In base B: [y]_{b_k} = [t Q^-1 d_k - sum_i y_i q_i^-1 + v]_{b_k} where
// y_i, v are the lift quantities of r; then y is lifted from B to Q (|y| <
// t N Q / 2 < B / 32, so that lift's estimate is never near a half-integer;
// a violation would be counted in `fault`).
//
// The sums over the other basis (sum_i y_i [Q/q_i]_{b_k} and the like) are
// matrix-vector products mod b_k; they run as exact FMA accumulations of
// split operands (conv_row) with one modular reduction per output.
#include "conv.h"
#include "kernels.h"

namespace nshe {


// Whether the lift takes its exact decision: S within 2^-40 of a
// half-integer, or within 1/4 under the debug switch (tb.lift_edge < 1/2 -
// 2^-40, a uniform flag: the default window stays a literal, which keeps the
// kernels' register counts).
__device__ __forceinline__ bool lift_near_half(double S, double v, const Tables& tb) {
  const double d = __builtin_fabs(S - v);
  return d > 0.5 - 0x1p-40 || (tb.lift_edge < 0.5 - 0x1p-40 && d > tb.lift_edge);
}

// Garner mixed-radix digits of X (canonical residues r, basis q_0..q_{L-1})
// compared with those of (Q-1)/2: returns X > (Q-1)/2.
// (Arguments by value: taking the address of the kernel's Tables argument
// would copy it to scratch memory in every thread.  A rare fallback: its
// loops stay rolled and its digits in private memory, so that it does not
// raise the register count - and lower the occupancy - of its callers.)
template <int L>
__device__ __noinline__ bool mrc_greater_than_half(const double* r, const double* __restrict__ P,
                                                   const double* __restrict__ Pinv,
                                                   const double* __restrict__ inv,
                                                   const double* __restrict__ half) {
  double a[L];
#pragma unroll 1
  for (int i = 0; i < L; ++i) {
    const double p = P[i], pinv = Pinv[i];
    double t = r[i];
#pragma unroll 1
    for (int j = 0; j < i; ++j) {
      t = mul_bal(t - a[j], inv[j * L + i], p, pinv);
      t = to_canonical(t, p);
    }
    a[i] = t;
  }
#pragma unroll 1
  for (int i = L - 1; i >= 0; --i) {
    const double h = half[i];
    if (a[i] != h) return a[i] > h;
  }
  return false;
}

// Per-poly block mapping of the per-coefficient kernels: block b covers
// coefficients [(b mod bpp) blockDim, ...) of poly b / bpp, so the poly and
// its base address are uniform (scalar registers): limb accesses are buffer
// loads with one per-lane offset and a scalar limb offset.
struct PolyBlock {
  size_t pc;
  int c;
  bool ok;
};

__device__ __forceinline__ PolyBlock poly_block(int n, size_t n_poly) {
  const int bpp = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const size_t pc = blockIdx.x / (unsigned)bpp;
  const int c = (int)(blockIdx.x - pc * bpp) * (int)blockDim.x + (int)threadIdx.x;
  return PolyBlock{pc, c, pc < n_poly && c < n};
}

// ------------------------------------------------ split base conversion ---

// ------------------------------------------------------------------ lift ---

// ext: [n_poly][L+LB][N]; limbs 0..L-1 (balanced, coefficient domain) are
// lifted to limbs L..L+LB-1 (the extension basis) in place.
template <int L>
__global__ void __launch_bounds__(256) k_lift(int n, size_t n_poly, double* ext, Tables tb) {
  constexpr int LB = L + 1;
  const PolyBlock pb = poly_block(n, n_poly);
  if (!pb.ok) return;
  const auto rs = make_rsrc(ext + pb.pc * (size_t)(L + LB) * n, (unsigned)((L + LB) * n * 8));
  const unsigned vo = (unsigned)pb.c * 8;
  const unsigned ls = (unsigned)n * 8;   // bytes per limb
  double y[L];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const double pinv = cld(tb.pinv, i);
    y[i] = mul_bal(buf_load(rs, vo, i * ls), cld(tb.q_hat_inv, i), cld(tb.p, i), pinv);
    S += y[i] * pinv;
  }
  double v = __builtin_rint(S);
  if (lift_near_half(S, v, tb)) {
    double r[L];
#pragma unroll
    for (int i = 0; i < L; ++i) r[i] = to_canonical(buf_load(rs, vo, i * ls), cld(tb.p, i));
    v = __builtin_floor(S) + (mrc_greater_than_half<L>(r, tb.p, tb.pinv, tb.mrc_inv, tb.mrc_half) ? 1.0 : 0.0);
    atomicAdd(tb.margin + MARGIN_LIFT, 1ull);
  }
  // |acc| <= (L / 4 + 7.2 + L/2 + 1) 2^48 < 2^53: reduce_bal is exact there
  // (its result within p/2 + 4)
  double yh[L], yl[L];
#pragma unroll
  for (int i = 0; i < L; ++i) split24(y[i], yh[i], yl[i]);
#pragma unroll
  for (int k = 0; k < LB; ++k) {
    const double b = cld(tb.p, L + k), binv = cld(tb.pinv, L + k);
    const double* sp = opaque_row(tb.q_hat_b_sp, k * L * 2);
    const double acc = conv_row<L>(yh, yl, sp, b, binv) -
                       v * cld(tb.Q_b, k);
    buf_store(reduce_bal(acc, b, binv), rs, vo, (L + k) * ls);
  }
}

// ------------------------------------------------- inverse-transform output ---

// Where a per-coefficient kernel reads coefficient c of a limb written by an
// inverse transform.  Plain: at c (byte offset v).  After the split inverse
// of a 2^15-point limb (FUSED) the coefficient is the inverse's last stage
// applied to the two half outputs U and V of its pair: U + V for the lower
// half of the coefficients, (U - V) w for the upper (hi), w = the full
// inverse's last-stage twiddle of the limb's prime.  Every such value is
// only ever multiplied by a constant, so w is folded into that constant
// (the "hi" tables) and the load returns U + V or U - V (|.| <= p + 8, as
// |U|, |V| <= p/2 + 4).  Lanes l and l + 32 of a wave hold the two
// coefficients of a pair and each loads both U and V (coef_load_both): the
// second load hits the cache lines of the first, and in the scale-and-round
// it measured faster than taking the partner lane's value with two lane
// swaps per value (pair_combine, which the mod-down + lift keeps: there the
// two loads measured slower).
struct CoefSrc {
  unsigned v;      // this lane's position (bytes): where it writes
  unsigned vu;     // the pair's U and V positions
  unsigned vv;
  double sg;       // -1 upper, +1 lower
  bool hi;
};

// U + sg V for a pair whose U is in lane l and V in lane l + 32 (sg = +1
// in the lower lanes, -1 in the upper): a lower lane gets U + V, an upper
// lane U - V.  v_permlane32_swap exchanges the upper half of one
// register's lanes with the lower half of another's (a VALU operation, no
// LDS round trip); swapping a register with itself leaves U in every
// lane's first result and V in every lane's second, so no lane selects.
__device__ __forceinline__ double pair_combine(double x, double sg) {
  const unsigned long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double u = __longlong_as_double(((unsigned long long)h[0] << 32) | l[0]);
  const double v = __longlong_as_double(((unsigned long long)h[1] << 32) | l[1]);
  return __builtin_fma(sg, v, u);
}

// Coefficient c's value (see CoefSrc; any lane may be inactive).
template <bool FUSED>
__device__ __forceinline__ double coef_load_both(__amdgpu_buffer_rsrc_t rs, const CoefSrc& s,
                                                 unsigned soff) {
  if constexpr (!FUSED) {
    return buf_load(rs, s.v, soff);
  } else {
    return __builtin_fma(s.sg, buf_load(rs, s.vv, soff), buf_load(rs, s.vu, soff));
  }
}

// The constant a coefficient of this lane is multiplied by: entry i of a
// [2][count] table (lower, then upper = lower times w).  FUSED lanes differ
// in the half they need, so they read it per lane (a vector load that hits
// the cache) rather than select between two scalar constants, which would
// keep both halves' constants in scalar registers.
template <bool FUSED>
__device__ __forceinline__ double coef_const(const CoefSrc& s, const double* tab, int i,
                                             int count) {
  if constexpr (!FUSED) return cld(tab, i);
  else return tab[(s.hi ? count : 0) + i];
}

// ----------------------------------------------------------------- scale ---

// dt: [n_poly][L+LB][N] coefficient domain (balanced).  Writes
// [round(t d / Q)]_Q into limbs 0..L-1 of the same poly.
// FUSED: dt holds the split inverse's half outputs (see CoefSrc); each
// wave takes 32 coefficient pairs (c, c + N/2), lanes 0-31 the lower
// coefficients and 32-63 the upper, and writes its outputs in place at the
// positions it alone reads.  A: data primes per key-switching digit (the
// third component's digit format).  tb.dig_src (not null, A = 3 only): the
// third component (the relinearization digit source) goes there instead,
// ciphertext ct at dig_src + ct 2 (L + A) N (the key-switch sums' stride),
// limb i at + i N, and coefficient c at position (c mod 2) N/2 + c/2
// (k_ntt_fwd_par's layout; in place, those positions are read by other
// waves).  (A table field, read where it is used: a kernel argument stays
// in scalar registers through the kernel and spills the 17-prime
// instance's.)
template <int L, bool FUSED, int A>
__global__ void __launch_bounds__(256) k_scale(int n, size_t n_poly, double* dt, Tables tb) {
  constexpr int LB = L + 1;
  const PolyBlock pb = poly_block(n, n_poly);
  // FUSED has a block barrier below: its launcher requires N to be a
  // multiple of the block, so pb.ok is the same for every thread of a block
  // and a block returns here as a whole or not at all (returning after the
  // barrier instead costs 8 VGPRs and a wave per SIMD)
  if (!pb.ok) return;
  const auto rs = make_rsrc(dt + pb.pc * (size_t)(L + LB) * n, (unsigned)((L + LB) * n * 8));
  CoefSrc cs{(unsigned)pb.c * 8, 0u, 0u, 1.0, false};
  if constexpr (FUSED) {
    const int t = (int)threadIdx.x, lane = t & 63;
    const int cp = ((pb.c - t) >> 1) + (t >> 6) * 32 + (lane & 31);
    cs.hi = lane >= 32;
    cs.vu = (unsigned)cp * 8;
    cs.vv = (unsigned)(cp + (n >> 1)) * 8;
    cs.v = cs.hi ? cs.vv : cs.vu;
    cs.sg = cs.hi ? -1.0 : 1.0;
  }
  // FUSED: the two rows of t_qhinv and c1 copied into LDS once per block,
  // so that each lane's constant (lower or upper row) is an LDS read that
  // half a wave shares, not a vector memory load
  __shared__ double kl[FUSED ? 2 * (L + LB) : 1];
  if constexpr (FUSED) {
    const int t = (int)threadIdx.x;
    if (t < 2 * L) kl[t] = tb.t_qhinv[t];
    if (t < 2 * LB) kl[2 * L + t] = tb.c1[t];
    __syncthreads();
  }
  const unsigned vo = cs.v;
  const unsigned ls = (unsigned)n * 8;   // bytes per limb
  const bool third = pb.pc % 3 == 2;
  double y[L];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int iq = opaque_idx(i);
    const double p = cld(tb.p, iq), pinv = cld(tb.pinv, iq);
    y[i] = mul_bal(coef_load_both<FUSED>(rs, cs, i * ls),
                   coef_const<FUSED>(cs, FUSED ? kl : tb.t_qhinv, iq, L), p, pinv);
    S += y[i] * pinv;
  }
  double v = __builtin_rint(S);
  if (lift_near_half(S, v, tb)) {
    double r[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
      r[i] = to_canonical(mul_bal(coef_load_both<FUSED>(rs, cs, i * ls),
                                  coef_const<FUSED>(cs, tb.t_q, i, L), p, pinv),
                          p);
    }
    v = __builtin_floor(S) + (mrc_greater_than_half<L>(r, tb.p, tb.pinv, tb.mrc_inv, tb.mrc_half) ? 1.0 : 0.0);
    atomicAdd(tb.margin + (FUSED ? MARGIN_SCALE_SPLIT : MARGIN_SCALE), 1ull);
  }
  // Split conversions (conv_row).  The base-B residues w_k wait in LDS (this
  // thread's own slots, [LB][blockDim]) between the two conversions, so
  // that the split inputs of one and of the other are never live together.
  // Every sum before a reduction stays below 2^53 (at most (L / 4 + 7.2 +
  // 1.75 + L/2 + 1) 2^48), where reduce_bal is exact with its result within
  // p/2 + 4, so |w_k| <= 2^48.
  extern __shared__ double wpark[];
  double* wp = wpark + threadIdx.x;
  const int bs = (int)blockDim.x;
  double S2 = 0.0;
  {
    double yh[L], yl[L];
#pragma unroll
    for (int i = 0; i < L; ++i) split24(y[i], yh[i], yl[i]);
#pragma unroll
    for (int k = 0; k < LB; ++k) {
      const int kq = opaque_idx(k), pk = L + kq;
      const double b = cld(tb.p, pk), binv = cld(tb.pinv, pk);
      const double* sp = opaque_row(tb.c2_sp, k * L * 2);
      const double acc = mul_lazy(coef_load_both<FUSED>(rs, cs, (L + k) * ls),
                                  coef_const<FUSED>(cs, FUSED ? kl + 2 * L : tb.c1, kq, LB), b, binv) +
                         v * cld(tb.b_hat_inv, kq) -
                         conv_row<L>(yh, yl, sp, b, binv);
      const double w = reduce_bal(acc, b, binv);
      wp[k * bs] = w;
      S2 += w * binv;
    }
  }
  const double v2 = __builtin_rint(S2);
  if (__builtin_fabs(S2 - v2) > 0.25) atomicAdd(tb.margin + MARGIN_FAULT, 1ull);
  double wh[LB], wl[LB];
#pragma unroll
  for (int k = 0; k < LB; ++k) split24(wp[k * bs], wh[k], wl[k]);
  const bool pairs = A > 1 && third;
  double grp[A];   // the current digit group's canonical mixed-radix digits
#pragma unroll
  for (int k = 0; k < A; ++k) grp[k] = 0.0;
  // where the outputs go: in place, or the digit source's own buffer and
  // position (see src above).  Every input has been read by now; formed
  // here, the destination's scalars are live only in this loop.
  // (three-prime digits only: with 16 or 17 primes the destination's
  // scalars spill the conversions' constants, measured slower)
  const bool own = A == 3 && third && tb.dig_src;
  const auto rw = make_rsrc(own ? tb.dig_src + (pb.pc / 3) * (size_t)(2 * (L + A)) * n
                                : dt + pb.pc * (size_t)(L + LB) * n,
                            (unsigned)((own ? L : L + LB) * n * 8));
  const unsigned wo = own ? (((vo >> 3) & 1u) * (unsigned)(n >> 1) + (vo >> 4)) * 8u : vo;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int iq = opaque_idx(i);
    const double q = cld(tb.p, iq), qinv = cld(tb.pinv, iq);
    const double* sp = opaque_row(tb.b_hat_q_sp, i * LB * 2);
    const double acc = conv_row<LB>(wh, wl, sp, q, qinv) -
                       v2 * cld(tb.B_q, iq);
    const double r = reduce_bal(acc, q, qinv);
    // the third component is only read as relinearization digits: its
    // canonical residues, or with A primes per digit each digit's canonical
    // mixed-radix digits (Garner: limb g + m of the group starting at g gets
    // v_m = t_m, t_0 = d_{g+m}, t_{k+1} = [(t_k - v_k) q_{g+k}^-1]_{q_{g+m}};
    // every difference is below 2^49 < 2 q)
    double o = third ? to_canonical(r, q) : r;
    if constexpr (A > 1) {
      const int m = i % A;
      if (pairs && m > 0) {
        double tt = o;
#pragma unroll
        for (int k = 0; k < m; ++k)
          tt = mul_bal(tt - grp[k], cld(tb.mrc_inv, (iq - m + k) * L + iq), q, qinv);
        o = to_canonical(tt, q);
      }
      grp[m] = o;
    }
    buf_store(o, rw, wo, i * ls);
  }
}

// ---------------------------------------------------------- key switching ---

// acc[ct][b][i] = sum_j dig[ct][j][i] * evk[j][b][i] (NTT domain) over the
// L / A digits, limbs i = 0..L+A-1 (the last A mod the special primes).
// The key is read once per chunk of CH ciphertexts.
template <int L, int A, int CH>
__global__ void __launch_bounds__(256) k_ks_mac(int n, int n_ct, const double* dig,
                                                const double* evk, double* acc, Tables tb) {
  constexpr int K = L + A;
  constexpr int DN = L / A;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)K * n) return;
  const int i = (int)(gid / n);
  const int c = (int)(gid - (size_t)i * n);
  const int prime = i < L ? i : L + 1 + i;
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  for (int c0 = 0; c0 < n_ct; c0 += CH) {
    double a0[CH], a1[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) a0[u] = a1[u] = 0.0;
    for (int j = 0; j < DN; ++j) {
      const double e0 = evk[((size_t)(j * 2 + 0) * K + i) * n + c];
      const double e1 = evk[((size_t)(j * 2 + 1) * K + i) * n + c];
      // every load of the chunk is issued before the products: past the
      // last ciphertext the index is clamped (a valid address) and the
      // result is never stored
      double dv[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int cu = c0 + u < n_ct ? c0 + u : n_ct - 1;
        dv[u] = __builtin_nontemporal_load(&dig[((size_t)(cu * DN + j) * K + i) * n + c]);
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        a0[u] += mul_lazy(dv[u], e0, p, pinv);
        a1[u] += mul_lazy(dv[u], e1, p, pinv);
      }
      // digit transforms are not reduced at their end: |dv| < 15.1 p (at
      // most ten unreduced stages from inputs below 2.61 p, the bound of a
      // two-prime digit's value; 13.5 p from one-prime digits below 2 p and
      // from three-prime digits, reduced to balanced form first;
      // 6.1 p at N = 2^15), so each product with a balanced key is below
      // (1/2 + 0.094 x 15.1) p = 1.92 p and eight of them plus a reduced sum
      // stay below 15.9 p < 2^53 / p (> 16.6 p for p < 2^48.95): reduce the
      // sums every 8 digits
      if ((j & 7) == 7) {
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          a0[u] = reduce_bal(a0[u], p, pinv);
          a1[u] = reduce_bal(a1[u], p, pinv);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (c0 + u < n_ct) {
        acc[((size_t)((c0 + u) * 2 + 0) * K + i) * n + c] = reduce_bal(a0[u], p, pinv);
        acc[((size_t)((c0 + u) * 2 + 1) * K + i) * n + c] = reduce_bal(a1[u], p, pinv);
      }
    }
  }
}

// k_ks_mac for digit transforms by coefficient parity (k_ntt_fwd_par,
// N = 2^15): half 0 of a digit's limb holds E, half 1 holds O, both in the
// 2^14 transform's order (standard index k at (k mod 32) 512 + k / 32).
// Thread (u, m), u < 16, m < 1024, takes k = 16 m + u, whose values in the
// full transform are X_0 = E_k + z O_k and X_1 = E_k - z O_k (z =
// psi^brv(2^14 + k), tw_last), at its standard positions 2k and 2k + 1:
// stored, as the key and the sums are, at 2u 1024 + m and (2u + 1) 1024 + m
// (consecutive threads, consecutive addresses); E_k and O_k sit at
// (16 (m mod 2) + u) 512 + m / 2.  The sums are those of k_ks_mac.
// Bounds: |E|, |O| < 5.9 p, so |X| < 7 p and each product with a balanced
// key is below 1.16 p: eight of them plus a reduced sum stay below 15.9 p.
template <int L, int A, int CH>
__global__ void __launch_bounds__(256) k_ks_mac_par(int n_ct, const double* dig,
                                                    const double* evk, double* acc, Tables tb) {
  constexpr int K = L + A;
  constexpr int DN = L / A;
  constexpr int NF = 1 << 15, NH = NF / 2;
  const int gid = blockIdx.x * 256 + threadIdx.x;
  if (gid >= K * NH) return;
  const int i = gid >> 14;
  const int t = gid & (NH - 1);
  const int u = t >> 10, m = t & 1023;
  const int prime = i < L ? i : L + 1 + i;
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const double z = tb.tw_last[(size_t)i * NH + t];
  const size_t pe = (size_t)(((m & 1) << 4) + u) * 512 + (m >> 1);
  const size_t p0 = (size_t)(2 * u) * 1024 + m;
  for (int c0 = 0; c0 < n_ct; c0 += CH) {
    // [key component][position] per ciphertext of the chunk
    double a00[CH], a01[CH], a10[CH], a11[CH];
#pragma unroll
    for (int v = 0; v < CH; ++v) a00[v] = a01[v] = a10[v] = a11[v] = 0.0;
    for (int j = 0; j < DN; ++j) {
      const double* kj = evk + ((size_t)(j * 2) * K + i) * NF + p0;
      const double e00 = kj[0], e01 = kj[1024];
      const double e10 = kj[(size_t)K * NF], e11 = kj[(size_t)K * NF + 1024];
      // every load of the chunk is issued before the products: past the
      // last ciphertext the index is clamped (a valid address) and the
      // result is never stored
      double ev[CH], od[CH];
#pragma unroll
      for (int v = 0; v < CH; ++v) {
        const int cv = c0 + v < n_ct ? c0 + v : n_ct - 1;
        const double* dp = dig + ((size_t)(cv * DN + j) * K + i) * NF + pe;
        ev[v] = __builtin_nontemporal_load(dp);
        od[v] = __builtin_nontemporal_load(dp + NH);
      }
#pragma unroll
      for (int v = 0; v < CH; ++v) {
        const double w = mul_lazy(od[v], z, p, pinv);
        const double x0 = ev[v] + w, x1 = ev[v] - w;
        a00[v] += mul_lazy(x0, e00, p, pinv);
        a01[v] += mul_lazy(x1, e01, p, pinv);
        a10[v] += mul_lazy(x0, e10, p, pinv);
        a11[v] += mul_lazy(x1, e11, p, pinv);
      }
      if ((j & 7) == 7) {
#pragma unroll
        for (int v = 0; v < CH; ++v) {
          a00[v] = reduce_bal(a00[v], p, pinv);
          a01[v] = reduce_bal(a01[v], p, pinv);
          a10[v] = reduce_bal(a10[v], p, pinv);
          a11[v] = reduce_bal(a11[v], p, pinv);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < CH; ++v) {
      if (c0 + v < n_ct) {
        double* o0 = acc + ((size_t)((c0 + v) * 2 + 0) * K + i) * NF + p0;
        double* o1 = acc + ((size_t)((c0 + v) * 2 + 1) * K + i) * NF + p0;
        o0[0] = reduce_bal(a00[v], p, pinv);
        o0[1024] = reduce_bal(a01[v], p, pinv);
        o1[0] = reduce_bal(a10[v], p, pinv);
        o1[1024] = reduce_bal(a11[v], p, pinv);
      }
    }
  }
}

// A special limb's residues [N^-1 x]_{P_k} (balanced) at coefficients c and
// c + N/2 from the split inverse's half outputs U (at a) and V (at a + ht):
// the inverse's last stage (U + V, (U - V) w) applied here.
__device__ __forceinline__ void special_pair(const double* a, int ht, int ip, double& lo,
                                             double& hi, const Tables& tb) {
  const double pk = cld(tb.p, ip), pkinv = cld(tb.pinv, ip);
  const double u = a[0], v = a[ht];
  const double ninvk = cld(tb.ninv, ip);
  lo = mul_bal(u + v, ninvk, pk, pkinv);
  hi = mul_bal(mul_lazy(u - v, cld(tb.tw_inv, ip * tb.tw_len + 1), pk, pkinv), ninvk, pk, pkinv);
}

// The centred residue r = [x]_P of a key-switch sum, P = P_0 ... P_{A-1},
// in mixed radix r = k_0 + P_0 k_1 + P_0 P_1 k_2 from its balanced residues
// a_m mod P_m (Garner, every digit balanced): k_0 = a_0,
// k_1 = [(a_1 - a_0) P_0^-1]_{P_1}, k_2 = [((a_2 - a_0) P_0^-1 - k_1) P_1^-1]_{P_2}
// (each difference below 2 P_m: all primes lie in [2^48, 2^49)).  With
// balanced digits |r| <= sum_m (P_m - 1)/2 prod_{l<m} P_l = (P - 1)/2: r is
// exactly the centred residue, with no comparison.
template <int A>
__device__ __forceinline__ void special_digits(const double (&a)[A], double (&k)[A],
                                               const Tables& tb, int L) {
  k[0] = a[0];
  if constexpr (A >= 2) {
    const int ip1 = 2 * L + 2;
    k[1] = mul_bal(a[1] - a[0], tb.p_inv_p[0], cld(tb.p, ip1), cld(tb.pinv, ip1));
  }
  if constexpr (A >= 3) {
    const int ip2 = 2 * L + 3;
    const double p2 = cld(tb.p, ip2), p2inv = cld(tb.pinv, ip2);
    const double t = mul_bal(a[2] - a[0], tb.p_inv_p[1], p2, p2inv);
    k[2] = mul_bal(t - k[1], tb.p_inv_p[2], p2, p2inv);
  }
}

// (x - r) P^-1 mod q_i up to the factor N^-1 folded into npq: x times
// [N^-1 P^-1]_{q_i} minus r's mixed-radix digits k_m times
// [(P_0 ... P_{m-1}) P^-1]_{q_i}.  Each lazy product is below 0.9 q_i
// (operands below 2 q_i), so the result is below 3.6 q_i.
template <int L, int A>
__device__ __forceinline__ double moddown_term(double x, double npq, const double (&k)[A], int i,
                                               double q, double qinv, const Tables& tb) {
  double r = mul_lazy(x, npq, q, qinv) - mul_lazy(k[0], cld(tb.P_inv_q, i), q, qinv);
#pragma unroll
  for (int m = 1; m < A; ++m) r -= mul_lazy(k[m], cld(tb.mr_q, (m - 1) * L + i), q, qinv);
  return r;
}

// new ct (into ext limbs 0..L-1) = e_b + (acc_b - [acc_b]_P) * P^-1, where
// [acc_b]_P is the centred residue mod P of the special limbs (special_k).
// Since mul_lazy(a0, .) needs |a0| < 2p only, P_k may exceed q_i (all
// < 2^49).
// FUSED: acc holds the split inverse's in-place half outputs of a 2^15-point
// limb (U of pair c at (c / 512) 1024 + c mod 512, V 512 further; see
// k_ntt_inv_half) and a thread produces both coefficients c and c + N/2.
template <int L, int A, bool FUSED>
__global__ void __launch_bounds__(256) k_moddown(int n, int n_ct, const double* __restrict__ acc,
                                                 const double* __restrict__ dt,
                                                 double* __restrict__ ext, int accumulate,
                                                 Tables tb) {
  constexpr int K = L + A;
  constexpr int W = 2 * L + 1;
  const int per = FUSED ? n >> 1 : n;      // threads per (ct, component)
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * 2 * per) return;
  const size_t cb = gid / per;             // ct * 2 + b
  const int c = (int)(gid - cb * per);
  const size_t ct = cb >> 1;
  const int b = (int)(cb & 1);
  const int ip = 2 * L + 1;
  const double* e = dt + ((ct * 3 + b) * (size_t)W) * n + c;
  double* o = ext + cb * (size_t)W * n + c;
  if constexpr (!FUSED) {
    const double* a = acc + cb * (size_t)K * n + c;
    // acc is inverse-transform output (N times the sum): the residues mod
    // the special primes are [N^-1 acc_Pk]_Pk
    double as[A], kP[A];
#pragma unroll
    for (int m = 0; m < A; ++m)
      as[m] = mul_bal(a[(size_t)(L + m) * n], cld(tb.ninv, ip + m), cld(tb.p, ip + m),
                      cld(tb.pinv, ip + m));
    special_digits<A>(as, kP, tb, L);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const double q = cld(tb.p, i), qinv = cld(tb.pinv, i);
      const double r = moddown_term<L, A>(a[(size_t)i * n], cld(tb.NP_inv_q, i), kP, i, q, qinv, tb);
      const double z = reduce_bal(e[(size_t)i * n] + r, q, qinv);
      o[(size_t)i * n] = accumulate ? reduce_bal(o[(size_t)i * n] + z, q, qinv) : z;
    }
  } else {
    const int ht = n >> 6;                 // 512: a half transform's threads
    const double* a = acc + cb * (size_t)K * n + (size_t)(c / ht) * 2 * ht + (c % ht);
    const size_t hn = (size_t)(n >> 1);
    double s_lo[A], s_hi[A], k_lo[A], k_hi[A];
#pragma unroll
    for (int m = 0; m < A; ++m)
      special_pair(a + (size_t)(L + m) * n, ht, ip + m, s_lo[m], s_hi[m], tb);
    special_digits<A>(s_lo, k_lo, tb, L);
    special_digits<A>(s_hi, k_hi, tb, L);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const double q = cld(tb.p, i), qinv = cld(tb.pinv, i);
      const double u = a[(size_t)i * n], v = a[(size_t)i * n + ht];
      const double lo = u + v;
      const double hi = mul_lazy(u - v, cld(tb.tw_inv, i * tb.tw_len + 1), q, qinv);
      const double npq = cld(tb.NP_inv_q, i);
      const double r_lo = moddown_term<L, A>(lo, npq, k_lo, i, q, qinv, tb);
      const double r_hi = moddown_term<L, A>(hi, npq, k_hi, i, q, qinv, tb);
      const double z_lo = reduce_bal(e[(size_t)i * n] + r_lo, q, qinv);
      const double z_hi = reduce_bal(e[(size_t)i * n + hn] + r_hi, q, qinv);
      o[(size_t)i * n] = accumulate ? reduce_bal(o[(size_t)i * n] + z_lo, q, qinv) : z_lo;
      o[(size_t)i * n + hn] = accumulate ? reduce_bal(o[(size_t)i * n + hn] + z_hi, q, qinv) : z_hi;
    }
  }
}

// A mod-down (split inverse, pairs as in k_moddown FUSED) written straight
// to the caller's int64 output, canonical residues in [0, q_i): with finish,
// the mask's finish out = (Delta, 0) - z (every residue negated and
// [Delta]_{q_i} added to the constant coefficient of c0); without, z.
// wt (table not null): a batched wave's ciphertexts, written through the
// table's out pointers.
template <int L, int A>
__global__ void __launch_bounds__(256) k_moddown_finish(int n, int n_ct,
                                                        const double* __restrict__ acc,
                                                        const double* __restrict__ dt,
                                                        int64_t* __restrict__ out, int finish,
                                                        Tables tb, WaveTab wt) {
  constexpr int K = L + A;
  constexpr int W = 2 * L + 1;
  const int per = n >> 1;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * 2 * per) return;
  const size_t cb = gid / per;             // ct * 2 + b
  const int c = (int)(gid - cb * per);
  const size_t ct = cb >> 1;
  const int b = (int)(cb & 1);
  const int ip = 2 * L + 1;
  const double* e = dt + ((ct * 3 + b) * (size_t)W) * n + c;
  int64_t* o = wt.table ? wt.table[(size_t)(*wt.wave) * wt.stride + ct].out + (size_t)b * L * n + c
                        : out + cb * (size_t)L * n + c;
  const int ht = n >> 6;
  const double* a = acc + cb * (size_t)K * n + (size_t)(c / ht) * 2 * ht + (c % ht);
  const size_t hn = (size_t)(n >> 1);
  double s_lo[A], s_hi[A], k_lo[A], k_hi[A];
#pragma unroll
  for (int m = 0; m < A; ++m)
    special_pair(a + (size_t)(L + m) * n, ht, ip + m, s_lo[m], s_hi[m], tb);
  special_digits<A>(s_lo, k_lo, tb, L);
  special_digits<A>(s_hi, k_hi, tb, L);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const double q = cld(tb.p, i), qinv = cld(tb.pinv, i);
    const double u = a[(size_t)i * n], v = a[(size_t)i * n + ht];
    const double lo = u + v;
    const double hi = mul_lazy(u - v, cld(tb.tw_inv, i * tb.tw_len + 1), q, qinv);
    const double npq = cld(tb.NP_inv_q, i);
    const double r_lo = moddown_term<L, A>(lo, npq, k_lo, i, q, qinv, tb);
    const double r_hi = moddown_term<L, A>(hi, npq, k_hi, i, q, qinv, tb);
    // finish: -(e + r), plus Delta at coefficient 0 of c0 (sg = -1 exactly
    // negates); else e + r
    const double sg = finish ? -1.0 : 1.0;
    double z_lo = sg * (e[(size_t)i * n] + r_lo);
    if (finish && b == 0 && c == 0) z_lo += cld(tb.delta_q, i);
    const double z_hi = sg * (e[(size_t)i * n + hn] + r_hi);
    o[(size_t)i * n] = to_i64(reduce_bal(z_lo, q, qinv), q);
    o[(size_t)i * n + hn] = to_i64(reduce_bal(z_hi, q, qinv), q);
  }
}

// The rest of a lift whose L residues o (balanced) and y_i = [o_i
// (Q/q_i)^-1]_{q_i}, S = sum_i y_i / q_i are already in registers: the
// overflow count v (exact fallback near a half-integer, as k_lift), then
// limbs L..2L of rs at vo.
template <int L, int SITE>
__device__ __forceinline__ void lift_tail(const double (&o)[L], const double (&y)[L], double S,
                                          __amdgpu_buffer_rsrc_t rs, unsigned vo, unsigned ls,
                                          const Tables& tb) {
  constexpr int LB = L + 1;
  double v = __builtin_rint(S);
  if (lift_near_half(S, v, tb)) {
    double r[L];
#pragma unroll
    for (int i = 0; i < L; ++i) r[i] = to_canonical(o[i], cld(tb.p, i));
    v = __builtin_floor(S) + (mrc_greater_than_half<L>(r, tb.p, tb.pinv, tb.mrc_inv, tb.mrc_half) ? 1.0 : 0.0);
    atomicAdd(tb.margin + SITE, 1ull);
  }
  double yh[L], yl[L];
#pragma unroll
  for (int i = 0; i < L; ++i) split24(y[i], yh[i], yl[i]);
#pragma unroll
  for (int k = 0; k < LB; ++k) {
    const int kq = opaque_idx(k), pk = L + kq;
    const double bb = cld(tb.p, pk), binv = cld(tb.pinv, pk);
    const double* sp = opaque_row(tb.q_hat_b_sp, k * L * 2);
    const double a = conv_row<L>(yh, yl, sp, bb, binv) -
                     v * cld(tb.Q_b, kq);
    buf_store(reduce_bal(a, bb, binv), rs, vo, (L + k) * ls);
  }
}

// The mod-down of the split inverse's output (k_moddown, FUSED) followed by
// the lift of its result (k_lift): within the squaring chain the next level
// lifts exactly what this level's mod-down writes, so one kernel saves
// re-reading it.  One thread per coefficient of each (ct, b) polynomial
// (blocks mapped like k_lift); lanes l and l + 32 of a wave hold the two
// coefficients of a pair (c, c + N/2) and exchange the key-switch sum's half
// outputs as the scale-and-round does, with the last inverse stage's
// twiddle folded into the second rows of NP_inv_q and ninv_P.
template <int L, int A>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_moddown_lift(int n, size_t n_poly,
                                                      const double* __restrict__ acc,
                                                      const double* __restrict__ dt,
                                                      double* __restrict__ ext, Tables tb) {
  constexpr int K = L + A;
  constexpr int W = 2 * L + 1;
  const PolyBlock pb = poly_block(n, n_poly);   // poly = ct * 2 + b
  if (!pb.ok) return;
  const int t = (int)threadIdx.x, lane = t & 63;
  const int cp = ((pb.c - t) >> 1) + (t >> 6) * 32 + (lane & 31);
  const bool hi = lane >= 32;
  const double sg = hi ? -1.0 : 1.0;
  const int ht = n >> 6;                         // 512: see k_ntt_inv_half
  const unsigned pos = (unsigned)((cp / ht) * 2 * ht + cp % ht + (hi ? ht : 0)) * 8;
  const unsigned vo = (unsigned)(cp + (hi ? n >> 1 : 0)) * 8;
  const unsigned ls = (unsigned)n * 8;
  const size_t cb = pb.pc, ct = cb >> 1;
  const int b = (int)(cb & 1);
  const auto ra = make_rsrc(acc + cb * (size_t)K * n, (unsigned)(K * n * 8));
  const auto re = make_rsrc(dt + (ct * 3 + b) * (size_t)W * n, (unsigned)(L * n * 8));
  const auto rs = make_rsrc(ext + cb * (size_t)W * n, (unsigned)(W * n * 8));
  const int row = hi ? 1 : 0;
  // [N^-1 acc_Pk]_Pk of this coefficient (balanced), then the centred
  // residue's mixed-radix digits
  const int ip = 2 * L + 1;
  double as[A], kP[A];
#pragma unroll
  for (int m = 0; m < A; ++m) {
    const double xP = buf_load(ra, pos, (L + m) * ls);
    as[m] = mul_bal(pair_combine(xP, sg), tb.ninv_P[2 * m + row], cld(tb.p, ip + m),
                    cld(tb.pinv, ip + m));
  }
  special_digits<A>(as, kP, tb, L);
  // the new ciphertext's residues are stored only after every load: buffer
  // stores between them would make each limb's loads wait for the previous
  // limb's (the compiler cannot tell the buffers apart)
  double o[L], y[L];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int iq = opaque_idx(i);
    const double q = cld(tb.p, iq), qinv = cld(tb.pinv, iq);
    const double x = buf_load(ra, pos, i * ls);
    const double r =
        moddown_term<L, A>(pair_combine(x, sg), tb.NP_inv_q[row * L + iq], kP, iq, q, qinv, tb);
    o[i] = reduce_bal(buf_load(re, vo, i * ls) + r, q, qinv);
    y[i] = mul_bal(o[i], cld(tb.q_hat_inv, iq), q, qinv);
    S += y[i] * qinv;
  }
#pragma unroll
  for (int i = 0; i < L; ++i) buf_store(o[i], rs, vo, i * ls);
  lift_tail<L, MARGIN_MODDOWN_LIFT>(o, y, S, rs, vo, ls, tb);
}

// Subtraction z = [x - y]_Q of two ciphertexts (int64, canonical; y one
// ciphertext broadcast when y_bcast) into ext limbs 0..L-1, followed by the
// lift of z (limbs L..2L): the first level of the chain, one kernel.  One
// thread per coefficient of each (ct, b) polynomial, blocks as in k_lift.
// wt (table not null): a batched wave's ciphertexts, x and y read through
// the table (a broadcast y is every entry's y).
template <int L>
__global__ void __launch_bounds__(256) k_sub_lift(int n, size_t n_poly,
                                                  const int64_t* __restrict__ xs,
                                                  const int64_t* __restrict__ ys, int y_bcast,
                                                  double* __restrict__ ext, Tables tb, WaveTab wt) {
  constexpr int W = 2 * L + 1;
  const PolyBlock pb = poly_block(n, n_poly);   // poly = ct * 2 + b
  if (!pb.ok) return;
  const size_t cb = pb.pc;
  const int b = (int)(cb & 1);
  const int64_t* xp;
  const int64_t* yp;
  if (wt.table) {
    const CtPtrs e = wt.table[(size_t)(*wt.wave) * wt.stride + (cb >> 1)];
    xp = e.x + (size_t)b * L * n + pb.c;
    yp = e.y + (size_t)b * L * n + pb.c;
  } else {
    xp = xs + cb * (size_t)L * n + pb.c;
    yp = (y_bcast ? ys + (size_t)b * L * n : ys + cb * (size_t)L * n) + pb.c;
  }
  const auto rs = make_rsrc(ext + cb * (size_t)W * n, (unsigned)(W * n * 8));
  const unsigned vo = (unsigned)pb.c * 8, ls = (unsigned)n * 8;
  double o[L], y[L];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int iq = opaque_idx(i);
    const double q = cld(tb.p, iq), qinv = cld(tb.pinv, iq);
    o[i] = reduce_bal((double)xp[(size_t)i * n] - (double)yp[(size_t)i * n], q, qinv);
    y[i] = mul_bal(o[i], cld(tb.q_hat_inv, iq), q, qinv);
    S += y[i] * qinv;
  }
#pragma unroll
  for (int i = 0; i < L; ++i) buf_store(o[i], rs, vo, i * ls);
  lift_tail<L, MARGIN_SUB_LIFT>(o, y, S, rs, vo, ls, tb);
}

// Canonical int64 residues of n_poly polynomials ([n_poly][L][N]) into ext
// limbs 0..L-1 (balanced) and their lift into limbs L..2L: the conversion
// (k_i64_to_polys) and k_lift in one pass, the same arithmetic.
template <int L>
__global__ void __launch_bounds__(256) k_i64_lift(int n, size_t n_poly,
                                                  const int64_t* __restrict__ in,
                                                  double* __restrict__ ext, Tables tb) {
  constexpr int W = 2 * L + 1;
  const PolyBlock pb = poly_block(n, n_poly);
  if (!pb.ok) return;
  const int64_t* ip = in + pb.pc * (size_t)L * n + pb.c;
  const auto rs = make_rsrc(ext + pb.pc * (size_t)W * n, (unsigned)(W * n * 8));
  const unsigned vo = (unsigned)pb.c * 8, ls = (unsigned)n * 8;
  double o[L], y[L];
  double S = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int iq = opaque_idx(i);
    const double q = cld(tb.p, iq), qinv = cld(tb.pinv, iq);
    o[i] = from_u64(ip[(size_t)i * n], q);
    y[i] = mul_bal(o[i], cld(tb.q_hat_inv, iq), q, qinv);
    S += y[i] * qinv;
  }
#pragma unroll
  for (int i = 0; i < L; ++i) buf_store(o[i], rs, vo, i * ls);
  lift_tail<L, MARGIN_I64_LIFT>(o, y, S, rs, vo, ls, tb);
}

// ------------------------------------------------------ plaintext products ---

// The basis plaintext of one slot: m_i = N^-1 zeta^-i mod t, zinv = zeta^-1
// for the slot's root zeta (t < 2^24, so products fit 64 bits).
__global__ void __launch_bounds__(256) k_basis_plain(int n, uint64_t t, uint64_t zinv,
                                                     uint64_t ninv_t, int64_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t r = 1, b = zinv;
  for (unsigned e = (unsigned)i; e; e >>= 1) {
    if (e & 1) r = r * b % t;
    b = b * b % t;
  }
  out[i] = (int64_t)(r * ninv_t % t);
}

// Plaintext polynomial (int64 [N] in [0, t)) -> its centred value times
// N^-1 in each data prime (limbs 0..L-1 at stride N): the operand of a
// pointwise product whose inverse transform returns N times the result.
__global__ void __launch_bounds__(256) k_plain_limbs(int n, int L, int64_t t, const int64_t* pt,
                                                     double* out, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)L * n) return;
  const int i = (int)(gid / n);
  const int c = (int)(gid - (size_t)i * n);
  const int64_t v = pt[c];
  const double x = (double)(v > t / 2 ? v - t : v);
  out[gid] = mul_bal(x, cld(tb.ninv, i), cld(tb.p, i), cld(tb.pinv, i));
}

// fx[ct][b][i] *= pt[i] (NTT domain, data limbs of [ct][2][W][N]).
__global__ void __launch_bounds__(256) k_pointwise_plain(int n, int L, int n_ct, double* fx,
                                                         const double* pt, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * 2 * L * n) return;
  const size_t row = gid / n;
  const int c = (int)(gid - row * n);
  const int i = (int)(row % L);
  const size_t cb = row / L;
  const size_t off = (cb * (2 * L + 1) + i) * n + c;
  fx[off] = mul_bal(fx[off], pt[(size_t)i * n + c], cld(tb.p, i), cld(tb.pinv, i));
}

// ----------------------------------------------------------- comparisons ---

// acc += the tensor of two transformed operands (acc = it when first):
// per limb of the extended basis, pointwise in the NTT domain, d0 = a0 b0,
// d1 = a0 b1 + a1 b0, d2 = a1 b1, each running sum kept as a balanced
// residue.  fa, fb: [n_ct][2][W][N] (balanced transform outputs); acc:
// [n_ct][3][W][N].  Summing products' tensors before one scale-and-round
// is exact while the sum stays inside the extended basis' range.
__global__ void __launch_bounds__(256) k_tensor_mac(int n, int W, size_t total,
                                                    const double* __restrict__ fa,
                                                    const double* __restrict__ fb,
                                                    double* __restrict__ acc, int first,
                                                    Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t per = (size_t)W * n;
  const size_t ct = gid / per, r = gid - ct * per;
  const int l = (int)(r / n);                 // extended-basis limb = prime index
  const double p = cld(tb.p, l), pinv = cld(tb.pinv, l);
  const double* a = fa + ct * 2 * per + r;
  const double* b = fb + ct * 2 * per + r;
  double* o = acc + ct * 3 * per + r;
  const double a0 = a[0], a1 = a[per], b0 = b[0], b1 = b[per];
  double d0 = mul_lazy(a0, b0, p, pinv);
  double d1 = mul_lazy(a0, b1, p, pinv) + mul_lazy(a1, b0, p, pinv);
  double d2 = mul_lazy(a1, b1, p, pinv);
  if (!first) {
    d0 += o[0];
    d1 += o[per];
    d2 += o[2 * per];
  }
  o[0] = reduce_bal(d0, p, pinv);
  o[per] = reduce_bal(d1, p, pinv);
  o[2 * per] = reduce_bal(d2, p, pinv);
}

// out[jj * out_stride + r] = [sum_t coef[jj * k + t] * b.p[t][r]]_q per
// residue r < per, jj < J <= 16 (int64 canonical in and out).
// Coefficients are small centred integers (|c| <= 2^15: the comparison
// polynomial's coefficients mod a Fermat prime t <= 65537), stored as
// doubles (exact) and uniform across the grid: scalar loads that the FMAs
// take as they are, with no conversion per use.  Each input v (balanced, |v| <= 2^48) is
// split once as v = vh 2^24 + vl (split24), so that every product is an
// exact FMA (|vh c| <= 2^39): two exact sums per output over k <= 256
// terms (below 2^47), combined once as Wh [2^24]_q + Wl.  JT: J fixed at
// compile time (16 or 1), or 0 for any J (a branch per output and term).
template <int JT>
__global__ void __launch_bounds__(256) k_lincomb(int n, int L, size_t per, int k, BabyPtrs b,
                                                 const double* coef, int Jr, int64_t* out,
                                                 size_t out_stride, Tables tb) {
  const int J = JT ? JT : Jr;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= per) return;
  const int i = (int)((gid / n) % L);
  const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
  double ah[16], al[16];
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) ah[jj] = al[jj] = 0.0;
  // babies in groups of G whose loads are all issued before their products
  // (one load per term would leave the loop waiting on memory latency)
  constexpr int G = 4;
  int t = 0;
  for (; t + G <= k; t += G) {
    double vh[G], vl[G];
#pragma unroll
    for (int u = 0; u < G; ++u) split24(from_u64(b.p[t + u][gid], p), vh[u], vl[u]);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      if (jj < J) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const double c = cld(coef, jj * k + t + u);
          ah[jj] = __builtin_fma(vh[u], c, ah[jj]);
          al[jj] = __builtin_fma(vl[u], c, al[jj]);
        }
      }
    }
  }
  for (; t < k; ++t) {
    double vh, vl;
    split24(from_u64(b.p[t][gid], p), vh, vl);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      if (jj < J) {
        const double c = cld(coef, jj * k + t);
        ah[jj] = __builtin_fma(vh, c, ah[jj]);
        al[jj] = __builtin_fma(vl, c, al[jj]);
      }
    }
  }
  const double t24 = cld(tb.two24, i);
#pragma unroll
  for (int jj = 0; jj < 16; ++jj)
    if (jj < J)
      out[(size_t)jj * out_stride + gid] =
          to_i64(reduce_bal(mul_lazy(ah[jj], t24, p, pinv) + al[jj], p, pinv), p);
}

// The trivial encryption (Delta, 0) of 1 in each of n_ct ciphertexts.
__global__ void __launch_bounds__(256) k_fill_one(int n, int L, size_t total, int64_t* out,
                                                  Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t row = gid / n;                 // (ct * 2 + b) * L + i
  const int c = (int)(gid - row * n);
  const int i = (int)(row % L);
  const int b = (int)((row / L) & 1);
  out[gid] = (b == 0 && c == 0) ? to_i64(cld(tb.delta_q, i), cld(tb.p, i)) : 0;
}

// out = [x - y]_Q or [y - x]_Q (negate), y broadcast over ct if y_bcast.
__global__ void __launch_bounds__(256) k_diff_i64(int n, int L, size_t total, const int64_t* x,
                                                  const int64_t* y, int y_bcast, int negate,
                                                  int64_t* out, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t per_ct = (size_t)2 * L * n;
  const int i = (int)((gid / n) % L);
  const int64_t q = (int64_t)cld(tb.p, i);
  const int64_t a = x[gid], b = y[y_bcast ? gid % per_ct : gid];
  int64_t d = negate ? b - a : a - b;
  out[gid] = d < 0 ? d + q : d;
}

// ------------------------------------------------------------- rotations ---

// Ring automorphism a(X) -> a(X^g) of the ciphertexts in ext (limbs
// 0..L-1, balanced) into the key-switching input layout of dt: component 0
// gets sigma(c0), component 1 zero, component 2 (the digit source) the
// canonical residues of sigma(c1).  Output coefficient j of sigma(a) is
// a_i for i = j g^-1 mod 2N when i < N, else -a_{i-N} (since X^N = -1).
__global__ void __launch_bounds__(256) k_automorph(int n, int L, int n_ct, unsigned ginv,
                                                   const double* ext, double* dt, Tables tb,
                                                   double* dsrc, size_t dsrc_stride,
                                                   int dsrc_split) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * 2 * L * n) return;
  const size_t row = gid / n;               // (ct * 2 + b) * L + i
  const int j = (int)(gid - row * n);
  const int i = (int)(row % L);
  const size_t cb = row / L;
  const size_t ct = cb >> 1;
  const int b = (int)(cb & 1);
  const size_t W = (size_t)2 * L + 1;
  const unsigned src = (unsigned)(((unsigned long long)j * ginv) % (2ull * n));
  const double* a = ext + (cb * W + i) * n;
  double v = src < (unsigned)n ? a[src] : -a[src - n];
  double* d = dt + (ct * 3 * W + i) * n + j;
  if (b == 0) {
    d[0] = v;
    d[W * n] = 0.0;
  } else if (dsrc) {
    // the digit source's own buffer (see k_scale)
    const int jp = dsrc_split ? (j & 1) * (n >> 1) + (j >> 1) : j;
    dsrc[ct * dsrc_stride + (size_t)i * n + jp] = to_canonical(v, cld(tb.p, i));
  } else {
    d[2 * W * n] = to_canonical(v, cld(tb.p, i));
  }
}

// The third component of dt (limbs 0..L-1) into the digit source's own
// buffer: ciphertext ct at src + ct src_stride, coefficient c at position
// (c mod 2) N/2 + c/2 (see k_scale).
__global__ void __launch_bounds__(256) k_digit_split(int n, int L, int n_ct, const double* dt,
                                                     double* src, size_t src_stride) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * L * n) return;
  const size_t row = gid / n;               // ct * L + i
  const int c = (int)(gid - row * n);
  const size_t ct = row / L;
  const int i = (int)(row - ct * L);
  const size_t W = (size_t)2 * L + 1;
  src[ct * src_stride + (size_t)i * n + (c & 1) * (n >> 1) + (c >> 1)] =
      dt[(ct * 3 * W + 2 * W + i) * n + c];
}

// A primes per key-switching digit (A = 2, 3): the digit source (limbs
// 0..L-1 of ciphertext ct at src + ct src_stride, canonical residues d_i, in
// any coefficient order) into each digit's
// canonical mixed-radix digits, in place (as k_scale writes them): limb
// g + m of the group starting at g = j A gets v_m = t_m, t_0 = d_{g+m},
// t_{k+1} = [(t_k - v_k) q_{g+k}^-1]_{q_{g+m}}, so that digit j,
// D_j = v_0 + q_g v_1 + q_g q_{g+1} v_2 in [0, Q_j), is [c]_{Q_j}.  One
// thread per (ciphertext, digit, coefficient).
template <int A>
__global__ void __launch_bounds__(256) k_digit_mrc(int n, int L, int n_ct, double* src,
                                                   size_t src_stride, Tables tb) {
  const int groups = L / A;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_ct * groups * n) return;
  const size_t row = gid / n;               // ct * groups + j
  const int c = (int)(gid - row * n);
  const int j = (int)(row % groups);
  const size_t ct = row / groups;
  const int g = j * A;
  double* d = src + ct * src_stride + (size_t)g * n + c;
  double v[A];
  v[0] = d[0];
#pragma unroll
  for (int m = 1; m < A; ++m) {
    const int ib = g + m;
    const double q = cld(tb.p, ib), qinv = cld(tb.pinv, ib);
    double t = d[(size_t)m * n];
#pragma unroll
    for (int k = 0; k < m; ++k) t = mul_bal(t - v[k], cld(tb.mrc_inv, (g + k) * L + ib), q, qinv);
    v[m] = to_canonical(t, q);
    d[(size_t)m * n] = v[m];
  }
}

// ------------------------------------------------------------ boundary ---

// ext[ct][b][i] (i < L) = balanced(x - y); y broadcast over ct if y_bcast.
__global__ void __launch_bounds__(256) k_sub_to_ext(int n, int L, int n_ct, const int64_t* x,
                                                    const int64_t* y, int y_bcast, double* ext,
                                                    Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per_ct = (size_t)2 * L * n;
  if (gid >= (size_t)n_ct * per_ct) return;
  const size_t ct = gid / per_ct;
  const size_t r = gid - ct * per_ct;       // (b * L + i) * n + c
  const int i = (int)((r / n) % L);
  const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
  const double xv = (double)x[gid];
  const double yv = (double)y[y_bcast ? r : gid];
  const size_t bi = r / n;                  // b * L + i
  const int b = (int)(bi / L);
  const int c = (int)(r - bi * n);
  ext[((ct * 2 + b) * (size_t)(2 * L + 1) + i) * n + c] = reduce_bal(xv - yv, p, pinv);
}

// out = [a + sum_{j < k} b[j * stride]]_q per residue (BFV addition of
// canonical residues; each partial sum is kept in [0, q) by one
// conditional subtraction, so any k is exact).
__global__ void __launch_bounds__(256) k_sum_i64(int n, int L, size_t total, const int64_t* a,
                                                 const int64_t* b, size_t stride, int k,
                                                 int64_t* out, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int i = (int)((gid / n) % L);
  const int64_t q = (int64_t)cld(tb.p, i);
  int64_t s = a[gid];
  for (int j = 0; j < k; ++j) {
    s += b[(size_t)j * stride + gid];
    s = s >= q ? s - q : s;
  }
  out[gid] = s;
}

// Batched waves: the ciphertexts of a wave are named by a device table of
// per-ciphertext pointers, [wave][stride] entries, and the wave by a device
// counter, so one captured graph serves every wave of the same size.
__global__ void __launch_bounds__(256) k_gather_sub(int n, int L, int cnt, int stride,
                                                    const CtPtrs* table, const int* wave,
                                                    double* ext, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per_ct = (size_t)2 * L * n;
  if (gid >= (size_t)cnt * per_ct) return;
  const size_t ct = gid / per_ct;
  const size_t r = gid - ct * per_ct;       // (b * L + i) * n + c
  const CtPtrs e = table[(size_t)(*wave) * stride + ct];
  const int i = (int)((r / n) % L);
  const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
  const double xv = (double)e.x[r];
  const double yv = (double)e.y[r];
  const size_t bi = r / n;
  const int b = (int)(bi / L);
  const int c = (int)(r - bi * n);
  ext[((ct * 2 + b) * (size_t)(2 * L + 1) + i) * n + c] = reduce_bal(xv - yv, p, pinv);
}

// out = ([-z0 + Delta e_0]_q, [-z1]_q) of the wave's ciphertexts in ext.
__global__ void __launch_bounds__(256) k_scatter_mask(int n, int L, int cnt, int stride,
                                                      const CtPtrs* table, const int* wave,
                                                      const double* ext, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per_ct = (size_t)2 * L * n;
  if (gid >= (size_t)cnt * per_ct) return;
  const size_t ct = gid / per_ct;
  const size_t r = gid - ct * per_ct;
  const CtPtrs e = table[(size_t)(*wave) * stride + ct];
  const size_t bi = r / n;
  const int b = (int)(bi / L);
  const int i = (int)(bi - (size_t)b * L);
  const int c = (int)(r - bi * n);
  const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
  double v = -ext[((ct * 2 + b) * (size_t)(2 * L + 1) + i) * n + c];
  if (b == 0 && c == 0) v = reduce_bal(v + cld(tb.delta_q, i), p, pinv);
  e.out[r] = to_i64(v, p);
}

__global__ void k_fill_table(TableChunk ch, CtPtrs* table) {
  const int i = threadIdx.x;
  if (i < ch.n) table[ch.first + i] = ch.e[i];
}

__global__ void k_set_counter(int* counter, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = v;
}

__global__ void k_bump_counter(int* counter, int step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += step;
}

__global__ void __launch_bounds__(256) k_sub_i64(int n, int L, size_t total, const int64_t* x,
                                                 const int64_t* y, int64_t* out, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int i = (int)((gid / n) % L);
  const double p = cld(tb.p, i);
  double z = (double)x[gid] - (double)y[gid];
  out[gid] = (int64_t)(z < 0.0 ? z + p : z);
}

// int64 [n_ct][npoly][L][N] canonical -> balanced doubles at
// out + ct * ct_stride + poly * poly_stride + i * N.
__global__ void __launch_bounds__(256) k_i64_to_polys(int n, int L, int npoly, size_t total,
                                                      const int64_t* in, double* out,
                                                      size_t ct_stride, size_t poly_stride,
                                                      int canon_from, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t row = gid / n;               // (ct * npoly + poly) * L + i
  const int c = (int)(gid - row * n);
  const int i = (int)(row % L);
  const size_t cp = row / L;
  const size_t ct = cp / npoly;
  const int poly = (int)(cp - ct * npoly);
  // polys from canon_from on keep the canonical residue (digit sources)
  out[ct * ct_stride + poly * poly_stride + (size_t)i * n + c] =
      poly >= canon_from ? (double)in[gid] : from_u64(in[gid], cld(tb.p, i));
}

// balanced doubles -> canonical int64 [n_ct][npoly][L][N].  With
// negate_delta, outputs [-x]_q plus [Delta]_q at coefficient 0 of poly 0.
__global__ void __launch_bounds__(256) k_polys_to_i64(int n, int L, int npoly, size_t total,
                                                      const double* in, size_t ct_stride,
                                                      size_t poly_stride, int64_t* out,
                                                      int negate_delta, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t row = gid / n;
  const int c = (int)(gid - row * n);
  const int i = (int)(row % L);
  const size_t cp = row / L;
  const size_t ct = cp / npoly;
  const int poly = (int)(cp - ct * npoly);
  const double p = cld(tb.p, i), pinv = cld(tb.pinv, i);
  double v = in[ct * ct_stride + poly * poly_stride + (size_t)i * n + c];
  if (negate_delta) {
    v = -v;
    if (poly == 0 && c == 0) v = reduce_bal(v + cld(tb.delta_q, i), p, pinv);
  }
  out[gid] = to_i64(v, p);
}

// rows of int64 residues -> balanced doubles; row r uses prime
// row_prime[r % nprime_rows].
__global__ void __launch_bounds__(256) k_i64_rows(size_t total, int n, const int64_t* in,
                                                  double* out, const int* row_prime,
                                                  int nprime_rows, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const size_t row = gid / n;
  const int prime = row_prime[row % nprime_rows];
  out[gid] = from_u64(in[gid], cld(tb.p, prime));
}

__device__ __forceinline__ int brv(int x, int bits) {
  return (int)(__builtin_bitreverse32((unsigned)x) >> (32 - bits));
}

// NTT-domain rows between the internal order and natural evaluation order:
// natural j holds a(psi^(2j+1)), i.e. standard position brv(j), stored at
// internal position (i mod E) * T + i / E.
__global__ void __launch_bounds__(256) k_ntt_order(size_t total, int log2n, int loge,
                                                   const double* in, int64_t* out,
                                                   const int* row_prime, int nprime_rows,
                                                   Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int n = 1 << log2n;
  const size_t row = gid / n;
  const int j = (int)(gid - row * n);
  const int prime = row_prime[row % nprime_rows];
  const int i = brv(j, log2n);
  const int E = 1 << loge;
  const int T = n >> loge;
  const int pos = (i & (E - 1)) * T + (i >> loge);
  out[gid] = to_i64(in[row * (size_t)n + pos], cld(tb.p, prime));
}

// p[0..words) = v (a fill kernel rather than hipMemsetAsync, so that calls
// a caller captures into a graph record no memset node).
__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* p, size_t words, uint64_t v) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < words) p[gid] = v;
}

// Input check of the debug switch: *bad = 1 if a residue of the int64
// polynomials [n_poly][L][N] lies outside [0, q_i).
__global__ void __launch_bounds__(256) k_check_residues(int n, int L, size_t total,
                                                        const int64_t* in, Tables tb) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int i = (int)((gid / (size_t)n) % (size_t)L);
  const int64_t v = in[gid];
  if (v < 0 || v >= (int64_t)tb.p[i]) atomicOr(tb.bad_input, 1);
}

// ---------------------------------------------------------------- host ---

// grid of the per-poly block mapping (see poly_block)
static inline dim3 poly_grid(size_t n_poly, int n, int block) {
  return dim3((unsigned)(n_poly * (size_t)((n + block - 1) / block)));
}

static inline dim3 grid_for(size_t total, int block = 256) {
  return dim3((unsigned)((total + block - 1) / block));
}

#define NSHE_L_CASES(X) X(2) X(3) X(4) X(8) X(12) X(15) X(16) X(17) X(20) X(24)
// data-prime counts built for two and three primes per key-switching digit
#define NSHE_L2_CASES(X) X(2) X(4) X(8) X(16)
#define NSHE_L3_CASES(X) X(3) X(12) X(15)

hipError_t run_lift(const Dims& d, double* ext, const Tables& tb, hipStream_t st) {
  const size_t np = (size_t)d.n_ct * 2;
  switch (d.L) {
#define C_(L_) \
  case L_: hipLaunchKernelGGL(k_lift<L_>, poly_grid(np, d.n, d.block), dim3(d.block), 0, st, d.n, np, ext, tb); break;
    NSHE_L_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_moddown_finish(const Dims& d, const double* acc, const double* dt, int64_t* out,
                              const Tables& tb, hipStream_t st, int finish) {
  if (!d.fused) return hipErrorInvalidValue;
  const size_t total = (size_t)d.n_ct * 2 * (d.n / 2);
#define C_(L_, A_)                                                                             \
  case L_:                                                                                     \
    hipLaunchKernelGGL((k_moddown_finish<L_, A_>), grid_for(total, d.block), dim3(d.block), 0, \
                       st, d.n, d.n_ct, acc, dt, out, finish, tb, d.tab);                      \
    break;
#define C1_(L_) C_(L_, 1)
#define C2_(L_) C_(L_, 2)
#define C3_(L_) C_(L_, 3)
  if (d.alpha == 1) {
    switch (d.L) {
      NSHE_L_CASES(C1_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 2) {
    switch (d.L) {
      NSHE_L2_CASES(C2_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 3) {
    switch (d.L) {
      NSHE_L3_CASES(C3_)
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef C1_
#undef C2_
#undef C3_
#undef C_
  return hipGetLastError();
}

hipError_t run_i64_lift(const Dims& d, const int64_t* in, double* ext, const Tables& tb,
                        hipStream_t st) {
  const size_t np = (size_t)d.n_ct * 2;
  switch (d.L) {
#define C_(L_)                                                                            \
  case L_:                                                                                \
    hipLaunchKernelGGL(k_i64_lift<L_>, poly_grid(np, d.n, d.block), dim3(d.block), 0, st, \
                       d.n, np, in, ext, tb);                                             \
    break;
    NSHE_L_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_sub_lift(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                        double* ext, const Tables& tb, hipStream_t st) {
  const size_t np = (size_t)d.n_ct * 2;
  switch (d.L) {
#define C_(L_)                                                                            \
  case L_:                                                                                \
    hipLaunchKernelGGL(k_sub_lift<L_>, poly_grid(np, d.n, d.block), dim3(d.block), 0, st, \
                       d.n, np, x, y, y_bcast, ext, tb, d.tab);                           \
    break;
    NSHE_L_CASES(C_)
#undef C_
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_moddown_lift(const Dims& d, const double* acc, const double* dt, double* ext,
                            const Tables& tb, hipStream_t st) {
  if (!d.fused) return hipErrorInvalidValue;
  const size_t np = (size_t)d.n_ct * 2;
#define C_(L_, A_)                                                                           \
  case L_:                                                                                   \
    hipLaunchKernelGGL((k_moddown_lift<L_, A_>), poly_grid(np, d.n, d.block), dim3(d.block), \
                       0, st, d.n, np, acc, dt, ext, tb);                                    \
    break;
#define C1_(L_) C_(L_, 1)
#define C2_(L_) C_(L_, 2)
#define C3_(L_) C_(L_, 3)
  if (d.alpha == 1) {
    switch (d.L) {
      NSHE_L_CASES(C1_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 2) {
    switch (d.L) {
      NSHE_L2_CASES(C2_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 3) {
    switch (d.L) {
      NSHE_L3_CASES(C3_)
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef C1_
#undef C2_
#undef C3_
#undef C_
  return hipGetLastError();
}


hipError_t run_scale(const Dims& d, double* dt, const Tables& tb, hipStream_t st,
                     int digit_pairs, double* src) {
  const size_t np = (size_t)d.n_ct * 3;
  Tables t = tb;
  t.dig_src = src;
  // the split-inverse variant's barrier needs whole blocks (see k_scale)
  if (d.fused && d.n % d.block) return hipErrorInvalidValue;
#define C_(L_, A_) \
  case L_:                                                                                     \
    if (d.fused)                                                                               \
      hipLaunchKernelGGL((k_scale<L_, true, A_>), poly_grid(np, d.n, d.block), dim3(d.block),  \
                         (size_t)(L_ + 1) * d.block * 8, st, d.n, np, dt, t);          \
    else                                                                                       \
      hipLaunchKernelGGL((k_scale<L_, false, A_>), poly_grid(np, d.n, d.block), dim3(d.block), \
                         (size_t)(L_ + 1) * d.block * 8, st, d.n, np, dt, t);          \
    break;
#define C1_(L_) C_(L_, 1)
#define C2_(L_) C_(L_, 2)
#define C3_(L_) C_(L_, 3)
  if (!digit_pairs) {
    switch (d.L) {
      NSHE_L_CASES(C1_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 2) {
    switch (d.L) {
      NSHE_L2_CASES(C2_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 3) {
    switch (d.L) {
      NSHE_L3_CASES(C3_)
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef C1_
#undef C2_
#undef C3_
#undef C_
  return hipGetLastError();
}

hipError_t run_ks_mac(const Dims& d, const double* dig, const double* evk, double* acc,
                      const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)(d.L + d.alpha) * d.n;
  // a chunk wider than the ciphertexts present would only repeat its
  // (clamped) loads and products: halve it down to them
  int ch = d.ks_chunk;
  while (ch > 4 && ch / 2 >= d.n_ct) ch /= 2;
  if (d.parity) {
    // four sums per ciphertext of a chunk: at most 16 ciphertexts
    if (d.n != (1 << 15)) return hipErrorInvalidValue;
    const size_t tp = (size_t)(d.L + d.alpha) * (d.n / 2);
    if (ch > 16) ch = 16;
#define P_(L_, A_) \
  case L_:                                                                                     \
    if (ch == 4)                                                                               \
      hipLaunchKernelGGL((k_ks_mac_par<L_, A_, 4>), grid_for(tp), dim3(256), 0, st, d.n_ct, dig, evk, acc, tb); \
    else if (ch == 8)                                                                          \
      hipLaunchKernelGGL((k_ks_mac_par<L_, A_, 8>), grid_for(tp), dim3(256), 0, st, d.n_ct, dig, evk, acc, tb); \
    else                                                                                       \
      hipLaunchKernelGGL((k_ks_mac_par<L_, A_, 16>), grid_for(tp), dim3(256), 0, st, d.n_ct, dig, evk, acc, tb); \
    break;
#define P1_(L_) P_(L_, 1)
#define P2_(L_) P_(L_, 2)
#define P3_(L_) P_(L_, 3)
    if (d.alpha == 1) {
      switch (d.L) {
        NSHE_L_CASES(P1_)
        default: return hipErrorInvalidValue;
      }
    } else if (d.alpha == 2) {
      switch (d.L) {
        NSHE_L2_CASES(P2_)
        default: return hipErrorInvalidValue;
      }
    } else if (d.alpha == 3) {
      switch (d.L) {
        NSHE_L3_CASES(P3_)
        default: return hipErrorInvalidValue;
      }
    } else {
      return hipErrorInvalidValue;
    }
#undef P1_
#undef P2_
#undef P3_
#undef P_
    return hipGetLastError();
  }
#define C_(L_, A_) \
  case L_:                                                                                     \
    if (ch == 4)                                                                               \
      hipLaunchKernelGGL((k_ks_mac<L_, A_, 4>), grid_for(total), dim3(256), 0, st, d.n, d.n_ct, dig, evk, acc, tb); \
    else if (ch == 8)                                                                          \
      hipLaunchKernelGGL((k_ks_mac<L_, A_, 8>), grid_for(total), dim3(256), 0, st, d.n, d.n_ct, dig, evk, acc, tb); \
    else if (ch == 32)                                                                         \
      hipLaunchKernelGGL((k_ks_mac<L_, A_, 32>), grid_for(total), dim3(256), 0, st, d.n, d.n_ct, dig, evk, acc, tb); \
    else                                                                                       \
      hipLaunchKernelGGL((k_ks_mac<L_, A_, 16>), grid_for(total), dim3(256), 0, st, d.n, d.n_ct, dig, evk, acc, tb); \
    break;
#define C1_(L_) C_(L_, 1)
#define C2_(L_) C_(L_, 2)
#define C3_(L_) C_(L_, 3)
  if (d.alpha == 1) {
    switch (d.L) {
      NSHE_L_CASES(C1_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 2) {
    switch (d.L) {
      NSHE_L2_CASES(C2_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 3) {
    switch (d.L) {
      NSHE_L3_CASES(C3_)
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef C1_
#undef C2_
#undef C3_
#undef C_
  return hipGetLastError();
}

hipError_t run_moddown(const Dims& d, const double* acc, const double* dt, double* ext,
                       const Tables& tb, hipStream_t st, int accumulate) {
  const size_t total = (size_t)d.n_ct * 2 * (d.fused ? d.n / 2 : d.n);
#define C_(L_, A_)                                                                              \
  case L_:                                                                                      \
    if (d.fused)                                                                                \
      hipLaunchKernelGGL((k_moddown<L_, A_, true>), grid_for(total, d.block), dim3(d.block), 0, \
                         st, d.n, d.n_ct, acc, dt, ext, accumulate, tb);                        \
    else                                                                                        \
      hipLaunchKernelGGL((k_moddown<L_, A_, false>), grid_for(total, d.block), dim3(d.block),   \
                         0, st, d.n, d.n_ct, acc, dt, ext, accumulate, tb);                     \
    break;
#define C1_(L_) C_(L_, 1)
#define C2_(L_) C_(L_, 2)
#define C3_(L_) C_(L_, 3)
  if (d.alpha == 1) {
    switch (d.L) {
      NSHE_L_CASES(C1_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 2) {
    switch (d.L) {
      NSHE_L2_CASES(C2_)
      default: return hipErrorInvalidValue;
    }
  } else if (d.alpha == 3) {
    switch (d.L) {
      NSHE_L3_CASES(C3_)
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef C1_
#undef C2_
#undef C3_
#undef C_
  return hipGetLastError();
}

hipError_t run_digit_mrc(const Dims& d, double* src, size_t src_stride, const Tables& tb,
                         hipStream_t st) {
  if (d.alpha < 2 || d.alpha > 3 || d.L % d.alpha) return hipErrorInvalidValue;
  const size_t total = (size_t)d.n_ct * (d.L / d.alpha) * d.n;
  if (d.alpha == 2)
    hipLaunchKernelGGL(k_digit_mrc<2>, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, src,
                       src_stride, tb);
  else
    hipLaunchKernelGGL(k_digit_mrc<3>, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, src,
                       src_stride, tb);
  return hipGetLastError();
}

hipError_t run_digit_split(const Dims& d, const double* dt, double* src, size_t src_stride,
                           hipStream_t st) {
  const size_t total = (size_t)d.n_ct * d.L * d.n;
  hipLaunchKernelGGL(k_digit_split, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, dt, src,
                     src_stride);
  return hipGetLastError();
}

hipError_t run_sub_to_ext(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                          double* ext, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_sub_to_ext, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, x, y,
                     y_bcast, ext, tb);
  return hipGetLastError();
}

hipError_t run_basis_plain(int n, uint64_t t, uint64_t zinv, uint64_t ninv_t, int64_t* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_basis_plain, grid_for(n), dim3(256), 0, st, n, t, zinv, ninv_t, out);
  return hipGetLastError();
}

hipError_t run_plain_limbs(const Dims& d, int64_t t, const int64_t* pt, double* out,
                           const Tables& tb, hipStream_t st) {
  hipLaunchKernelGGL(k_plain_limbs, grid_for((size_t)d.L * d.n), dim3(256), 0, st, d.n, d.L, t, pt,
                     out, tb);
  return hipGetLastError();
}

hipError_t run_pointwise_plain(const Dims& d, double* fx, const double* pt, const Tables& tb,
                               hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_pointwise_plain, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, fx, pt,
                     tb);
  return hipGetLastError();
}

hipError_t run_tensor_mac(const Dims& d, const double* fa, const double* fb, double* acc,
                          int first, const Tables& tb, hipStream_t st) {
  const int W = 2 * d.L + 1;
  const size_t total = (size_t)d.n_ct * W * d.n;
  hipLaunchKernelGGL(k_tensor_mac, grid_for(total), dim3(256), 0, st, d.n, W, total, fa, fb, acc,
                     first, tb);
  return hipGetLastError();
}

hipError_t run_lincomb(const Dims& d, int k, const BabyPtrs& b, const double* coef, int J,
                       int64_t* out, size_t out_stride, const Tables& tb, hipStream_t st) {
  const size_t per = (size_t)d.n_ct * 2 * d.L * d.n;
  if (k < 1 || k > BabyPtrs::CAP || J < 1 || J > 16 || (J > 1 && out_stride < per))
    return hipErrorInvalidValue;
  if (J == 16)
    hipLaunchKernelGGL(k_lincomb<16>, grid_for(per), dim3(256), 0, st, d.n, d.L, per, k, b, coef,
                       J, out, out_stride, tb);
  else if (J == 1)
    hipLaunchKernelGGL(k_lincomb<1>, grid_for(per), dim3(256), 0, st, d.n, d.L, per, k, b, coef,
                       J, out, out_stride, tb);
  else
    hipLaunchKernelGGL(k_lincomb<0>, grid_for(per), dim3(256), 0, st, d.n, d.L, per, k, b, coef,
                       J, out, out_stride, tb);
  return hipGetLastError();
}

hipError_t run_fill_one(const Dims& d, int64_t* out, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_fill_one, grid_for(total), dim3(256), 0, st, d.n, d.L, total, out, tb);
  return hipGetLastError();
}

hipError_t run_diff_i64(const Dims& d, const int64_t* x, const int64_t* y, int y_bcast,
                        int negate, int64_t* out, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_diff_i64, grid_for(total), dim3(256), 0, st, d.n, d.L, total, x, y,
                     y_bcast, negate, out, tb);
  return hipGetLastError();
}

hipError_t run_automorph(const Dims& d, unsigned ginv, const double* ext, double* dt,
                         const Tables& tb, hipStream_t st, double* src, size_t src_stride,
                         int src_split) {
  if (src_split && !src) return hipErrorInvalidValue;
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_automorph, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, ginv, ext,
                     dt, tb, src, src_stride, src_split);
  return hipGetLastError();
}

hipError_t run_sum_i64(const Dims& d, const int64_t* a, const int64_t* b, size_t stride, int k,
                       int64_t* out, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_sum_i64, grid_for(total), dim3(256), 0, st, d.n, d.L, total, a, b, stride,
                     k, out, tb);
  return hipGetLastError();
}

hipError_t run_gather_sub(const Dims& d, int stride, const CtPtrs* table, const int* wave,
                          double* ext, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_gather_sub, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, stride,
                     table, wave, ext, tb);
  return hipGetLastError();
}

hipError_t run_scatter_mask(const Dims& d, int stride, const CtPtrs* table, const int* wave,
                            const double* ext, const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_scatter_mask, grid_for(total), dim3(256), 0, st, d.n, d.L, d.n_ct, stride,
                     table, wave, ext, tb);
  return hipGetLastError();
}

hipError_t run_fill_table(const TableChunk& ch, CtPtrs* table, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_table, dim3(1), dim3(TableChunk::CAP), 0, st, ch, table);
  return hipGetLastError();
}

hipError_t run_set_counter(int* counter, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, st, counter, v);
  return hipGetLastError();
}

hipError_t run_bump_counter(int* counter, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_bump_counter, dim3(1), dim3(64), 0, st, counter, step);
  return hipGetLastError();
}

hipError_t run_sub_i64(const Dims& d, const int64_t* x, const int64_t* y, int64_t* out,
                       const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * 2 * d.L * d.n;
  hipLaunchKernelGGL(k_sub_i64, grid_for(total), dim3(256), 0, st, d.n, d.L, total, x, y, out, tb);
  return hipGetLastError();
}

hipError_t run_i64_to_polys(const Dims& d, const int64_t* in, int npoly_in, double* out,
                            size_t out_ct_stride, size_t out_poly_stride, int canon_from,
                            const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * npoly_in * d.L * d.n;
  hipLaunchKernelGGL(k_i64_to_polys, grid_for(total), dim3(256), 0, st, d.n, d.L, npoly_in, total,
                     in, out, out_ct_stride, out_poly_stride, canon_from, tb);
  return hipGetLastError();
}

hipError_t run_polys_to_i64(const Dims& d, const double* in, int npoly, size_t in_ct_stride,
                            size_t in_poly_stride, int64_t* out, int negate_delta,
                            const Tables& tb, hipStream_t st) {
  const size_t total = (size_t)d.n_ct * npoly * d.L * d.n;
  hipLaunchKernelGGL(k_polys_to_i64, grid_for(total), dim3(256), 0, st, d.n, d.L, npoly, total,
                     in, in_ct_stride, in_poly_stride, out, negate_delta, tb);
  return hipGetLastError();
}

hipError_t run_i64_to_dbl_limbs(size_t rows, int n, const int64_t* in, double* out,
                                const int* row_prime, int nprime_rows, const Tables& tb,
                                hipStream_t st) {
  const size_t total = rows * n;
  hipLaunchKernelGGL(k_i64_rows, grid_for(total), dim3(256), 0, st, total, n, in, out, row_prime,
                     nprime_rows, tb);
  return hipGetLastError();
}

hipError_t run_fill_u64(void* p, size_t words, uint64_t v, hipStream_t st) {
  if (!words) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, grid_for(words), dim3(256), 0, st, static_cast<uint64_t*>(p),
                     words, v);
  return hipGetLastError();
}

hipError_t run_check_residues(int n, int L, size_t n_poly, const int64_t* in, const Tables& tb,
                              hipStream_t st) {
  const size_t total = n_poly * L * (size_t)n;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_check_residues, grid_for(total), dim3(256), 0, st, n, L, total, in, tb);
  return hipGetLastError();
}

hipError_t run_ntt_order(int log2n, size_t rows, const double* in, int64_t* out,
                         const int* row_prime, int nprime_rows, int to_natural,
                         const Tables& tb, hipStream_t st) {
  int loge = 0, r0 = 0;
  if (ntt_rounds(log2n, &loge, &r0) < 0 || !to_natural) return hipErrorInvalidValue;
  const size_t total = rows << log2n;
  hipLaunchKernelGGL(k_ntt_order, grid_for(total), dim3(256), 0, st, total, log2n, loge, in, out,
                     row_prime, nprime_rows, tb);
  return hipGetLastError();
}

}  // namespace nshe
