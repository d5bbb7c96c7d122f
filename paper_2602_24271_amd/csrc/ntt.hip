// Negacyclic NTT / inverse NTT over one polynomial limb per workgroup,
// register-resident, for gfx950.
//
// Transform: the Cooley-Tukey merged-twist negacyclic NTT.  Stage s (0 ..
// LOGN-1) pairs indices differing in bit b = LOGN-1-s and multiplies by
// psi^(brv(2^s + m)) (m = index >> (b+1)), psi a primitive 2N-th root of
// unity mod p; the output at standard position i is a(psi^(2 brv(i) + 1)).
// The inverse runs the Gentleman-Sande butterflies with inverse twiddles in
// reverse stage order and scales by N^-1.
//
// Work decomposition (one workgroup = one N-point limb, T = N / E threads,
// E = 2^LOGE values per thread held in VGPRs): stages are grouped in
// rounds; within a round every thread owns the E indices that differ in
// the round's LOGE stage bits, so the round is a radix-E transform done in
// registers.  Between rounds the limb is exchanged through LDS (padded by
// one word per 32 so every access pattern is bank-conflict free); a limb
// of 2^15 doubles does not fit in 160 KB of LDS, so it is exchanged as two
// 32-bit halves.  Round 0 holds the top LOGE index bits (extra low bits
// make it several independent sub-transforms when LOGN is not a multiple
// of LOGE); the last round holds the bottom LOGE bits.
//
// HBM layout: coefficient-domain limbs are in natural order; NTT-domain
// limbs are stored in the "internal" order pos = (i mod E) * T + i / E of
// the standard position i, so both the load (round 0) and the store (last
// round) are unit-stride across threads.  Only pointwise kernels and the
// inverse transform read the NTT domain, and they do not care about order.
//
// Twiddles: per round a table [2^s_start][E] holding, for each value u of
// the index bits above the round, the E-1 twiddles the round needs in the
// order (stage k, j < 2^k) -> slot 2^k + j.  Values are balanced residues.
#include "kernels.h"

namespace nshe {

template <int LOGN>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int LOGE = LOGN >= 11 ? 5 : (LOGN >= 7 ? 4 : LOGN);
  static constexpr int E = 1 << LOGE;
  static constexpr int T = N / E;
  static constexpr int ROUNDS = (LOGN + LOGE - 1) / LOGE;
  static constexpr int R0 = LOGN - (ROUNDS - 1) * LOGE;
  // LDS words (32-bit) for one padded exchange buffer
  static constexpr bool SPLIT = N > 8192;  // 64-bit limb too large for one pass
  static constexpr int PADDED = N + (N >> 5) + 1;
  static constexpr int LDS_WORDS = SPLIT ? PADDED : 2 * PADDED;

  __host__ __device__ static constexpr int s_start(int r) {
    return r == 0 ? 0 : R0 + (r - 1) * LOGE;
  }
  // lowest index bit held in registers during round r
  __host__ __device__ static constexpr int lo(int r) {
    return r == 0 ? LOGN - LOGE : LOGN - s_start(r) - LOGE;
  }
  __host__ __device__ static constexpr int stages(int r) { return r == 0 ? R0 : LOGE; }
  // offset of round r's twiddle table (in doubles)
  __host__ __device__ static constexpr int tw_off(int r) {
    int off = 0;
    for (int i = 0; i < r; ++i) off += (1 << s_start(i)) * E;
    return off;
  }
  __host__ __device__ static constexpr int tw_len() { return tw_off(ROUNDS); }
};

__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }

template <int LOGN>
__device__ __forceinline__ int round_index(int r, int tid, int e) {
  using S = NttShape<LOGN>;
  const int lo = S::lo(r);
  return ((tid >> lo) << (lo + S::LOGE)) | (e << lo) | (tid & ((1 << lo) - 1));
}

// pad32 is additive over disjoint bit sets, so the padded LDS slot of
// (tid, e) is a per-thread base plus a compile-time offset per element.
template <int LOGN>
__device__ __forceinline__ int slot_base(int r, int tid) {
  return pad32(round_index<LOGN>(r, tid, 0));
}

template <int LOGN>
__device__ __forceinline__ constexpr int slot_off(int r, int e) {
  return (e << NttShape<LOGN>::lo(r)) + ((e << NttShape<LOGN>::lo(r)) >> 5);
}

// Move the E values of every thread from round r0's index map to r1's.
template <int LOGN>
__device__ __forceinline__ void exchange(double (&x)[NttShape<LOGN>::E], int r0, int r1,
                                         uint32_t* lds) {
  using S = NttShape<LOGN>;
  const int tid = threadIdx.x;
  const int b0 = slot_base<LOGN>(r0, tid);
  const int b1 = slot_base<LOGN>(r1, tid);
  if constexpr (S::SPLIT) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int e = 0; e < S::E; ++e) {
        unsigned long long v = __double_as_longlong(x[e]);
        lds[b0 + slot_off<LOGN>(r0, e)] = half ? (uint32_t)(v >> 32) : (uint32_t)v;
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < S::E; ++e) {
        uint32_t w = lds[b1 + slot_off<LOGN>(r1, e)];
        unsigned long long v = __double_as_longlong(x[e]);
        v = half ? ((v & 0xffffffffull) | ((unsigned long long)w << 32))
                 : ((v & 0xffffffff00000000ull) | w);
        x[e] = __longlong_as_double(v);
      }
      __syncthreads();
    }
  } else {
    double* d = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int e = 0; e < S::E; ++e) d[b0 + slot_off<LOGN>(r0, e)] = x[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = d[b1 + slot_off<LOGN>(r1, e)];
    __syncthreads();
  }
}

__device__ __forceinline__ void ct_bfly(double& X, double& Y, double W, double p, double pinv) {
  double xr = reduce_bal(X, p, pinv);
  double t = mul_lazy(Y, W, p, pinv);
  X = xr + t;
  Y = xr - t;
}

__device__ __forceinline__ void gs_bfly(double& X, double& Y, double W, double p, double pinv) {
  double s = X + Y;
  double d = X - Y;
  X = reduce_bal(s, p, pinv);
  Y = mul_lazy(d, W, p, pinv);
}

// Round r of the forward transform on this thread's registers.
template <int LOGN>
__device__ __forceinline__ void fwd_round(double (&x)[NttShape<LOGN>::E], int r,
                                          const double* __restrict__ tw, double p, double pinv) {
  using S = NttShape<LOGN>;
  const int tid = threadIdx.x;
  const int u = r == 0 ? 0 : (tid >> S::lo(r));
  const auto tr = make_rsrc(tw, S::tw_len() * 8);
  const unsigned tvo = (S::tw_off(r) + u * S::E) * 8;
  const int R = S::stages(r);
#pragma unroll
  for (int k = 0; k < S::LOGE; ++k) {
    if (k >= R) break;
    const int eb = S::LOGE - 1 - k;
    double w[1 << (S::LOGE - 1)];
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) w[j] = buf_load(tr, tvo, ((1 << k) + j) * 8);
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      if (e & (1 << eb)) continue;
      ct_bfly(x[e], x[e | (1 << eb)], w[e >> (eb + 1)], p, pinv);
    }
  }
}

template <int LOGN>
__device__ __forceinline__ void inv_round(double (&x)[NttShape<LOGN>::E], int r,
                                          const double* __restrict__ tw, double p, double pinv) {
  using S = NttShape<LOGN>;
  const int tid = threadIdx.x;
  const int u = r == 0 ? 0 : (tid >> S::lo(r));
  const auto tr = make_rsrc(tw, S::tw_len() * 8);
  const unsigned tvo = (S::tw_off(r) + u * S::E) * 8;
  const int R = S::stages(r);
#pragma unroll
  for (int kk = 0; kk < S::LOGE; ++kk) {
    const int k = S::LOGE - 1 - kk;
    if (k >= R) continue;
    const int eb = S::LOGE - 1 - k;
    double w[1 << (S::LOGE - 1)];
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) w[j] = buf_load(tr, tvo, ((1 << k) + j) * 8);
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      if (e & (1 << eb)) continue;
      gs_bfly(x[e], x[e | (1 << eb)], w[e >> (eb + 1)], p, pinv);
    }
  }
}

// Work item of an NTT launch: item = limb * npoly + poly (limb-major, so
// that items sharing a prime - and its twiddle tables - are adjacent), and
// workgroups are spread so that each XCD (workgroup id mod 8) receives one
// contiguous item range and therefore only a few primes' tables.
__device__ __forceinline__ int xcd_item(int count) {
  const int per = (count + 7) >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

template <int LOGN, int MODE>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_ntt_fwd(NttJob job, Tables tb) {
  using S = NttShape<LOGN>;
  __shared__ uint32_t lds[S::LDS_WORDS];
  const int item = xcd_item(job.count);
  if (item >= job.count) return;
  const int limb = item / job.npoly;
  const int poly = item - limb * job.npoly;
  const int prime = job.limb_prime[limb];
  const double p = tb.p[prime], pinv = tb.pinv[prime];
  const double* __restrict__ tw = tb.tw_fwd + (size_t)prime * tb.tw_len;
  double* dst = job.base + ((size_t)poly * job.poly_stride + (size_t)limb * S::N);
  const auto rd = make_rsrc(dst, S::N * 8);
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  double x[S::E];
  if constexpr (MODE == NTT_DIGIT) {
    // poly = ct * L + j; limb = target prime i.  Source: digit j of the
    // third component, balanced mod q_j; D_j = canonical value in [0, q_j).
    const int ct = poly / job.digits;
    const int j = poly - ct * job.digits;
    const double qj = tb.p[j];
    const auto rs = make_rsrc(job.src + (size_t)ct * job.src_ct_stride + (size_t)j * S::N, S::N * 8);
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      double v = buf_load(rs, vo, e * S::T * 8);
      v = v < 0.0 ? v + qj : v;
      x[e] = reduce_bal(v, p, pinv);
    }
  } else {
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = buf_load(rd, vo, e * S::T * 8);
  }
#pragma unroll
  for (int r = 0; r < S::ROUNDS; ++r) {
    if (r > 0) exchange<LOGN>(x, r - 1, r, lds);
    fwd_round<LOGN>(x, r, tw, p, pinv);
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(reduce_bal(x[e], p, pinv), rd, vo, e * S::T * 8);
}

template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_ntt_inv(NttJob job, Tables tb) {
  using S = NttShape<LOGN>;
  __shared__ uint32_t lds[S::LDS_WORDS];
  const int item = xcd_item(job.count);
  if (item >= job.count) return;
  const int limb = item / job.npoly;
  const int poly = item - limb * job.npoly;
  const int prime = job.limb_prime[limb];
  const double p = tb.p[prime], pinv = tb.pinv[prime];
  const double* __restrict__ tw = tb.tw_inv + (size_t)prime * tb.tw_len;
  double* dst = job.base + ((size_t)poly * job.poly_stride + (size_t)limb * S::N);
  const auto rd = make_rsrc(dst, S::N * 8);
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  double x[S::E];
#pragma unroll
  for (int e = 0; e < S::E; ++e) x[e] = buf_load(rd, vo, e * S::T * 8);
#pragma unroll
  for (int rr = 0; rr < S::ROUNDS; ++rr) {
    const int r = S::ROUNDS - 1 - rr;
    if (rr > 0) exchange<LOGN>(x, r + 1, r, lds);
    inv_round<LOGN>(x, r, tw, p, pinv);
  }
  const double ninv = tb.ninv[prime];
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(mul_bal(x[e], ninv, p, pinv), rd, vo, e * S::T * 8);
}

// ---------------------------------------------------------------- host ---

template <int LOGN>
static hipError_t launch_ntt(const NttJob& job, const Tables& tb, int dir, hipStream_t st) {
  using S = NttShape<LOGN>;
  const int per = (job.count + 7) >> 3;
  dim3 grid(per * 8), block(S::T);
  if (dir == 0)
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_INPLACE>), grid, block, 0, st, job, tb);
  else if (dir == 1)
    hipLaunchKernelGGL((k_ntt_inv<LOGN>), grid, block, 0, st, job, tb);
  else
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_DIGIT>), grid, block, 0, st, job, tb);
  return hipGetLastError();
}

hipError_t run_ntt(int log2n, const NttJob& job, const Tables& tb, int dir, hipStream_t st) {
  if (job.count <= 0) return hipSuccess;
  switch (log2n) {
    case 3: return launch_ntt<3>(job, tb, dir, st);
    case 4: return launch_ntt<4>(job, tb, dir, st);
    case 5: return launch_ntt<5>(job, tb, dir, st);
    case 6: return launch_ntt<6>(job, tb, dir, st);
    case 7: return launch_ntt<7>(job, tb, dir, st);
    case 8: return launch_ntt<8>(job, tb, dir, st);
    case 9: return launch_ntt<9>(job, tb, dir, st);
    case 10: return launch_ntt<10>(job, tb, dir, st);
    case 11: return launch_ntt<11>(job, tb, dir, st);
    case 12: return launch_ntt<12>(job, tb, dir, st);
    case 13: return launch_ntt<13>(job, tb, dir, st);
    case 14: return launch_ntt<14>(job, tb, dir, st);
    case 15: return launch_ntt<15>(job, tb, dir, st);
    default: return hipErrorInvalidValue;
  }
}

// Host description of the transform shape, for building twiddle tables.
int ntt_rounds(int log2n, int* loge, int* r0) {
#define NSHE_SHAPE(L_)                                  \
  case L_:                                              \
    *loge = NttShape<L_>::LOGE;                         \
    *r0 = NttShape<L_>::R0;                             \
    return NttShape<L_>::ROUNDS;
  switch (log2n) {
    NSHE_SHAPE(3) NSHE_SHAPE(4) NSHE_SHAPE(5) NSHE_SHAPE(6) NSHE_SHAPE(7)
    NSHE_SHAPE(8) NSHE_SHAPE(9) NSHE_SHAPE(10) NSHE_SHAPE(11) NSHE_SHAPE(12)
    NSHE_SHAPE(13) NSHE_SHAPE(14) NSHE_SHAPE(15)
    default: return -1;
  }
#undef NSHE_SHAPE
}

}  // namespace nshe
