// Negacyclic NTT / inverse NTT over one polynomial limb per workgroup,
// register-resident, for gfx950.
//
// Transform: the Cooley-Tukey merged-twist negacyclic NTT.  Stage s (0 ..
// LOGN-1) pairs indices differing in bit b = LOGN-1-s and multiplies by
// psi^(brv(2^s + m)) (m = index >> (b+1)), psi a primitive 2N-th root of
// unity mod p; the output at standard position i is a(psi^(2 brv(i) + 1)).
// The inverse runs the Gentleman-Sande butterflies with inverse twiddles in
// reverse stage order and returns N times the coefficients: the N^-1 factor
// is folded into the constants of every consumer of an inverse transform.
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
// Twiddles: round 0 (the top index bits) uses the same E - 1 twiddles in
// every thread, slot 2^k + j for stage k, j < 2^k; later rounds keep per
// index row only each stage's first twiddle and derive the others (see
// TwSrc).  Values are balanced residues.
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
  // offset (doubles) of round r's rows in the compact table (rounds >= 1,
  // 8 slots per row)
  __host__ __device__ static constexpr int cmp_off(int r) {
    int off = 0;
    for (int i = 1; i < r; ++i) off += (1 << s_start(i)) * 8;
    return off;
  }
  __host__ __device__ static constexpr int cmp_len() { return cmp_off(ROUNDS); }
};

__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }

__host__ __device__ constexpr int brv_c(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

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

// LDS word address of element e in round r: a per-thread base plus a
// constant.  Offsets beyond the 16-bit immediate of ds_read/ds_write are
// split off into a per-chunk base (CH elements per chunk).
template <int LOGN, int BYTES>
__device__ __forceinline__ constexpr int lds_chunk() {
  int ch = NttShape<LOGN>::E;
  for (int r = 0; r < NttShape<LOGN>::ROUNDS; ++r)
    while (ch > 1 && slot_off<LOGN>(r, ch - 1) * BYTES >= 65536) ch >>= 1;
  return ch;
}

// The thread that holds index i in round r (the inverse of round_index).
template <int LOGN>
__host__ __device__ constexpr int round_tid(int r, int i) {
  using S = NttShape<LOGN>;
  const int lo = S::lo(r);
  return ((i >> (lo + S::LOGE)) << lo) | (i & ((1 << lo) - 1));
}

// Between the last two rounds (when neither is round 0) the values move
// only among threads of one wavefront: round ROUNDS-2 holds index bits
// [LOGE, 2 LOGE) in registers and the last round bits [0, LOGE), so an
// index keeps its bits from 2 LOGE up in the thread number under both maps
// and the E threads that trade values share tid >> LOGE.
template <int LOGN>
__host__ __device__ constexpr bool wave_local(int r0, int r1) {
  using S = NttShape<LOGN>;
  const int a = r0 < r1 ? r0 : r1, b = r0 < r1 ? r1 : r0;
  return a >= 1 && b == S::ROUNDS - 1 && b - a == 1 && S::E <= 64;
}

// Every index's two holders (under the maps of a wave-local pair of
// rounds) are in the same wavefront of 64 threads.
template <int LOGN>
constexpr bool wave_local_sound() {
  using S = NttShape<LOGN>;
  for (int a = 0; a + 1 < S::ROUNDS; ++a) {
    if (!wave_local<LOGN>(a, a + 1)) continue;
    for (int i = 0; i < S::N; ++i)
      if ((round_tid<LOGN>(a, i) >> 6) != (round_tid<LOGN>(a + 1, i) >> 6)) return false;
  }
  return true;
}
static_assert(wave_local_sound<15>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<14>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<13>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<12>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<11>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<10>(), "wave-local exchanges stay inside a wavefront");
static_assert(wave_local_sound<9>(), "wave-local exchanges stay inside a wavefront");

// Order one pass's LDS writes before its reads (and the reads before the
// next pass's writes): a workgroup barrier, or for a wave-local exchange
// only a wavefront-scope fence, since one wavefront's LDS operations are
// carried out in issue order.
__device__ __forceinline__ void lds_pass_sync(bool wave_only) {
  if (wave_only) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS byte address of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const uint32_t* p) {
  return (uint32_t)(size_t)(const __attribute__((address_space(3))) uint32_t*)p;
}

// 32 LDS words at a + k STRIDE (bytes), k = 0..31, each into its own
// register, issued and waited for inside one asm block (no read is in
// flight past it).  Written out because the compiler pairs such reads
// (ds_read2) into adjacent registers, which in an exchange are halves of
// different doubles and then cost a register move each.
template <int STRIDE>
__device__ __forceinline__ void lds_read32(uint32_t (&w)[32], uint32_t a) {
  static_assert(STRIDE > 0 && 31 * STRIDE < 65536, "offsets fit the 16-bit immediate");
  asm volatile(
      "ds_read_b32 %0, %32 offset:%c33*0\n\t"
      "ds_read_b32 %1, %32 offset:%c33*1\n\t"
      "ds_read_b32 %2, %32 offset:%c33*2\n\t"
      "ds_read_b32 %3, %32 offset:%c33*3\n\t"
      "ds_read_b32 %4, %32 offset:%c33*4\n\t"
      "ds_read_b32 %5, %32 offset:%c33*5\n\t"
      "ds_read_b32 %6, %32 offset:%c33*6\n\t"
      "ds_read_b32 %7, %32 offset:%c33*7\n\t"
      "ds_read_b32 %8, %32 offset:%c33*8\n\t"
      "ds_read_b32 %9, %32 offset:%c33*9\n\t"
      "ds_read_b32 %10, %32 offset:%c33*10\n\t"
      "ds_read_b32 %11, %32 offset:%c33*11\n\t"
      "ds_read_b32 %12, %32 offset:%c33*12\n\t"
      "ds_read_b32 %13, %32 offset:%c33*13\n\t"
      "ds_read_b32 %14, %32 offset:%c33*14\n\t"
      "ds_read_b32 %15, %32 offset:%c33*15\n\t"
      "ds_read_b32 %16, %32 offset:%c33*16\n\t"
      "ds_read_b32 %17, %32 offset:%c33*17\n\t"
      "ds_read_b32 %18, %32 offset:%c33*18\n\t"
      "ds_read_b32 %19, %32 offset:%c33*19\n\t"
      "ds_read_b32 %20, %32 offset:%c33*20\n\t"
      "ds_read_b32 %21, %32 offset:%c33*21\n\t"
      "ds_read_b32 %22, %32 offset:%c33*22\n\t"
      "ds_read_b32 %23, %32 offset:%c33*23\n\t"
      "ds_read_b32 %24, %32 offset:%c33*24\n\t"
      "ds_read_b32 %25, %32 offset:%c33*25\n\t"
      "ds_read_b32 %26, %32 offset:%c33*26\n\t"
      "ds_read_b32 %27, %32 offset:%c33*27\n\t"
      "ds_read_b32 %28, %32 offset:%c33*28\n\t"
      "ds_read_b32 %29, %32 offset:%c33*29\n\t"
      "ds_read_b32 %30, %32 offset:%c33*30\n\t"
      "ds_read_b32 %31, %32 offset:%c33*31\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5]), "=&v"(w[6]), "=&v"(w[7]),
        "=&v"(w[8]), "=&v"(w[9]), "=&v"(w[10]), "=&v"(w[11]), "=&v"(w[12]), "=&v"(w[13]), "=&v"(w[14]), "=&v"(w[15]),
        "=&v"(w[16]), "=&v"(w[17]), "=&v"(w[18]), "=&v"(w[19]), "=&v"(w[20]), "=&v"(w[21]), "=&v"(w[22]), "=&v"(w[23]),
        "=&v"(w[24]), "=&v"(w[25]), "=&v"(w[26]), "=&v"(w[27]), "=&v"(w[28]), "=&v"(w[29]), "=&v"(w[30]), "=&v"(w[31])
      : "v"(a), "i"(STRIDE)
      : "memory");
}

// Round R's slot offsets are e times that of element 1 (true when the
// round's lowest register bit is 0 or at least 5).
template <int LOGN, int R>
constexpr bool linear_slots() {
  for (int e = 0; e < NttShape<LOGN>::E; ++e)
    if (slot_off<LOGN>(R, e) != e * slot_off<LOGN>(R, 1)) return false;
  return true;
}

// One pass's words of round R's 32 elements into their halves of x.
template <int LOGN, int R>
__device__ __forceinline__ void take_words(double (&x)[NttShape<LOGN>::E], uint32_t a, int half) {
  static_assert(NttShape<LOGN>::E == 32 && linear_slots<LOGN, R>(), "32 evenly spaced slots");
  uint32_t w[32];
  lds_read32<slot_off<LOGN>(R, 1) * 4>(w, a);
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    unsigned long long v = __double_as_longlong(x[e]);
    v = half ? ((v & 0xffffffffull) | ((unsigned long long)w[e] << 32))
             : ((v & 0xffffffff00000000ull) | w[e]);
    x[e] = __longlong_as_double(v);
  }
}

// Exchanges of this size read their words with lds_read32.
template <int LOGN>
constexpr bool word_reads() {
  using S = NttShape<LOGN>;
  if constexpr (S::E != 32 || S::ROUNDS != 3 || !S::SPLIT) return false;
  else return linear_slots<LOGN, 0>() && linear_slots<LOGN, 1>() && linear_slots<LOGN, 2>() &&
              31 * slot_off<LOGN>(0, 1) * 4 < 65536;
}

// Move the E values of every thread from round r0's index map to r1's.
// The base addresses are made opaque per pass (inline asm), so that no
// per-element address registers stay live across the barriers.  Each pass
// is write, barrier, read; a barrier separates a pass's reads from the next
// pass's writes.  After the last read there is none: the next exchange
// starts with it instead (wait_prev), so that a wave starts the round's
// arithmetic as soon as its own values have arrived.  A wave-local
// exchange (see wave_local) orders its passes within the wavefront only;
// it still needs wait_prev when the previous exchange was not wave-local,
// as other wavefronts may be reading its slots.  WORDS: read each pass's
// words one per register (lds_read32) where the size allows; measured
// faster only for the tensor inverse (the other transforms keep the
// compiler's paired reads).
template <int LOGN, bool WORDS = false>
__device__ __forceinline__ void exchange(double (&x)[NttShape<LOGN>::E], int r0, int r1,
                                         uint32_t* lds, bool wait_prev) {
  using S = NttShape<LOGN>;
  const int tid = threadIdx.x;
  const bool local = wave_local<LOGN>(r0, r1);
  if (wait_prev) __syncthreads();
  if constexpr (S::SPLIT) {
    constexpr int C0 = lds_chunk<LOGN, 4>();
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      int b0 = slot_base<LOGN>(r0, tid);
      asm volatile("" : "+v"(b0));
#pragma unroll
      for (int c = 0; c < S::E; c += C0) {
        uint32_t* base = lds + b0 + slot_off<LOGN>(r0, c);
#pragma unroll
        for (int e = c; e < c + C0; ++e) {
          unsigned long long v = __double_as_longlong(x[e]);
          base[slot_off<LOGN>(r0, e) - slot_off<LOGN>(r0, c)] =
              half ? (uint32_t)(v >> 32) : (uint32_t)v;
        }
      }
      lds_pass_sync(local);
      int b1 = slot_base<LOGN>(r1, tid);
      asm volatile("" : "+v"(b1));
      if constexpr (WORDS && word_reads<LOGN>()) {
        const uint32_t a = lds_addr(lds + b1);
        if (r1 == 0)
          take_words<LOGN, 0>(x, a, half);
        else if (r1 == 1)
          take_words<LOGN, 1>(x, a, half);
        else
          take_words<LOGN, 2>(x, a, half);
        if (half == 0) lds_pass_sync(local);
        continue;
      }
#pragma unroll
      for (int c = 0; c < S::E; c += C0) {
        const uint32_t* base = lds + b1 + slot_off<LOGN>(r1, c);
#pragma unroll
        for (int e = c; e < c + C0; ++e) {
          const uint32_t w = base[slot_off<LOGN>(r1, e) - slot_off<LOGN>(r1, c)];
          unsigned long long v = __double_as_longlong(x[e]);
          v = half ? ((v & 0xffffffffull) | ((unsigned long long)w << 32))
                   : ((v & 0xffffffff00000000ull) | w);
          x[e] = __longlong_as_double(v);
        }
      }
      if (half == 0) lds_pass_sync(local);
    }
  } else {
    double* d = reinterpret_cast<double*>(lds);
    constexpr int C0 = lds_chunk<LOGN, 8>();
    int b0 = slot_base<LOGN>(r0, tid);
    asm volatile("" : "+v"(b0));
#pragma unroll
    for (int c = 0; c < S::E; c += C0) {
      double* base = d + b0 + slot_off<LOGN>(r0, c);
#pragma unroll
      for (int e = c; e < c + C0; ++e)
        base[slot_off<LOGN>(r0, e) - slot_off<LOGN>(r0, c)] = x[e];
    }
    lds_pass_sync(local);
    int b1 = slot_base<LOGN>(r1, tid);
    asm volatile("" : "+v"(b1));
#pragma unroll
    for (int c = 0; c < S::E; c += C0) {
      const double* base = d + b1 + slot_off<LOGN>(r1, c);
#pragma unroll
      for (int e = c; e < c + C0; ++e) x[e] = base[slot_off<LOGN>(r1, e) - slot_off<LOGN>(r1, c)];
    }
  }
}

// Cooley-Tukey butterfly without reducing X.  With |W| <= 0.55 p (a
// balanced table twiddle, or one derived by a lazy product) and p < 2^49
// the product T = [Y W] has |T| <= (1/2 + d) p, where the quotient error
// d <= |Y W / p| 3 2^-53 <= 0.103 |Y| / p, so a stage maps a bound b p on
// the inputs to (1.103 b + 0.5) p.  From inputs below 2p (a canonical
// digit of another prime of the chain) ten stages stay below 13.5 p, so
// every intermediate is an integer below 2^53 and every product is exact
// (its quotient below 2^53, h - q p and the final sum exactly
// representable).  A reduction every ten stages therefore suffices; see
// fwd_reduces_after.  Five stages from a reduced input end below 3.9 p.
__device__ __forceinline__ void ct_bfly(double& X, double& Y, double W, double p, double pinv) {
  double t = mul_lazy(Y, W, p, pinv);
  double x = X;
  X = x + t;
  Y = x - t;
}

// Gentleman-Sande butterfly; the sum is reduced on every third stage only
// (REDUCE_SUM, gs_reduces), the difference feeds the modular product
// directly.  A stage maps a bound B p on its inputs to sums below 2 B p (or
// p/2 when reduced) and products of differences below (0.5 + 0.206 B) p
// (|X - Y| <= 2 B p, |W| <= 0.55 p).  From balanced inputs, stage by stage:
// 1, 2, 0.91, 1.82, 3.64, 1.25, 2.5, 5.0, 1.53, 3.06, 6.12, 1.76, 3.52, 7.04
// (fourteen stages) and 1.95 after a fifteenth: every difference entering a
// product stays below 14.1 p, inside mul_lazy's exact range (quotient below
// 2^53, remainder and correction exactly representable, for |a| < 16 p and
// p < 2^49), and every sum below 2^52.  The rule runs over the global stage
// count, whatever the round boundaries; the last round reduces every value.
__host__ __device__ constexpr bool gs_reduces(int g) { return g % 3 == 2; }

template <bool REDUCE_SUM>
__device__ __forceinline__ void gs_bfly(double& X, double& Y, double W, double p, double pinv) {
  double s = X + Y;
  double d = X - Y;
  X = REDUCE_SUM ? reduce_bal(s, p, pinv) : s;
  Y = mul_lazy(d, W, p, pinv);
}

// Largest number of forward stages between two reductions (see ct_bfly).
constexpr int FWD_STAGES_PER_REDUCTION = 10;

// Bound (in units of p) on the values after `stages` Cooley-Tukey stages
// from inputs below b p (ct_bfly: b -> 1.103 b + 0.5).  Every value must stay
// below 2^53 / p > 16.6 p (p < 2^48.95) to be an exact integer.
constexpr double ct_bound(double b, int stages) {
  for (int i = 0; i < stages; ++i) b = 1.103 * b + 0.5;
  return b;
}
// Inputs of digit transforms: a one-prime digit is below 2 p; a two-prime
// digit's value is formed on load as v_0 + [q_{2j}]_p v_1 from canonical
// mixed-radix digits below 1.93 p (all primes in [2^48, 2^48.95)), so below
// (1.93 + 0.5 + 0.094 x 1.93) p < 2.61 p.
// A three-prime digit's value v_0 + [q_g]_p v_1 + [q_g q_{g+1}]_p v_2 is below
// (1.93 + 2 x 0.68) p < 3.3 p, too large for ten stages: it is reduced to
// balanced form (below p/2) before the transform.
constexpr double DIGIT_IN = 2.0, DIGIT2_IN = 2.61;
static_assert(ct_bound(DIGIT_IN, FWD_STAGES_PER_REDUCTION) < 13.5, "one-prime digit bound");
static_assert(ct_bound(DIGIT2_IN, FWD_STAGES_PER_REDUCTION) < 15.1, "two-prime digit bound");
static_assert(15.1 < 16.6, "exact below 2^53");

// Whether the forward transform reduces at the end of round r, given
// `pre` stages done (unreduced) before round 0: at the last round, and
// whenever the next round would take the count past the limit.
template <int LOGN>
__host__ __device__ constexpr bool fwd_reduces_after(int r, int pre) {
  using S = NttShape<LOGN>;
  int since = pre;
  for (int i = 0; i < S::ROUNDS; ++i) {
    since += S::stages(i);
    const bool red = i == S::ROUNDS - 1 || since + S::stages(i + 1) > FWD_STAGES_PER_REDUCTION;
    if (i == r) return red;
    if (red) since = 0;
  }
  return true;
}

template <int LOGN>
constexpr bool fwd_schedule_ok(int pre) {
  using S = NttShape<LOGN>;
  int since = pre;
  for (int i = 0; i < S::ROUNDS; ++i) {
    since += S::stages(i);
    if (since > FWD_STAGES_PER_REDUCTION) return false;
    if (fwd_reduces_after<LOGN>(i, pre)) since = 0;
  }
  return true;
}

// Twiddle sources of a transform.  Round 0's twiddles are the same for
// every thread (slot 2^k + j of a [E] row, through the scalar cache).  In a
// later round the twiddle of stage k, slot j for index row u is
// W(k, j) = W(k, 0) omega_k^(+-brv_k(j)) (the bits of j, of u and of the
// stage are disjoint in the bit-reversed exponent): the compact table keeps
// W(k, 0) per row (8 slots, stage k at slot k, stored slot-major within a
// round; rounds r >= 1 one after the other) and cst the per-(stage, slot)
// constants shared by all rows, so a
// thread loads 5 twiddles per round instead of 31 and derives the rest
// with one modular product each.
struct TwSrc {
  const double* tw0;   // round 0 row
  const double* cmp;   // compact rows of rounds >= 1
  const double* cst;   // [32] slot 2^k + j: omega_k^(+-brv_k(j))
};

// Rounds r >= 1 (LOGE stages each) with compact twiddles.  A stage's base
// twiddle is loaded one stage ahead, fenced on the previous stage's inputs
// so that the loads are not all hoisted to the top (register pressure).
// Forward (FWD): Cooley-Tukey stages k = 0..LOGE-1.  Inverse: Gentleman-
// Sande stages k = LOGE-1..0, the sum reduced per gs_reduces (g0 =
// stages done before this round).
// reduce_x0 (forward): reduce the X operand of each first-stage butterfly
// as it is used.
template <int LOGN, bool FWD>
__device__ __forceinline__ void compact_round(double (&x)[NttShape<LOGN>::E], int r, int g0,
                                              const TwSrc& t, double p, double pinv,
                                              bool reduce_x0 = false) {
  using S = NttShape<LOGN>;
  // slot k of row u at k rows + u (slot-major: one slot's loads by a wave
  // are contiguous)
  const unsigned rows = 1u << S::s_start(r);
  const auto rl = make_rsrc(t.cmp + S::cmp_off(r), rows * 64);
  const unsigned lo = (threadIdx.x >> S::lo(r)) * 8;
  double wcur = buf_load(rl, lo, (FWD ? 0 : S::LOGE - 1) * rows * 8), wnxt = 0.0;
#pragma unroll
  for (int kk = 0; kk < S::LOGE; ++kk) {
    const int k = FWD ? kk : S::LOGE - 1 - kk;
    const int eb = S::LOGE - 1 - k;
    if (kk + 1 < S::LOGE) {
      unsigned o = lo;
      asm volatile("" : "+v"(o) : "v"(x[0]));
      wnxt = buf_load(rl, o, (FWD ? k + 1 : k - 1) * rows * 8);
    }
    const double wk = wcur;
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      // a lazy product: |w| <= 0.55 p (see ct_bfly)
      const double w = j == 0 ? wk : mul_lazy(wk, cld(t.cst, (1 << k) + j), p, pinv);
#pragma unroll
      for (int b = 0; b < (1 << eb); ++b) {
        const int e = (j << (eb + 1)) | b;
        if constexpr (FWD) {
          if (kk == 0 && reduce_x0) {
            x[e] = reduce_bal(x[e], p, pinv);
            asm volatile("" : "+v"(x[e]));   // keep it next to its butterfly
          }
          ct_bfly(x[e], x[e | (1 << eb)], w, p, pinv);
        } else {
          if (gs_reduces(g0 + kk))
            gs_bfly<true>(x[e], x[e | (1 << eb)], w, p, pinv);
          else
            gs_bfly<false>(x[e], x[e | (1 << eb)], w, p, pinv);
        }
      }
    }
    wcur = wnxt;
  }
}

// Round 1 of a half-limb transform with every twiddle read from LDS: the
// round has only 2^R0 index rows (16 for the 2^14-point halves), so a
// workgroup copies their full rows (32 slots, stage k slot 2^k + j) into
// LDS once and reads them there, shared by the 2^lo(1) threads of a row,
// instead of loading each stage's first twiddle and deriving the others
// with a modular product.
constexpr int LDS_ROW = 32;

template <int LOGN, bool FWD>
__device__ __forceinline__ void lds_round(double (&x)[NttShape<LOGN>::E], int r, int g0,
                                          const double* ltw, double p, double pinv) {
  using S = NttShape<LOGN>;
  const int row = (threadIdx.x >> S::lo(r)) * LDS_ROW;
#pragma unroll
  for (int kk = 0; kk < S::LOGE; ++kk) {
    const int k = FWD ? kk : S::LOGE - 1 - kk;
    const int eb = S::LOGE - 1 - k;
    // a stage's reads wait for the previous stage's results (registers:
    // otherwise all 31 are hoisted to the round's start)
    int rk = row;
    asm volatile("" : "+v"(rk) : "v"(x[0]));
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      const double w = ltw[rk + (1 << k) + j];
#pragma unroll
      for (int b = 0; b < (1 << eb); ++b) {
        const int e = (j << (eb + 1)) | b;
        if constexpr (FWD) {
          ct_bfly(x[e], x[e | (1 << eb)], w, p, pinv);
        } else {
          if (gs_reduces(g0 + kk))
            gs_bfly<true>(x[e], x[e | (1 << eb)], w, p, pinv);
          else
            gs_bfly<false>(x[e], x[e | (1 << eb)], w, p, pinv);
        }
      }
    }
  }
}

// Round r of the forward transform on this thread's registers (LDS1: round
// 1's twiddle rows are in LDS at ltw).
template <int LOGN, bool LDS1 = false>
__device__ __forceinline__ void fwd_round(double (&x)[NttShape<LOGN>::E], int r, bool reduce,
                                          const TwSrc& ts, double p, double pinv,
                                          const double* ltw = nullptr, bool reduce_x0 = false) {
  using S = NttShape<LOGN>;
  if (LDS1 && r == 1) {
    lds_round<LOGN, true>(x, r, 0, ltw, p, pinv);
  } else if (r > 0) {
    compact_round<LOGN, true>(x, r, 0, ts, p, pinv, reduce_x0);
  } else {
#pragma unroll
    for (int k = 0; k < S::R0; ++k) {
      const int eb = S::LOGE - 1 - k;
#pragma unroll
      for (int j = 0; j < (1 << k); ++j) {
        const double w = cld(ts.tw0, (1 << k) + j);
#pragma unroll
        for (int b = 0; b < (1 << eb); ++b) {
          const int e = (j << (eb + 1)) | b;
          ct_bfly(x[e], x[e | (1 << eb)], w, p, pinv);
        }
      }
    }
  }
  if (reduce) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = reduce_bal(x[e], p, pinv);
  }
}

// Round r of the inverse; g0 = stages done before it (the sum-reduction
// rule runs over the global stage count).  Round 0 is the last one
// processed and reduces every value at its end.
template <int LOGN, bool LDS1 = false>
__device__ __forceinline__ void inv_round(double (&x)[NttShape<LOGN>::E], int r, int g0,
                                          const TwSrc& ts, double p, double pinv,
                                          const double* ltw = nullptr) {
  using S = NttShape<LOGN>;
  if (LDS1 && r == 1) {
    lds_round<LOGN, false>(x, r, g0, ltw, p, pinv);
    return;
  }
  if (r > 0) {
    compact_round<LOGN, false>(x, r, g0, ts, p, pinv);
    return;
  }
#pragma unroll
  for (int kk = S::LOGE - S::R0; kk < S::LOGE; ++kk) {
    const int k = S::LOGE - 1 - kk;
    const int eb = S::LOGE - 1 - k;
#pragma unroll
    for (int j = 0; j < (1 << k); ++j) {
      const double w = cld(ts.tw0, (1 << k) + j);
#pragma unroll
      for (int b = 0; b < (1 << eb); ++b) {
        const int e = (j << (eb + 1)) | b;
        if (gs_reduces(g0 + kk - (S::LOGE - S::R0)))
          gs_bfly<true>(x[e], x[e | (1 << eb)], w, p, pinv);
        else
          gs_bfly<false>(x[e], x[e | (1 << eb)], w, p, pinv);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) x[e] = reduce_bal(x[e], p, pinv);
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
  int limb, poly;
  if (MODE == NTT_DIGIT || MODE == NTT_DIGIT2 || MODE == NTT_DIGIT3) {
    // The digit transforms read one source limb per (ciphertext, digit) for
    // all L + alpha target primes.  Split the (source x prime) grid into 8
    // blocks, one per XCD: two halves of the primes x four quarters of the
    // sources.  Each XCD then keeps about half the primes' twiddle tables
    // in its L2, reads each of its sources once (the half's transforms of
    // a source are numbered consecutively) and every source is read twice.
    const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int ph = (job.nlimb + 1) >> 1;                 // primes in half 0
    const int g = x & 1;
    const int np = g ? job.nlimb - ph : ph;
    const int sq = (job.npoly + 3) >> 2;                  // sources per quarter
    const int src = (x >> 1) * sq + l / np;
    if (l / np >= sq || src >= job.npoly) return;
    poly = src;
    limb = g * ph + l % np;
  } else {
    const int item = xcd_item(job.count);
    if (item >= job.count) return;
    limb = item / job.npoly;
    poly = item - limb * job.npoly;
  }
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const TwSrc tw{tb.tw_fwd + (size_t)prime * tb.tw_len,
                 tb.tw_cmp_f + (size_t)prime * tb.tw_cmp_len, tb.tw_cst_f + (size_t)prime * 32};
  const size_t off = (size_t)poly * job.poly_stride + (size_t)limb * S::N;
  double* dst = job.base + off;
  const auto rd = make_rsrc(dst, S::N * 8);
  const auto ro = make_rsrc((job.out ? job.out : job.base) + off, S::N * 8);
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  double x[S::E];
  static_assert(fwd_schedule_ok<LOGN>(0), "forward reduction schedule");
  if constexpr (MODE == NTT_DIGIT) {
    // poly = ct * L + j; limb = target prime i.  Source: limb j of the
    // third component, stored as the canonical digit D_j in [0, q_j),
    // below 2 p_i: transformed as it is (see ct_bfly for the bound).
    const int ct = poly / job.digits;
    const int j = poly - ct * job.digits;
    const auto rs = make_rsrc(job.src + (size_t)ct * job.src_ct_stride + (size_t)j * S::N, S::N * 8);
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      const int e = brv_c(i, S::LOGE);
      x[e] = buf_load(rs, vo, e * S::T * 8);
    }
  } else if constexpr (MODE == NTT_DIGIT2) {
    // Two primes per digit: limbs 2j and 2j + 1 of the source hold digit
    // j's canonical mixed-radix digits (v_0, v_1); its value in the target
    // prime is v_0 + [q_{2j}]_p v_1, below DIGIT2_IN p.
    const int ct = poly / job.digits;
    const int j = poly - ct * job.digits;
    const double* s0 = job.src + (size_t)ct * job.src_ct_stride + (size_t)(2 * j) * S::N;
    const auto rs0 = make_rsrc(s0, S::N * 8);
    const auto rs1 = make_rsrc(s0 + S::N, S::N * 8);
    const double cq = cld(tb.dig_c, j * job.nlimb + limb);
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      const int e = brv_c(i, S::LOGE);
      x[e] = buf_load(rs0, vo, e * S::T * 8) + mul_lazy(buf_load(rs1, vo, e * S::T * 8), cq, p, pinv);
    }
  } else if constexpr (MODE == NTT_DIGIT3) {
    // Three primes per digit: limbs 3j .. 3j + 2 hold (v_0, v_1, v_2); the
    // value in the target prime, reduced to balanced form (DIGIT_IN above).
    const int ct = poly / job.digits;
    const int j = poly - ct * job.digits;
    const double* s0 = job.src + (size_t)ct * job.src_ct_stride + (size_t)(3 * j) * S::N;
    const auto rs0 = make_rsrc(s0, S::N * 8);
    const auto rs1 = make_rsrc(s0 + S::N, S::N * 8);
    const auto rs2 = make_rsrc(s0 + 2 * S::N, S::N * 8);
    const double c1 = cld(tb.dig_c, (j * job.nlimb + limb) * 2);
    const double c2 = cld(tb.dig_c, (j * job.nlimb + limb) * 2 + 1);
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      const int e = brv_c(i, S::LOGE);
      const unsigned o = e * S::T * 8;
      x[e] = reduce_bal(buf_load(rs0, vo, o) + mul_lazy(buf_load(rs1, vo, o), c1, p, pinv) +
                            mul_lazy(buf_load(rs2, vo, o), c2, p, pinv),
                        p, pinv);
    }
  } else {
    // loads in bit-reversed element order: the first stage pairs e with
    // e + E/2, so it can start as soon as the first two loads land
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      const int e = brv_c(i, S::LOGE);
      x[e] = buf_load(rd, vo, e * S::T * 8);
    }
  }
#pragma unroll
  for (int r = 0; r < S::ROUNDS; ++r) {
    if (r > 0) exchange<LOGN>(x, r - 1, r, lds, r > 1);
    fwd_round<LOGN>(x, r,
                    fwd_reduces_after<LOGN>(r, 0) &&
                        !((MODE == NTT_DIGIT || MODE == NTT_DIGIT2 || MODE == NTT_DIGIT3) &&
                          r == S::ROUNDS - 1),
                    tw, p, pinv);
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(x[e], ro, vo, e * S::T * 8);
}

// Tensor component of a squaring from one limb of the operand's
// transforms: a^2 (CROSS false, a = ra) or 2 a0 a1 (CROSS true, a0 = ra,
// a1 = rb).  Loads run one group of G elements ahead of the products, each
// group's addresses fenced on the previous group's results.  LAZY leaves
// the products unreduced (below 0.875 p): the 14 stages of a half-limb
// inverse then keep sums below 7.7 p and the differences entering a
// product below 13.9 p (gs_reduces' sequence from 0.875 p).
template <int LOGN, bool CROSS, bool LAZY = false>
__device__ __forceinline__ void tensor_square(double (&x)[NttShape<LOGN>::E],
                                              __amdgpu_buffer_rsrc_t ra,
                                              __amdgpu_buffer_rsrc_t rb, unsigned vo,
                                              double p, double pinv) {
  using S = NttShape<LOGN>;
  constexpr int G = 4;
  double ba[2][G], bb[2][G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    ba[0][i] = buf_load(ra, vo, i * S::T * 8);
    if constexpr (CROSS) bb[0][i] = buf_load(rb, vo, i * S::T * 8);
  }
#pragma unroll
  for (int g = 0; g < S::E; g += G) {
    const int slot = (g / G) & 1;
    if (g + G < S::E) {
      unsigned v = vo;
      if (g) asm volatile("" : "+v"(v) : "v"(x[g - 1]));
#pragma unroll
      for (int i = 0; i < G; ++i) {
        ba[slot ^ 1][i] = buf_load(ra, v, (g + G + i) * S::T * 8);
        if constexpr (CROSS) bb[slot ^ 1][i] = buf_load(rb, v, (g + G + i) * S::T * 8);
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const double a = ba[slot][i];
      const double pr = CROSS ? mul_lazy(a + a, bb[slot][i], p, pinv) : mul_lazy(a, a, p, pinv);
      x[g + i] = LAZY ? pr : reduce_bal(pr, p, pinv);
    }
  }
}

// Tensor component of a product: a b (CROSS false) or a b + c d (CROSS
// true), loads in groups of 8 elements, each group fenced on the previous
// one's results.
template <int LOGN, bool CROSS>
__device__ __forceinline__ void tensor_product(double (&x)[NttShape<LOGN>::E],
                                               __amdgpu_buffer_rsrc_t ra,
                                               __amdgpu_buffer_rsrc_t rb,
                                               __amdgpu_buffer_rsrc_t rc,
                                               __amdgpu_buffer_rsrc_t rd, unsigned vo,
                                               double p, double pinv) {
  using S = NttShape<LOGN>;
  unsigned v = vo;
#pragma unroll
  for (int g = 0; g < S::E; g += 8) {
    if (g) asm volatile("" : "+v"(v) : "v"(x[g - 1]));
#pragma unroll
    for (int e = g; e < g + 8 && e < S::E; ++e) {
      const unsigned so = e * S::T * 8;
      if constexpr (CROSS) {
        const double a = buf_load(ra, v, so), b = buf_load(rb, v, so);
        const double c = buf_load(rc, v, so), d = buf_load(rd, v, so);
        x[e] = reduce_bal(mul_lazy(a, b, p, pinv) + mul_lazy(c, d, p, pinv), p, pinv);
      } else {
        x[e] = mul_bal(buf_load(ra, v, so), buf_load(rb, v, so), p, pinv);
      }
    }
  }
}

template <int LOGN, int MODE>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_ntt_inv(NttJob job, Tables tb) {
  using S = NttShape<LOGN>;
  __shared__ uint32_t lds[S::LDS_WORDS];
  const int item = xcd_item(job.count);
  if (item >= job.count) return;
  const int limb = item / job.npoly;
  const int poly = item - limb * job.npoly;
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const TwSrc tw{tb.tw_inv + (size_t)prime * tb.tw_len,
                 tb.tw_cmp_i + (size_t)prime * tb.tw_cmp_len, tb.tw_cst_i + (size_t)prime * 32};
  const size_t off = (size_t)poly * job.poly_stride + (size_t)limb * S::N;
  double* dst = job.base + off;
  const auto rd = make_rsrc(dst, S::N * 8);
  const auto ro = make_rsrc((job.out ? job.out : job.base) + off, S::N * 8);
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  double x[S::E];
  if constexpr (MODE == INV_TENSOR || MODE == INV_TENSOR2) {
    // poly = ct * 3 + k: form the k-th tensor component from the operands'
    // transforms (a in src, b in src_b, or b = a for a squaring):
    // d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1.  k is uniform over the
    // block, so it selects a whole load loop once: branches inside the loop
    // would make every load wait for the one before it.
    const int ct = poly / 3;
    const int k = poly - ct * 3;
    const size_t o0 = (size_t)ct * job.src_ct_stride + (size_t)limb * S::N;
    const size_t o1 = o0 + job.src_ct_stride / 2;
    const auto ra0 = make_rsrc(job.src + o0, S::N * 8);
    const auto ra1 = make_rsrc(job.src + o1, S::N * 8);
    if constexpr (MODE == INV_TENSOR) {
      if (k == 1)
        tensor_square<LOGN, true>(x, ra0, ra1, vo, p, pinv);
      else
        tensor_square<LOGN, false>(x, k == 2 ? ra1 : ra0, ra1, vo, p, pinv);
    } else {
      const auto rb0 = make_rsrc(job.src_b + o0, S::N * 8);
      const auto rb1 = make_rsrc(job.src_b + o1, S::N * 8);
      if (k == 1)
        tensor_product<LOGN, true>(x, ra0, rb1, ra1, rb0, vo, p, pinv);
      else if (k == 0)
        tensor_product<LOGN, false>(x, ra0, rb0, ra0, rb0, vo, p, pinv);
      else
        tensor_product<LOGN, false>(x, ra1, rb1, ra1, rb1, vo, p, pinv);
    }
  } else {
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = buf_load(rd, vo, e * S::T * 8);
  }
  int g0 = 0;  // stages done before the current round
#pragma unroll
  for (int rr = 0; rr < S::ROUNDS; ++rr) {
    const int r = S::ROUNDS - 1 - rr;
    if (rr > 0) exchange<LOGN>(x, r + 1, r, lds, rr > 1);
    inv_round<LOGN>(x, r, g0, tw, p, pinv);
    g0 += S::stages(r);
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(x[e], ro, vo, e * S::T * 8);
}

// ---------------------------------------------------------------- host ---

// Forward transform of a 2^15-point limb by two workgroups of 512 threads,
// one per half.  Stage 0 pairs index i with i + 2^14 and nothing later
// mixes the halves, so each workgroup loads the whole limb, keeps its half
// of stage 0 (X + W Y or X - W Y, W = psi^(2^14)) and runs stages 1..14 as
// a 2^14-point transform whose twiddles are the full transform's for that
// half: psi_br[2^s' (2 + h) + m'] at sub-stage s', block m'.  Half a limb
// needs 72 KB of LDS (the exchange buffer and round 1's twiddle rows) and
// at most 128 VGPRs per thread, so two workgroups share a CU and one loads
// or stores while the other computes.  Outputs land at the full
// transform's positions: standard index h 2^14 + i' at
// (i' mod 32) 1024 + h 512 + i' / 32.
template <int MODE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt_fwd_half(NttJob job, Tables tb) {
  static_assert(MODE == NTT_INPLACE, "digit transforms run by coefficient parity (k_ntt_fwd_par)");
  using S = NttShape<14>;
  constexpr int NF = 1 << 15;
  constexpr int R1 = 1 << S::s_start(1);   // round 1's index rows
  static_assert(R1 * LDS_ROW == 512, "one table entry per thread");
  __shared__ uint32_t lds[S::LDS_WORDS];
  __shared__ double ltw[R1 * LDS_ROW];
  const int item2 = xcd_item(job.count * 2);
  if (item2 >= job.count * 2) return;
  const int h = item2 & 1;
  const int item = item2 >> 1;
  const int limb = item / job.npoly;
  const int poly = item - limb * job.npoly;
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  // half 1 takes X - W Y = X + (-W) Y: one uniform sign flip of the twiddle
  const double w0 = h ? -cld(tb.tw_half0, prime) : cld(tb.tw_half0, prime);
  const TwSrc tw{tb.tw_half + ((size_t)prime * 2 + h) * tb.tw_half_len,
                 tb.tw_cmp_h + ((size_t)prime * 2 + h) * tb.tw_cmp_h_len,
                 tb.tw_cst_f + (size_t)prime * 32};
  // round 1's rows into LDS (read after the first exchange's barriers)
  ltw[threadIdx.x] = tb.tw_r1_f[((size_t)prime * 2 + h) * 512 + threadIdx.x];
  // Both halves read the whole input limb, so the output must be another
  // buffer (the host never launches this kernel in place).
  const size_t off = (size_t)poly * job.poly_stride + (size_t)limb * NF;
  const auto rd = make_rsrc(job.out + off, NF * 8);
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  double x[S::E];
  static_assert(fwd_schedule_ok<14>(1), "forward reduction schedule");
  // the schedule reduces after round 1 (stage 0 and rounds 0, 1: ten
  // stages) and at the end; the mid reduction is replaced by the half one
  constexpr int HALF_REDUCE_ROUND = 2;
  static_assert(S::ROUNDS == 3 && fwd_reduces_after<14>(HALF_REDUCE_ROUND - 1, 1) &&
                    1 + S::stages(0) + S::stages(1) == FWD_STAGES_PER_REDUCTION,
                "half reduction placement");
  {
    const auto rs = make_rsrc(job.base + off, NF * 8);
    // Loads in groups of G elements, software-pipelined one group ahead:
    // group g + 1 is issued (fenced on group g - 1's results) before group g
    // is processed, so at most two groups of loads are in flight.
    constexpr int G = 8;
    double bx[2][G], by[2][G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      bx[0][i] = buf_load(rs, vo, i * S::T * 8);
      by[0][i] = buf_load(rs, vo, (i * S::T + (NF >> 1)) * 8);
    }
#pragma unroll
    for (int g = 0; g < S::E; g += G) {
      const int slot = (g / G) & 1;
      if (g + G < S::E) {
        unsigned v = vo;
        if (g) asm volatile("" : "+v"(v) : "v"(x[g - 1]));
#pragma unroll
        for (int i = 0; i < G; ++i) {
          bx[slot ^ 1][i] = buf_load(rs, v, (g + G + i) * S::T * 8);
          by[slot ^ 1][i] = buf_load(rs, v, ((g + G + i) * S::T + (NF >> 1)) * 8);
        }
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const double X = bx[slot][i], Y = by[slot][i];
        x[g + i] = X + mul_lazy(Y, w0, p, pinv);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < S::ROUNDS; ++r) {
    if (r > 0) exchange<14>(x, r - 1, r, lds, r > 1);
    // Inputs are residues of the limb's prime (below p in absolute value):
    // the ten stages to the end of round 1 leave values below 13.5 p
    // (ct_bound, as from inputs below 2 p).  Only the X operands of round
    // 2's first stage (elements 0..E/2-1: it pairs e with e + E/2) are
    // reduced, at that round's start: its products take |Y| < 13.5 p
    // (results below 1.9 p), so it outputs below 2.4 p and the last four
    // stages below 6 p (ct_bfly's bound), half the reductions of reducing
    // every value after round 1; the last round reduces every value.
    fwd_round<14, true>(x, r, fwd_reduces_after<14>(r, 1) && r != HALF_REDUCE_ROUND - 1, tw, p,
                        pinv, ltw, r == HALF_REDUCE_ROUND);
  }
  const unsigned so = (h * S::T + tid) * 8;
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(x[e], rd, so, e * 1024 * 8);
}

// Digit transforms of 2^15-point limbs by coefficient parity.  With x_e
// and x_o a digit's even and odd coefficients, x(z) = x_e(z^2) + z x_o(z^2);
// the full transform's standard positions 2k and 2k + 1 are the points z
// and -z, z = psi^(2 brv_14(k) + 1), so its outputs there are
// E_k + z O_k and E_k - z O_k, E and O the 2^14-point negacyclic transforms
// of x_e and x_o for the root psi^2.  Since psi^(2 brv_14(i)) =
// psi^(brv_15(i)) for i < 2^14, those transforms use the full transform's
// twiddles of stages 0..13 (slot 2^s + m).  One workgroup of 512 threads
// takes one parity h of one (digit, target prime): it loads every second
// coefficient of the digit's sources (SPLIT: half h of sources that their
// producers store by coefficient parity, c at (c mod 2) 2^14 + c/2, read
// contiguously; otherwise natural order, where the other parity's workgroup,
// on the same XCD, reads the other half of the same cache lines), forms
// each value in the target prime once, and stores the unreduced result to half
// h of the limb in the 2^14 transform's order (standard index k at
// (k mod 32) 512 + k / 32).  The last stage, E_k +- z O_k, is left to the
// key-switch product (k_ks_mac_par): unlike a split by the top index bit
// (k_ntt_fwd_half), no source is loaded, and no digit value formed, twice.
//
// Bounds: nine stages (rounds 0 and 1) from a one-prime digit below 2 p or a
// two-prime one below 2.61 p stay below 13.2 p (three-prime digits start
// reduced); round 2 reduces the X operands of its first stage only, so that
// stage ends below (1/2 + 1/2 + 0.103 x 13.2) p and the last four below
// PAR_OUT p; the key-switch product's E + z O then stays below 7 p.
constexpr double PAR_MID = ct_bound(DIGIT2_IN, 9);
constexpr double PAR_OUT = ct_bound(1.0 + 0.103 * PAR_MID, 4);
static_assert(PAR_MID < 15.1 && PAR_OUT < 5.9 && 1.103 * PAR_OUT + 0.5 < 7.0,
              "parity digit transform bounds");
static_assert(ct_bound(DIGIT_IN, 9) < PAR_MID, "one-prime digits are the smaller");

template <int MODE, bool SPLIT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt_fwd_par(NttJob job, Tables tb) {
  using S = NttShape<14>;
  constexpr int NF = 1 << 15;
  constexpr int R1 = 1 << S::s_start(1);   // round 1's index rows
  static_assert(R1 * LDS_ROW == 512, "one table entry per thread");
  static_assert(MODE == NTT_DIGIT || MODE == NTT_DIGIT2 || MODE == NTT_DIGIT3, "digit modes");
  __shared__ uint32_t lds[S::LDS_WORDS];
  __shared__ double ltw[R1 * LDS_ROW];
  // the digit transforms' XCD split (k_ntt_fwd), the two parities of a
  // (source, prime) pair in consecutive workgroups of one XCD
  const int xc = blockIdx.x & 7, l2 = blockIdx.x >> 3;
  const int h = l2 & 1;
  const int l = l2 >> 1;
  const int ph = (job.nlimb + 1) >> 1;
  const int g = xc & 1;
  const int np = g ? job.nlimb - ph : ph;
  const int sq = (job.npoly + 3) >> 2;
  const int src = (xc >> 1) * sq + l / np;
  if (l / np >= sq || src >= job.npoly) return;
  const int poly = src;
  const int limb = g * ph + l % np;
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const TwSrc tw{tb.tw_fwd + (size_t)prime * tb.tw_len,
                 tb.tw_cmp_par + (size_t)prime * tb.tw_cmp_h_len,
                 tb.tw_cst_f + (size_t)prime * 32};
  // round 1's rows into LDS (read after the first exchange's barriers)
  ltw[threadIdx.x] = tb.tw_r1_par[(size_t)prime * 512 + threadIdx.x];
  const int ct = poly / job.digits;
  const int j = poly - ct * job.digits;
  const double* s0 = job.src + (size_t)ct * job.src_ct_stride + (size_t)(MODE == NTT_DIGIT3 ? 3 * j : MODE == NTT_DIGIT2 ? 2 * j : j) * NF;
  // element e of thread tid in round 0 is sub-index e 512 + tid, source
  // coefficient 2 (e 512 + tid) + h, stored there or (SPLIT) at
  // h 2^14 + e 512 + tid
  const int tid = threadIdx.x;
  const unsigned vo = SPLIT ? (h * (NF / 2) + tid) * 8 : (2 * tid + h) * 8;
  constexpr unsigned ES = SPLIT ? S::T * 8 : 2 * S::T * 8;
  double x[S::E];
  if constexpr (MODE == NTT_DIGIT) {
    // canonical digits in [0, q_j), below 2 p
    const auto rs = make_rsrc(s0, NF * 8);
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = buf_load(rs, vo, e * ES);
  } else if constexpr (MODE == NTT_DIGIT2) {
    // v_0 + [q_{2j}]_p v_1, below DIGIT2_IN p; loads one group of G ahead,
    // each group's addresses fenced on the previous group's results
    const auto rs0 = make_rsrc(s0, NF * 8);
    const auto rs1 = make_rsrc(s0 + NF, NF * 8);
    const double cq = cld(tb.dig_c, j * job.nlimb + limb);
    constexpr int G = 8;
    double ax[2][G], bx[2][G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      ax[0][i] = buf_load(rs0, vo, i * ES);
      bx[0][i] = buf_load(rs1, vo, i * ES);
    }
#pragma unroll
    for (int g0 = 0; g0 < S::E; g0 += G) {
      const int slot = (g0 / G) & 1;
      if (g0 + G < S::E) {
        unsigned v = vo;
        if (g0) asm volatile("" : "+v"(v) : "v"(x[g0 - 1]));
#pragma unroll
        for (int i = 0; i < G; ++i) {
          ax[slot ^ 1][i] = buf_load(rs0, v, (g0 + G + i) * ES);
          bx[slot ^ 1][i] = buf_load(rs1, v, (g0 + G + i) * ES);
        }
      }
#pragma unroll
      for (int i = 0; i < G; ++i) x[g0 + i] = ax[slot][i] + mul_lazy(bx[slot][i], cq, p, pinv);
    }
  } else {
    // v_0 + [q_g]_p v_1 + [q_g q_{g+1}]_p v_2 reduced to balanced form
    // (k_ntt_fwd); loads as above
    const auto rs0 = make_rsrc(s0, NF * 8);
    const auto rs1 = make_rsrc(s0 + NF, NF * 8);
    const auto rs2 = make_rsrc(s0 + 2 * NF, NF * 8);
    const double c1 = cld(tb.dig_c, (j * job.nlimb + limb) * 2);
    const double c2 = cld(tb.dig_c, (j * job.nlimb + limb) * 2 + 1);
    constexpr int G = 4;
    double ax[2][G], bx[2][G], cx[2][G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      ax[0][i] = buf_load(rs0, vo, i * ES);
      bx[0][i] = buf_load(rs1, vo, i * ES);
      cx[0][i] = buf_load(rs2, vo, i * ES);
    }
#pragma unroll
    for (int g0 = 0; g0 < S::E; g0 += G) {
      const int slot = (g0 / G) & 1;
      if (g0 + G < S::E) {
        unsigned v = vo;
        if (g0) asm volatile("" : "+v"(v) : "v"(x[g0 - 1]));
#pragma unroll
        for (int i = 0; i < G; ++i) {
          ax[slot ^ 1][i] = buf_load(rs0, v, (g0 + G + i) * ES);
          bx[slot ^ 1][i] = buf_load(rs1, v, (g0 + G + i) * ES);
          cx[slot ^ 1][i] = buf_load(rs2, v, (g0 + G + i) * ES);
        }
      }
#pragma unroll
      for (int i = 0; i < G; ++i)
        x[g0 + i] = reduce_bal(ax[slot][i] + mul_lazy(bx[slot][i], c1, p, pinv) +
                                   mul_lazy(cx[slot][i], c2, p, pinv),
                               p, pinv);
    }
  }
  // the forward schedule would reduce after round 1 (nine stages) and at
  // the end: the first is replaced by the reduction of round 2's first-stage
  // X operands, the second left to the key-switch product (bounds above)
  static_assert(S::ROUNDS == 3 && S::stages(0) + S::stages(1) == 9 &&
                    !fwd_reduces_after<14>(0, 0) && fwd_reduces_after<14>(1, 0),
                "parity reduction placement");
#pragma unroll
  for (int r = 0; r < S::ROUNDS; ++r) {
    if (r > 0) exchange<14>(x, r - 1, r, lds, r > 1);
    fwd_round<14, true>(x, r, false, tw, p, pinv, ltw, r == 2);
  }
  const auto rd = make_rsrc(job.out + (size_t)poly * job.poly_stride + (size_t)limb * NF +
                                (size_t)h * (NF / 2),
                            NF / 2 * 8);
#pragma unroll
  for (int e = 0; e < S::E; ++e) buf_store(x[e], rd, tid * 8, e * S::T * 8);
}

// The key-switch product fused with the digit transforms (N = 2^15): a
// workgroup of 512 threads takes one ciphertext, one target prime of the
// key-switching basis (limb i < L + 1) and one output half h, and for each
// digit D_j = [c2]_{q_j}, j = 0..L-1, runs the half-limb forward transform
// (the split by the top index bit of k_ntt_fwd_half) in prime i, then multiplies the result by
// the key's NTT-domain limbs evk[j][0][i] and evk[j][1][i] (same positions)
// and adds the products to two sums held in registers across the digits.
// The digits' transforms are never written; the sums are written once, in
// the layout of k_ks_mac's output (the split inverse's input).  Bounds: the
// unreduced digit transforms stay below 6 p (k_ntt_fwd_half's schedule
// from inputs below 2 p), so each
// lazy product with a balanced key is below 1.05 p and eight of them plus
// a reduced sum below 9 p < 2^53 / p: the sums are reduced every 8 digits.
// Work items: ciphertexts in groups of CG = min(4, n_ct); within a group,
// item = (limb, half) pair * CG + ciphertext, groups one after the other,
// and each XCD takes a contiguous range, so that the workgroups resident on
// an XCD at one time cover a few ciphertexts times a few (limb, half) pairs
// and share both the digits' source limbs and the key's limbs through L2.
// Registers: 32 values plus 2 x 32 sums per thread (two waves per SIMD,
// one workgroup per CU).
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
k_ks_fused(NttJob job, const double* __restrict__ evk, double* __restrict__ acc, Tables tb) {
  using S = NttShape<14>;
  constexpr int NF = 1 << 15;
  constexpr int R1 = 1 << S::s_start(1);
  static_assert(R1 * LDS_ROW == 512, "one table entry per thread");
  __shared__ uint32_t lds[S::LDS_WORDS];
  __shared__ double ltw[R1 * LDS_ROW];
  const int n_ct = job.npoly, L = job.digits, K = job.nlimb;
  const int cg = n_ct < 4 ? n_ct : 4;
  const int count = ((n_ct + cg - 1) / cg) * cg * 2 * K;
  const int item = xcd_item(count);
  if (item >= count) return;
  const int pair = (item / cg) % (2 * K);
  const int ct = (item / (cg * 2 * K)) * cg + item % cg;
  if (ct >= n_ct) return;
  const int limb = pair >> 1, h = pair & 1;
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const double w0 = h ? -cld(tb.tw_half0, prime) : cld(tb.tw_half0, prime);
  const TwSrc tw{tb.tw_half + ((size_t)prime * 2 + h) * tb.tw_half_len,
                 tb.tw_cmp_h + ((size_t)prime * 2 + h) * tb.tw_cmp_h_len,
                 tb.tw_cst_f + (size_t)prime * 32};
  // round 1's rows into LDS once (read after the first exchange's barriers)
  ltw[threadIdx.x] = tb.tw_r1_f[((size_t)prime * 2 + h) * 512 + threadIdx.x];
  const int tid = threadIdx.x;
  const unsigned vo = tid * 8;
  const unsigned so = (h * S::T + tid) * 8;   // this thread's output positions
  static_assert(fwd_schedule_ok<14>(1), "forward reduction schedule");
  constexpr int HALF_REDUCE_ROUND = 2;
  static_assert(S::ROUNDS == 3 && fwd_reduces_after<14>(HALF_REDUCE_ROUND - 1, 1) &&
                    1 + S::stages(0) + S::stages(1) == FWD_STAGES_PER_REDUCTION,
                "half reduction placement");
  double a0[S::E], a1[S::E];
#pragma unroll
  for (int e = 0; e < S::E; ++e) a0[e] = a1[e] = 0.0;
  double x[S::E];
  // digit j's source: canonical residues in [0, q_j), below 2 p_i; the X
  // operands of stage 0 of the next digit are loaded into x[e] as soon as
  // this digit's product has used x[e], so they arrive during the products
  const double* src = job.src + (size_t)ct * job.src_ct_stride;
  {
    const auto rs = make_rsrc(src, NF * 8);
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = buf_load(rs, vo, e * S::T * 8);
  }
  for (int j = 0; j < L; ++j) {
    const auto rs = make_rsrc(src + (size_t)j * NF, NF * 8);
    // stage 0 of this half: X + w0 Y (lazy), X and Y NF/2 apart
    constexpr int G = 8;
#pragma unroll
    for (int g = 0; g < S::E; g += G) {
      double y[G];
#pragma unroll
      for (int i = 0; i < G; ++i) y[i] = buf_load(rs, vo, ((g + i) * S::T + (NF >> 1)) * 8);
#pragma unroll
      for (int i = 0; i < G; ++i) x[g + i] += mul_lazy(y[i], w0, p, pinv);
    }
#pragma unroll
    for (int r = 0; r < S::ROUNDS; ++r) {
      // the first exchange of a later digit waits for every wave's reads of
      // the previous digit's last exchange
      if (r > 0) exchange<14>(x, r - 1, r, lds, r > 1 || j > 0);
      fwd_round<14, true>(x, r,
                          fwd_reduces_after<14>(r, 1) && r != HALF_REDUCE_ROUND - 1 &&
                              r != S::ROUNDS - 1,
                          tw, p, pinv, ltw, r == HALF_REDUCE_ROUND);
    }
    const size_t kj = (size_t)j * 2 * K + limb;
    const auto rk0 = make_rsrc(evk + kj * NF, NF * 8);
    const auto rk1 = make_rsrc(evk + (kj + K) * NF, NF * 8);
    // past the last digit the next-digit loads read out of range (zeros)
    const auto rn = make_rsrc(src + (size_t)(j + 1) * NF, j + 1 < L ? NF * 8 : 0);
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const double k0 = buf_load(rk0, so, e * 1024 * 8);
      const double k1 = buf_load(rk1, so, e * 1024 * 8);
      a0[e] += mul_lazy(x[e], k0, p, pinv);
      a1[e] += mul_lazy(x[e], k1, p, pinv);
      x[e] = buf_load(rn, vo, e * S::T * 8);
    }
    if ((j & 7) == 7) {
#pragma unroll
      for (int e = 0; e < S::E; ++e) {
        a0[e] = reduce_bal(a0[e], p, pinv);
        a1[e] = reduce_bal(a1[e], p, pinv);
      }
    }
  }
  const auto ro0 = make_rsrc(acc + ((size_t)ct * 2 * K + limb) * NF, NF * 8);
  const auto ro1 = make_rsrc(acc + ((size_t)(ct * 2 + 1) * K + limb) * NF, NF * 8);
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    buf_store(reduce_bal(a0[e], p, pinv), ro0, so, e * 1024 * 8);
    buf_store(reduce_bal(a1[e], p, pinv), ro1, so, e * 1024 * 8);
  }
}

// Inverse of a 2^15-point limb by two workgroups of 512 threads that stop
// before the last Gentleman-Sande stage.  Every stage but the last pairs
// indices with the same top bit h, so half h (standard indices h 2^14 + i')
// is an independent 2^14-point inverse with the full transform's inverse
// twiddles for that half (the mirror of k_ntt_fwd_half): 72 KB of LDS,
// two workgroups per CU.  The last stage, X + Y and (X - Y) w with
// w = the full inverse's round-0 twiddle at slot 1, couples the halves and
// is left to the consumer, which loads X = U[i'] and Y = V[i'] (U, V: the
// two halves' outputs, reduced to balanced residues).  Input: internal
// order, element e of thread tid at e 1024 + h 512 + tid.  Output (i' =
// 512 e + tid):
//   NTT_INPLACE (the key-switch sum, read by the mod-down): in place, at
//     the positions read, so U[i'] is at (i' / 512) 1024 + (i' mod 512) and
//     V[i'] 512 further;
//   INV_TENSOR, INV_TENSOR2 (read by the scale-and-round): U[i'] at i',
//     V[i'] at 2^14 + i' (the natural positions of the two coefficients the
//     last stage produces from them).
template <int MODE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt_inv_half(NttJob job, Tables tb) {
  using S = NttShape<14>;
  constexpr int NF = 1 << 15;
  constexpr int R1 = 1 << S::s_start(1);
  static_assert(R1 * LDS_ROW == 512, "one table entry per thread");
  __shared__ uint32_t lds[S::LDS_WORDS];
  __shared__ double ltw[R1 * LDS_ROW];
  const int item2 = xcd_item(job.count * 2);
  if (item2 >= job.count * 2) return;
  const int h = item2 & 1;
  const int item = item2 >> 1;
  const int limb = item / job.npoly;
  const int poly = item - limb * job.npoly;
  const int prime = cldi(job.limb_prime, limb);
  const double p = cld(tb.p, prime), pinv = cld(tb.pinv, prime);
  const TwSrc tw{tb.tw_half_inv + ((size_t)prime * 2 + h) * tb.tw_half_len,
                 tb.tw_cmp_hi + ((size_t)prime * 2 + h) * tb.tw_cmp_h_len,
                 tb.tw_cst_i + (size_t)prime * 32};
  // round 1's rows into LDS (read after the barrier that opens the first
  // exchange: that exchange itself is wave-local)
  ltw[threadIdx.x] = tb.tw_r1_i[((size_t)prime * 2 + h) * 512 + threadIdx.x];
  const size_t off = (size_t)poly * job.poly_stride + (size_t)limb * NF;
  const auto rd = make_rsrc(job.base + off, NF * 8);
  const auto ro = make_rsrc((job.out ? job.out : job.base) + off, NF * 8);
  const int tid = threadIdx.x;
  const unsigned vi = (h * S::T + tid) * 8;
  double x[S::E];
  if constexpr (MODE == INV_TENSOR || MODE == INV_TENSOR2) {
    // as in k_ntt_inv (same element stride, 1024), from this half's slots
    const int ct = poly / 3;
    const int k = poly - ct * 3;
    const size_t o0 = (size_t)ct * job.src_ct_stride + (size_t)limb * NF;
    const size_t o1 = o0 + job.src_ct_stride / 2;
    const auto ra0 = make_rsrc(job.src + o0, NF * 8);
    const auto ra1 = make_rsrc(job.src + o1, NF * 8);
    if constexpr (MODE == INV_TENSOR) {
      if (k == 1)
        tensor_square<15, true, true>(x, ra0, ra1, vi, p, pinv);
      else
        tensor_square<15, false, true>(x, k == 2 ? ra1 : ra0, ra1, vi, p, pinv);
    } else {
      const auto rb0 = make_rsrc(job.src_b + o0, NF * 8);
      const auto rb1 = make_rsrc(job.src_b + o1, NF * 8);
      if (k == 1)
        tensor_product<15, true>(x, ra0, rb1, ra1, rb0, vi, p, pinv);
      else if (k == 0)
        tensor_product<15, false>(x, ra0, rb0, ra0, rb0, vi, p, pinv);
      else
        tensor_product<15, false>(x, ra1, rb1, ra1, rb1, vi, p, pinv);
    }
  } else {
#pragma unroll
    for (int e = 0; e < S::E; ++e) x[e] = buf_load(rd, vi, e * 1024 * 8);
  }
  int g0 = 0;  // stages done before the current round
#pragma unroll
  for (int rr = 0; rr < S::ROUNDS; ++rr) {
    const int r = S::ROUNDS - 1 - rr;
    static_assert(S::ROUNDS == 3 && wave_local<14>(2, 1) && !wave_local<14>(1, 0),
                  "exchange barriers of the half inverse");
    if (rr > 0)
      exchange<14, MODE == INV_TENSOR || MODE == INV_TENSOR2>(x, r + 1, r, lds, true);
    inv_round<14, true>(x, r, g0, tw, p, pinv, ltw);
    g0 += S::stages(r);
  }
  if constexpr (MODE == NTT_INPLACE) {
#pragma unroll
    for (int e = 0; e < S::E; ++e) buf_store(x[e], ro, vi, e * 1024 * 8);
  } else {
    const unsigned so = (h * (NF >> 1) + tid) * 8;
#pragma unroll
    for (int e = 0; e < S::E; ++e) buf_store(x[e], ro, so, e * S::T * 8);
  }
}

// Workgroups per XCD for a launch (grid = 8 x this); `halves` = 2 when each
// limb is split over two workgroups.
static int per_xcd(const NttJob& job, int dir, int halves) {
  if (dir == 2) {
    const int ph = (job.nlimb + 1) >> 1;
    const int sq = (job.npoly + 3) >> 2;
    return sq * ph * halves;
  }
  return (job.count * halves + 7) >> 3;
}

template <int LOGN>
static hipError_t launch_ntt(const NttJob& job, const Tables& tb, int dir, hipStream_t st) {
  using S = NttShape<LOGN>;
  if constexpr (LOGN == 15) {
    if ((dir == 1 || dir == 3 || dir == 4) && job.split_inv && tb.tw_half_inv) {
      dim3 grid(per_xcd(job, dir, 2) * 8), block(512);
      if (dir == 1)
        hipLaunchKernelGGL((k_ntt_inv_half<NTT_INPLACE>), grid, block, 0, st, job, tb);
      else if (dir == 4)
        hipLaunchKernelGGL((k_ntt_inv_half<INV_PLAIN>), grid, block, 0, st, job, tb);
      else if (job.src_b == nullptr)
        hipLaunchKernelGGL((k_ntt_inv_half<INV_TENSOR>), grid, block, 0, st, job, tb);
      else
        hipLaunchKernelGGL((k_ntt_inv_half<INV_TENSOR2>), grid, block, 0, st, job, tb);
      return hipGetLastError();
    }
    if (dir == 2 && job.parity && job.split && tb.tw_cmp_par) {
      dim3 grid(per_xcd(job, dir, 2) * 8), block(512);
      // (sources stored by parity: three-prime digits, see the scale-and-round)
      if (job.alpha == 2)
        hipLaunchKernelGGL((k_ntt_fwd_par<NTT_DIGIT2, false>), grid, block, 0, st, job, tb);
      else if (job.alpha == 3 && job.src_split)
        hipLaunchKernelGGL((k_ntt_fwd_par<NTT_DIGIT3, true>), grid, block, 0, st, job, tb);
      else if (job.alpha == 3)
        hipLaunchKernelGGL((k_ntt_fwd_par<NTT_DIGIT3, false>), grid, block, 0, st, job, tb);
      else
        hipLaunchKernelGGL((k_ntt_fwd_par<NTT_DIGIT, false>), grid, block, 0, st, job, tb);
      return hipGetLastError();
    }
    if (dir == 0 && job.out && job.out != job.base && tb.tw_half && job.split) {
      dim3 grid(per_xcd(job, dir, 2) * 8), block(512);
      hipLaunchKernelGGL((k_ntt_fwd_half<NTT_INPLACE>), grid, block, 0, st, job, tb);
      return hipGetLastError();
    }
  }
  // direction 4 without the split inverse: a plain inverse into out
  if (dir == 4) {
    if (!job.out || job.out == job.base) return hipErrorInvalidValue;
    dir = 1;
  }
  const int per = per_xcd(job, dir, 1);
  dim3 grid(per * 8), block(S::T);
  if (dir == 0)
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_INPLACE>), grid, block, 0, st, job, tb);
  else if (dir == 1)
    hipLaunchKernelGGL((k_ntt_inv<LOGN, NTT_INPLACE>), grid, block, 0, st, job, tb);
  else if (dir == 2 && job.alpha == 2)
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_DIGIT2>), grid, block, 0, st, job, tb);
  else if (dir == 2 && job.alpha == 3)
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_DIGIT3>), grid, block, 0, st, job, tb);
  else if (dir == 2)
    hipLaunchKernelGGL((k_ntt_fwd<LOGN, NTT_DIGIT>), grid, block, 0, st, job, tb);
  else if (job.src_b == nullptr)
    hipLaunchKernelGGL((k_ntt_inv<LOGN, INV_TENSOR>), grid, block, 0, st, job, tb);
  else
    hipLaunchKernelGGL((k_ntt_inv<LOGN, INV_TENSOR2>), grid, block, 0, st, job, tb);
  return hipGetLastError();
}

hipError_t run_ks_fused(const NttJob& job, const double* evk, double* acc, const Tables& tb,
                        hipStream_t st) {
  if (!tb.tw_half || job.npoly <= 0) return hipErrorInvalidValue;
  const int cg = job.npoly < 4 ? job.npoly : 4;
  const int count = ((job.npoly + cg - 1) / cg) * cg * 2 * job.nlimb;
  dim3 grid(((count + 7) >> 3) * 8), block(512);
  hipLaunchKernelGGL(k_ks_fused, grid, block, 0, st, job, evk, acc, tb);
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
