// Measurement kernels (not on the evaluation path): the chip-wide ceiling of
// the exact FP64 modular product, and one residue-base conversion (17 -> 18
// or 18 -> 17 primes) computed two ways, the split-FMA rows the library
// uses (conv_row) and integer MFMA on signed byte digits, timed and
// compared residue for residue.
//
// MFMA form.  out_k = sum_i y_i M_ik (mod m_k), |y_i| < 2^48.  Each input is
// written in seven signed base-256 digits, y = sum_a d_a(y) 256^a with
// d_a in [-128, 127] (the bytes of y + sum_a 128 256^a, each minus 128),
// and each folded constant M'_(i,a),k = [256^a M_ik]_(m_k) (balanced) in
// seven signed digits as well.  Then
//   sum_i y_i M_ik = sum_b 256^b S_kb (mod m_k),
//   S_kb = sum_(i,a) d_a(y_i) d_b(M'_(i,a),k),
// a product of a [rows (k, b)] x [K (i, a)] int8 matrix of constants with a
// [K] x [coefficients] int8 matrix of digits, exact in int32 (|S| <= 17 * 7 *
// 128 * 128 < 2^21).  v_mfma_i32_32x32x32_i8 computes it in 32 x 32 tiles
// (any consistent order of K between the two operands; C's lane l holds
// column l mod 32 and, in VGPR r, row 8 (r / 4) + 4 (l / 32) + r mod 4).
// Rows are (k, b) with b = 0..7 (b = 7 zero) so a 32-row tile holds four
// outputs; a lane half holds bytes 4h..4h+3 of each: it forms T_h = sum_r
// 256^r S_k,4h+r exactly (below 2^46), half 1 multiplies by [2^32]_(m_k),
// and one v_permlane32_swap per word brings both halves of an output into
// one lane, which adds and reduces.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nshe_probe.h"
#include "conv.h"

namespace nshe {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ------------------------------------------------------ modular ceiling ---

// Eight independent chains of dependent lazy modular products per thread.
__global__ void __launch_bounds__(256) k_probe_modmul(double* out, int iters, double p,
                                                      double pinv, double w) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = (double)((gid * 8 + c) % 1000003) + 1.0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = mul_lazy(x[c], w, p, pinv);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[gid] = s;
}

// -------------------------------------------------- FP64 MFMA overlap ---

typedef double v4d __attribute__((ext_vector_type(4)));

// MODE 0: 64 FP64 FMAs per lane and iteration (eight chains); 1: four
// independent 16x16x4 FP64 MFMAs per wave and iteration (4096 FMAs per
// wave, 64 per lane); 2: both.
template <int MODE>
__global__ void __launch_bounds__(256) k_probe_overlap(double* out, int iters, double seed) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = seed + (double)threadIdx.x, b = 1.0 + 1e-9 * (double)threadIdx.x;
  double v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = a + c;
  v4d acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
    if constexpr (MODE != 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    if constexpr (MODE != 1) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = __builtin_fma(v[c], b, 1e-300);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += v[c];
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[gid] = s;
}

// ------------------------------------------------------- conversion ---

// Balanced pseudo-random residues: v[r][c] for row r (prime m[r]).
__global__ void __launch_bounds__(256) k_probe_fill(double* v, size_t n, int rows,
                                                    const double* m, uint64_t seed) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * rows) return;
  uint64_t z = seed + gid * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  const double p = m[gid / n];
  const double u = (double)(z >> 15);        // < 2^49
  const double r = u - p * __builtin_floor(u / p);
  v[gid] = r > 0.5 * p ? r - p : r;
}

template <int NT, int NO>
__global__ void __launch_bounds__(256) k_conv_fma(size_t n, const double* __restrict__ y,
                                                  double* __restrict__ out,
                                                  const double* sp, const double* m,
                                                  const double* minv) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double yh[NT], yl[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) split24(y[(size_t)i * n + c], yh[i], yl[i]);
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int kq = opaque_idx(k);
    const double mk = cld(m, kq), mi = cld(minv, kq);
    const double* row = opaque_row(sp, kq * NT * 2);
    const double a = conv_row<NT>(yh, yl, row, mk, mi);
    out[(size_t)k * n + c] = reduce_bal(a, mk, mi);
  }
}

// Signed base-256 digits of |y| < 2^48 (seven, the eighth zero) as two
// words: y + 2^52 + 2^51 keeps 2^51 + y in the low 52 bits of the double,
// and adding sum_a 128 256^a - 2^51 and flipping each digit byte's top bit
// maps byte u to u - 128.
__device__ __forceinline__ void digits7(double y, int& lo, int& hi) {
  const double t = y + 0x1.8p52;
  const uint64_t bits = (uint64_t)__double_as_longlong(t) & 0xfffffffffffffull;
  const uint64_t v = bits + (0x0080808080808080ull - (1ull << 51));
  lo = (int)((uint32_t)v ^ 0x80808080u);
  hi = (int)((uint32_t)(v >> 32) ^ 0x00808080u);
}

// One wave per 32 coefficients (lanes l and l + 32 share coefficient l mod
// 32); blocks of four waves.  atab: [RB][KB][64] lane operands of the
// constant tiles.  c32: [2^32]_(m_k) balanced.
template <int NT, int NO>
__global__ void __launch_bounds__(256) k_conv_mfma(size_t n, const double* __restrict__ y,
                                                   double* __restrict__ out, const v4i* atab,
                                                   const double* c32, const double* m,
                                                   const double* minv) {
  constexpr int KB = (NT + 3) / 4, RB = (NO + 3) / 4, H = RB * 2;
  __shared__ v4i lt[RB * KB * 64];
  for (int i = threadIdx.x; i < RB * KB * 64; i += blockDim.x) lt[i] = atab[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, h = lane >> 5;
  const size_t c = ((size_t)blockIdx.x * 4 + wv) * 32 + (lane & 31);
  const bool ok = c < n;
  v4i bop[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = 4 * kb + 2 * h + t;
      int lo = 0, hi = 0;
      if (ok && i < NT) digits7(y[(size_t)i * n + c], lo, hi);
      bop[kb][2 * t] = lo;
      bop[kb][2 * t + 1] = hi;
    }
  }
  v16i acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = v16i{};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
      acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(lt[(rb * KB + kb) * 64 + lane], bop[kb],
                                                      acc[rb], 0, 0, 0);
  // this half's share of each output: T_h, times [2^32]_m in half 1
  double P[RB * 4];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = rb * 4 + q;
      const double T = (double)acc[rb][4 * q] + 256.0 * (double)acc[rb][4 * q + 1] +
                       65536.0 * (double)acc[rb][4 * q + 2] +
                       16777216.0 * (double)acc[rb][4 * q + 3];
      if (k < NO) {
        const double mk = cld(m, k), mi = cld(minv, k);
        P[k] = mul_lazy(T, h ? cld(c32, k) : 1.0, mk, mi);
      } else {
        P[k] = 0.0;
      }
    }
  // half 0 finishes outputs 0..H-1, half 1 outputs H..2H-1
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const unsigned long long a = __double_as_longlong(P[k]), b = __double_as_longlong(P[k + H]);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32),
                                                     false, false);
    const double u = __longlong_as_double(((unsigned long long)hi[0] << 32) | lo[0]);
    const double v = __longlong_as_double(((unsigned long long)hi[1] << 32) | lo[1]);
    const int kk = h ? k + H : k;
    if (ok && kk < NO) {
      const double mk = h ? cld(m, k + H < NO ? k + H : 0) : cld(m, k);
      const double mi = h ? cld(minv, k + H < NO ? k + H : 0) : cld(minv, k);
      out[(size_t)kk * n + c] = reduce_bal(u + v, mk, mi);
    }
  }
}

// Residues of a and b (balanced or within p/2 + 4) that differ mod m[row].
__global__ void __launch_bounds__(256) k_probe_compare(const double* a, const double* b,
                                                       size_t n, int rows, const double* m,
                                                       unsigned long long* bad) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * rows) return;
  const double p = m[gid / n];
  if (to_canonical(a[gid], p) != to_canonical(b[gid], p)) atomicAdd(bad, 1ull);
}

}  // namespace nshe

using namespace nshe;

namespace {

thread_local std::string g_probe_err;

int probe_fail(const std::string& msg) {
  g_probe_err = msg;
  return -4;
}

#define PCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return probe_fail(std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

typedef unsigned __int128 u128;
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
double bal(uint64_t x, uint64_t m) { return x > m / 2 ? (double)x - (double)m : (double)x; }

// signed base-256 digit b (0..6) of |v| < 2^48
int digit(int64_t v, int b) {
  const uint64_t u = (uint64_t)(v + (int64_t)0x0080808080808080ll);
  return (int)((u >> (8 * b)) & 0xff) - 128;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

template <int NT, int NO>
int run_conversion(const uint64_t* qin, const uint64_t* qout, size_t n, int reps,
                   nshe_conv_probe* res) {
  constexpr int KB = (NT + 3) / 4, RB = (NO + 3) / 4;
  // constants: M_ik uniform-looking, balanced mod qout[k]
  std::vector<int64_t> M((size_t)NT * NO);
  uint64_t z = 0x1234567ull;
  for (int i = 0; i < NT; ++i)
    for (int k = 0; k < NO; ++k) {
      z = z * 6364136223846793005ull + 1442695040888963407ull;
      const uint64_t mk = qout[k];
      M[(size_t)i * NO + k] = (int64_t)bal((z >> 11) % mk, mk);
    }
  std::vector<double> sp((size_t)NO * NT * 2), mo(NO), mi(NO), c32(NO), mq(NT);
  for (int k = 0; k < NO; ++k) {
    const uint64_t mk = qout[k];
    mo[k] = (double)mk;
    mi[k] = 1.0 / (double)mk;
    c32[k] = bal((1ull << 32) % mk, mk);
    for (int i = 0; i < NT; ++i) {
      const double cb = (double)M[(size_t)i * NO + k];
      const double c1 = __builtin_nearbyint(cb * 0x1p-24);
      sp[((size_t)k * NT + i) * 2] = c1;
      sp[((size_t)k * NT + i) * 2 + 1] = cb - c1 * 0x1p24;
    }
  }
  for (int i = 0; i < NT; ++i) mq[i] = (double)qin[i];
  // MFMA constant tiles: lane l of tile (rb, kb): row r = l mod 32 (output
  // k = 4 rb + r / 8, digit b = r mod 8), byte t of half l / 32: input
  // i = 4 kb + 2 (l / 32) + t / 8, digit a = t mod 8
  std::vector<int32_t> at((size_t)RB * KB * 64 * 4, 0);
  for (int rb = 0; rb < RB; ++rb)
    for (int kb = 0; kb < KB; ++kb)
      for (int l = 0; l < 64; ++l)
        for (int t = 0; t < 16; ++t) {
          const int r = l % 32, k = 4 * rb + r / 8, b = r % 8;
          const int i = 4 * kb + 2 * (l / 32) + t / 8, a = t % 8;
          int d = 0;
          if (k < NO && i < NT && a < 7 && b < 7) {
            const uint64_t mk = qout[k];
            uint64_t f = 1;
            for (int s = 0; s < a; ++s) f = mulmod(f, 256, mk);
            const int64_t Mik = M[(size_t)i * NO + k];
            const uint64_t Mc = Mik < 0 ? (uint64_t)(Mik + (int64_t)mk) : (uint64_t)Mik;
            d = digit((int64_t)bal(mulmod(Mc, f, mk), mk), b);
          }
          int32_t& w = at[(((size_t)rb * KB + kb) * 64 + l) * 4 + t / 4];
          w = (int32_t)((uint32_t)w | ((uint32_t)(uint8_t)(int8_t)d << (8 * (t % 4))));
        }
  DevBuf dy, dof, dom, dtab, dbad;
  const size_t tab_doubles = sp.size() + 3 * (size_t)NO + NT;
  PCHK(hipMalloc(&dy.p, (size_t)NT * n * 8));
  PCHK(hipMalloc(&dof.p, (size_t)NO * n * 8));
  PCHK(hipMalloc(&dom.p, (size_t)NO * n * 8));
  PCHK(hipMalloc(&dtab.p, tab_doubles * 8 + at.size() * 4 + 256));
  PCHK(hipMalloc(&dbad.p, 8));
  double* tb = static_cast<double*>(dtab.p);
  double *d_sp = tb, *d_m = d_sp + sp.size(), *d_mi = d_m + NO, *d_c32 = d_mi + NO,
         *d_mq = d_c32 + NO;
  v4i* d_at = reinterpret_cast<v4i*>(reinterpret_cast<char*>(dtab.p) +
                                     ((tab_doubles * 8 + 255) & ~(size_t)255));
  PCHK(hipMemcpy(d_sp, sp.data(), sp.size() * 8, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(d_m, mo.data(), NO * 8, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(d_mi, mi.data(), NO * 8, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(d_c32, c32.data(), NO * 8, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(d_mq, mq.data(), NT * 8, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(d_at, at.data(), at.size() * 4, hipMemcpyHostToDevice));
  PCHK(hipMemset(dbad.p, 0, 8));
  double* y = static_cast<double*>(dy.p);
  double* of = static_cast<double*>(dof.p);
  double* om = static_cast<double*>(dom.p);
  const dim3 blk(256);
  hipLaunchKernelGGL(k_probe_fill, dim3((unsigned)((NT * n + 255) / 256)), blk, 0, 0, y, n, NT,
                     d_mq, 42ull);
  PCHK(hipGetLastError());
  const dim3 gf((unsigned)((n + 255) / 256)), gm((unsigned)((n + 127) / 128));
  hipEvent_t e0, e1;
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  float ms_f = 0.f, ms_m = 0.f;
  for (int pass = 0; pass < 2; ++pass) {   // pass 0 warms up
    PCHK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL((k_conv_fma<NT, NO>), gf, blk, 0, 0, n, y, of, d_sp, d_m, d_mi);
    PCHK(hipEventRecord(e1, 0));
    PCHK(hipEventSynchronize(e1));
    PCHK(hipEventElapsedTime(&ms_f, e0, e1));
    PCHK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL((k_conv_mfma<NT, NO>), gm, blk, 0, 0, n, y, om, d_at, d_c32, d_m, d_mi);
    PCHK(hipEventRecord(e1, 0));
    PCHK(hipEventSynchronize(e1));
    PCHK(hipEventElapsedTime(&ms_m, e0, e1));
  }
  hipLaunchKernelGGL(k_probe_compare, dim3((unsigned)((NO * n + 255) / 256)), blk, 0, 0, of, om, n,
                     NO, d_m, static_cast<unsigned long long*>(dbad.p));
  PCHK(hipGetLastError());
  unsigned long long bad = 0;
  PCHK(hipMemcpy(&bad, dbad.p, 8, hipMemcpyDeviceToHost));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  res->coefficients = n;
  res->ms_fma = ms_f / reps;
  res->ms_mfma = ms_m / reps;
  res->mismatches = bad;
  return 0;
}

}  // namespace

extern "C" {

const char* nshe_probe_last_error(void) { return g_probe_err.c_str(); }

int nshe_probe_modmul(int hip_device, int iters, nshe_modmul_probe* out) {
  if (!out || iters < 1) return probe_fail("bad argument");
  PCHK(hipSetDevice(hip_device));
  const uint64_t p = 562949953421231ull;  // any odd p < 2^49 (rounding-quotient product)
  const int blocks = 256 * 16, threads = 256;
  DevBuf buf;
  PCHK(hipMalloc(&buf.p, (size_t)blocks * threads * 8));
  double* o = static_cast<double*>(buf.p);
  const double pd = (double)p, pinv = 1.0 / pd, w = bal(0x123456789abull % p, p);
  hipEvent_t e0, e1;
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  float ms = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    PCHK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(k_probe_modmul, dim3(blocks), dim3(threads), 0, 0, o, iters, pd, pinv, w);
    PCHK(hipEventRecord(e1, 0));
    PCHK(hipEventSynchronize(e1));
    PCHK(hipEventElapsedTime(&ms, e0, e1));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const double products = (double)blocks * threads * 8 * iters;
  out->ms = ms;
  out->products_per_s = products / (ms * 1e-3);
  out->fp64_ops_per_s = out->products_per_s * 6.0;
  return 0;
}

int nshe_probe_fp64_overlap(int hip_device, int iters, nshe_overlap_probe* out) {
  if (!out || iters < 1) return probe_fail("bad argument");
  PCHK(hipSetDevice(hip_device));
  const int blocks = 256 * 16, threads = 256;
  DevBuf buf;
  PCHK(hipMalloc(&buf.p, (size_t)blocks * threads * 8));
  double* o = static_cast<double*>(buf.p);
  hipEvent_t e0, e1;
  PCHK(hipEventCreate(&e0));
  PCHK(hipEventCreate(&e1));
  float ms[3] = {0.f, 0.f, 0.f};
  for (int mode = 0; mode < 3; ++mode) {
    for (int pass = 0; pass < 2; ++pass) {
      PCHK(hipEventRecord(e0, 0));
      if (mode == 0)
        hipLaunchKernelGGL(k_probe_overlap<0>, dim3(blocks), dim3(threads), 0, 0, o, iters, 1.0);
      else if (mode == 1)
        hipLaunchKernelGGL(k_probe_overlap<1>, dim3(blocks), dim3(threads), 0, 0, o, iters, 1.0);
      else
        hipLaunchKernelGGL(k_probe_overlap<2>, dim3(blocks), dim3(threads), 0, 0, o, iters, 1.0);
      PCHK(hipGetLastError());
      PCHK(hipEventRecord(e1, 0));
      PCHK(hipEventSynchronize(e1));
      PCHK(hipEventElapsedTime(&ms[mode], e0, e1));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const double fmas = (double)blocks * threads * 64 * iters;
  out->ms_valu = ms[0];
  out->ms_mfma = ms[1];
  out->ms_both = ms[2];
  out->fma_per_s_valu = fmas / (ms[0] * 1e-3);
  out->fma_per_s_mfma = fmas / (ms[1] * 1e-3);
  return 0;
}

int nshe_probe_conversion(int hip_device, const uint64_t* in_primes, int n_in,
                          const uint64_t* out_primes, int n_out, size_t n_coef, int reps,
                          nshe_conv_probe* out) {
  if (!in_primes || !out_primes || !out || n_coef == 0 || reps < 1)
    return probe_fail("bad argument");
  PCHK(hipSetDevice(hip_device));
  if (n_in == 17 && n_out == 18) return run_conversion<17, 18>(in_primes, out_primes, n_coef, reps, out);
  if (n_in == 18 && n_out == 17) return run_conversion<18, 17>(in_primes, out_primes, n_coef, reps, out);
  return probe_fail("supported shapes: 17 -> 18 and 18 -> 17 primes");
}

}  // extern "C"
