// C ABI: context (parameter validation, extension basis, constant tables,
// twiddles, relinearization key) and the evaluation entry points.
#include "../../include/nshe.h"

#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace nshe {

using u64 = uint64_t;
using u128 = unsigned __int128;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ------------------------------------------------------- host number theory

static u64 mulmod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }

static u64 powmod(u64 a, u64 e, u64 m) {
  u64 r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit n (the first twelve primes as bases).
static bool is_prime(u64 n) {
  static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (u64 p : bases)
    if (n % p == 0) return n == p;
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (u64 a : bases) {
    u64 x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        composite = false;
        break;
      }
    }
    if (composite) return false;
  }
  return true;
}

static u64 invmod(u64 a, u64 m) { return powmod(a % m, m - 2, m); }  // m prime

static u64 primitive_root(u64 q) {
  std::vector<u64> fs;
  u64 n = q - 1;
  for (u64 d = 2; d * d <= n; d += (d == 2 ? 1 : 2)) {
    if (n % d == 0) {
      fs.push_back(d);
      while (n % d == 0) n /= d;
    }
  }
  if (n > 1) fs.push_back(n);
  for (u64 g = 2;; ++g) {
    bool ok = true;
    for (u64 f : fs)
      if (powmod(g, (q - 1) / f, q) == 1) {
        ok = false;
        break;
      }
    if (ok) return g;
  }
}

static double bal(u64 x, u64 m) {
  x %= m;
  return x > m / 2 ? (double)x - (double)m : (double)x;
}

static u64 prod_mod(const std::vector<u64>& v, int skip, u64 m) {
  u64 r = 1 % m;
  for (int i = 0; i < (int)v.size(); ++i)
    if (i != skip) r = mulmod(r, v[i] % m, m);
  return r;
}

static int brv(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i)
    if (x & (1 << i)) r |= 1 << (bits - 1 - i);
  return r;
}

// Cyclic transform y_k = sum_e x_e w^(e k) mod p, length a power of two
// (iterative radix 2; p < 2^31).
static std::vector<u64> cyclic_transform(std::vector<u64> x, u64 w, u64 p) {
  const size_t n = x.size();
  int bits = 0;
  while ((size_t(1) << bits) < n) ++bits;
  for (size_t i = 0; i < n; ++i) {
    const size_t r = (size_t)brv((int)i, bits);
    if (r > i) std::swap(x[i], x[r]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const u64 wl = powmod(w, n / len, p);
    for (size_t s = 0; s < n; s += len) {
      u64 tw = 1;
      for (size_t j = 0; j < len / 2; ++j) {
        const u64 a = x[s + j], b = x[s + j + len / 2] * tw % p;
        x[s + j] = (a + b) % p;
        x[s + j + len / 2] = (a + p - b) % p;
        tw = tw * wl % p;
      }
    }
  }
  return x;
}

// Coefficients c_0..c_(p-1) of the polynomial f with f(z) = [z in A],
// A = {-(p-1)/2, ..., -1} mod p (the sum of Fermat equalities over the
// negative half): c_0 = f(0) = 0, c_k = -sum_{z != 0} f(z) z^-k for
// 1 <= k <= p-2 (a cyclic transform over the multiplicative group, with z =
// gamma^e for a primitive root gamma), c_(p-1) = -|A|.  p = 2^K + 1 prime.
static std::vector<u64> comparison_poly(u64 p) {
  const u64 n = p - 1, h = n / 2;
  u64 g = 2;
  while (powmod(g, n / 2, p) == 1) ++g;  // 2 is the only prime factor of p - 1
  std::vector<u64> f(n, 0);
  u64 z = 1;
  for (u64 e = 0; e < n; ++e) {
    f[e] = z > h ? 1 : 0;
    z = z * g % p;
  }
  const std::vector<u64> y = cyclic_transform(f, powmod(g, p - 2, p), p);
  std::vector<u64> c(p, 0);
  for (u64 k = 1; k + 1 < p; ++k) c[k] = (p - y[k]) % p;
  c[p - 1] = (p - h) % p;
  return c;
}

static int centred_small(u64 v, u64 p) { return v > p / 2 ? (int)v - (int)p : (int)v; }

}  // namespace nshe

using namespace nshe;

struct nshe_ctx {
  int device = 0;
  int log2n = 0, n = 0, L = 0, LB = 0, K = 0;
  int alpha = 1, dnum = 0;  // data primes per key-switching digit, digits
  u64 t = 0;
  int squarings = -1;
  std::vector<u64> primes;  // q_0..q_{L-1}, b_0..b_L, P_0..P_{alpha-1}
  int loge = 0, r0 = 0, rounds = 0, tw_len = 0;
  void* dev_tables = nullptr;
  int* lp_ext = nullptr;  // identity over 2L+1 limbs
  int* lp_ks = nullptr;   // 0..L-1, 2L+1..2L+alpha
  Tables tb{};
  double* evk = nullptr;  // [dnum][2][L+alpha][N] NTT domain
  bool has_key = false;
  struct GraphEntry {
    hipGraphExec_t exec;
  };
  std::map<std::vector<uintptr_t>, GraphEntry> graphs;
  // kernel timing (HIP events around every launch of a non-graph call)
  bool prof = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double work;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipStream_t cap_stream = nullptr;  // capture-only stream (the null stream cannot capture)
  // the EQ call's second half (tuning streams = 2): its stream and the
  // events that fork it from, and join it back to, the caller's stream
  hipStream_t half_stream = nullptr;
  hipEvent_t half_fork = nullptr, half_join = nullptr;
  nshe_tuning tune{32, 1, 128, 0, 0, 2};  // the autotuner's choice at 32 ciphertexts, N = 2^15
  std::map<uint32_t, double*> galois;  // Galois element -> switching key (NTT domain)
  // comparison polynomial (t = 2^K + 1 prime; lt_K = 0 otherwise): k babies,
  // m giants, coefficient matrix [m][k] (centred ints) on the device
  int lt_K = 0, lt_k = 0, lt_m = 0, lt_top = 0;
  int lt_depth = 0;  // multiplicative depth of the comparison program
  const double* lt_coef = nullptr;  // (exact small integers)
  // noise budget (see budget_of): multiplications a fresh ciphertext takes
  int depth_budget = 0;
  double fresh_bits = 0.0, level_bits = 0.0;
  uint32_t debug = 0;  // NSHE_DEBUG_* switches
  void* scratch = nullptr;  // this device's copy of the no-allocation scratch
};

namespace nshe {

// the exact-lift window: the default, and the debug switch's 1/4
constexpr double kLiftEdge = 0.5 - 0x1p-40;
constexpr double kLiftEdgeWide = 0.25;

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess)                                                       \
      return fail(NSHE_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

static int W_of(const nshe_ctx* c) { return 2 * c->L + 1; }
// limbs of the key-switching basis Q u P
static int KS_of(const nshe_ctx* c) { return c->L + c->alpha; }

// 2^15-point limbs: the inverse transforms feeding the scale-and-round and
// the mod-down run as two half-limb workgroups each, their last stage
// applied by those consumers (with the split forward, under one tuning flag).
static bool split_inverse(const nshe_ctx* c) {
  return c->log2n == 15 && c->tune.split_forward && c->tb.tw_half_inv;
}

static Dims dims(const nshe_ctx* c, int n_ct) {
  Dims d{c->n, c->L, c->LB, n_ct};
  d.block = c->tune.ew_block;
  d.ks_chunk = c->tune.ks_chunk;
  d.fused = split_inverse(c) ? 1 : 0;
  d.alpha = c->alpha;
  return d;
}

// ------------------------------------------------------------ profiling

enum Kind { K_SUB, K_LIFT, K_NTT_FWD, K_NTT_INV_TENSOR, K_NTT_INV, K_SCALE, K_NTT_DIGIT,
            K_KS_MAC, K_MODDOWN, K_CONVERT, K_AUTOMORPH, K_ADD, K_LINCOMB, K_MODDOWN_LIFT,
            K_TENSOR_MAC, K_KS_FUSED, K_COUNT };
static const char* kKindName[K_COUNT] = {"sub",   "lift",      "ntt_fwd", "ntt_inv_tensor",
                                         "ntt_inv", "scale", "ntt_digit", "ks_mac",
                                         "moddown", "convert", "automorph", "add", "lincomb",
                                         "moddown_lift", "tensor_mac", "ks_fused"};

static hipEvent_t take_event(nshe_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events on its stream when profiling is on.
struct Prof {
  nshe_ctx* c;
  int kind;
  hipStream_t st;
  double work;
  hipEvent_t a = nullptr;
  Prof(nshe_ctx* c_, int kind_, hipStream_t st_, double work_)
      : c(c_), kind(kind_), st(st_), work(work_) {
    if (c->prof && (a = take_event(c))) (void)hipEventRecord(a, st);
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c->recs.push_back(nshe_ctx::Rec{kind, a, b, work});
  }
};

static double ntt_work(const nshe_ctx* c, int polys_times_limbs) {
  return (double)polys_times_limbs * (c->n / 2) * c->log2n;
}

// ------------------------------------------------------------- workspace

struct Ws {
  double* ext;   // [n_ct][2][W][N]  current ciphertext (limbs 0..L-1) and its lift
  double* fx;    // [n_ct][2][W][N]  the operand's transform
  double* dt;    // [n_ct][3][W][N]
  double* dig;   // [n_ct][dnum][K][N]  (a second operand's lift and transform first)
  double* acc;   // [n_ct][2][K][N], K = L + alpha
};

static size_t dig_limbs(const nshe_ctx* c) {
  const size_t W = W_of(c), K = KS_of(c), D = c->dnum;
  return std::max(D * K, 4 * W);
}

static size_t ws_doubles(const nshe_ctx* c, int n_ct) {
  const size_t W = W_of(c), K = KS_of(c), N = c->n;
  return (size_t)n_ct * N * (2 * W + 2 * W + 3 * W + dig_limbs(c) + 2 * K);
}

static Ws carve(const nshe_ctx* c, void* ws, int n_ct) {
  const size_t W = W_of(c), N = c->n;
  const size_t dig = dig_limbs(c);
  double* p = static_cast<double*>(ws);
  Ws w;
  w.ext = p;
  p += (size_t)n_ct * 2 * W * N;
  w.fx = p;
  p += (size_t)n_ct * 2 * W * N;
  w.dt = p;
  p += (size_t)n_ct * 3 * W * N;
  w.dig = p;
  p += (size_t)n_ct * dig * N;
  w.acc = p;
  return w;
}

static int check_ws(const nshe_ctx* c, void* ws, size_t bytes, int n_ct) {
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  if (bytes < ws_doubles(c, n_ct) * sizeof(double))
    return fail(NSHE_ENOMEM, "workspace smaller than nshe_workspace_bytes(ctx, n_ct)");
  return NSHE_OK;
}

// ---------------------------------------------------------- level pieces

static int ntt_job_ext(nshe_ctx* c, double* base, double* out, int npoly, int dir,
                       hipStream_t st) {
  NttJob j{};
  j.split = c->tune.split_forward;
  j.base = base;
  j.out = out;
  j.poly_stride = (size_t)W_of(c) * c->n;
  j.npoly = npoly;
  j.nlimb = W_of(c);
  j.limb_prime = c->lp_ext;
  j.count = npoly * j.nlimb;
  Prof pf(c, dir ? K_NTT_INV : K_NTT_FWD, st, ntt_work(c, j.count));
  HIPCHK(run_ntt(c->log2n, j, c->tb, dir, st));
  return NSHE_OK;
}

static int ntt_job_ks(nshe_ctx* c, double* base, double* out, int npoly, int dir,
                      hipStream_t st, bool for_moddown = false) {
  NttJob j{};
  j.split = c->tune.split_forward;
  j.split_inv = for_moddown && split_inverse(c) ? 1 : 0;
  j.base = base;
  j.out = out;
  j.poly_stride = (size_t)KS_of(c) * c->n;
  j.npoly = npoly;
  j.nlimb = KS_of(c);
  j.limb_prime = c->lp_ks;
  j.count = npoly * j.nlimb;
  Prof pf(c, dir ? K_NTT_INV : K_NTT_FWD, st, ntt_work(c, j.count));
  HIPCHK(run_ntt(c->log2n, j, c->tb, dir, st));
  return NSHE_OK;
}

// Lift the ciphertexts held in ext (limbs 0..L-1) and transform all limbs
// into fx.
// (lifted: the mod-down that wrote ext already lifted it)
static int prepare_operand(nshe_ctx* c, double* ext, double* fx, int n_ct, hipStream_t st,
                           bool lifted = false) {
  Dims d = dims(c, n_ct);
  if (!lifted) {
    Prof pf(c, K_LIFT, st, 2.0 * n_ct * c->n);
    HIPCHK(run_lift(d, ext, c->tb, st));
  }
  return ntt_job_ext(c, ext, fx, n_ct * 2, 0, st);
}

// fx (NTT domain, operands; the first in fx_a when given, else w.fx; the
// second in fx_b, or squaring) -> dt limbs 0..L-1 of the 3 components:
// [round(t d_k / Q)]_Q, coefficient domain; the third as the
// relinearization digit source (each digit's mixed-radix digits when
// alpha > 1) unless
// `residues` asks for its canonical residues (a three-component output).
// 2^15-point limbs with the split transforms: the key-switch product may
// run fused with the digit transforms (k_ks_fused), a tuning choice.
static bool ks_fused(const nshe_ctx* c) {
  return c->log2n == 15 && c->tune.split_forward && c->tune.ks_fused && c->tb.tw_half &&
         c->alpha == 1;
}

// 2^15-point limbs with the split transforms: the key-switch digits are
// transformed by coefficient parity (k_ntt_fwd_par) and the key-switch
// product applies the last stage (k_ks_mac_par), unless the product runs
// fused.
static bool parity_digits(const nshe_ctx* c) {
  return c->log2n == 15 && c->tune.split_forward && c->tb.tw_cmp_par && c->tb.tw_last &&
         !ks_fused(c);
}

// Where the relinearization digit source (the third component's limbs
// 0..L-1: canonical residues, or each digit's mixed-radix digits) is
// written and read: in place in dt, or, for the digit transforms by parity
// with three-prime digits, in the key-switch sum buffer (idle until the
// key-switch product) by coefficient parity, c at (c mod 2) N/2 + c/2, so
// that each parity's transform reads its half contiguously.  In place, that
// order would overwrite values the scale-and-round's other waves have still
// to read; with 16 or 17 data primes the scale-and-round's extra destination
// spills its scalar registers (measured slower), so one- and two-prime
// digits stay in place and the transform reads every second value.
struct DigitSrc {
  double* p;       // ciphertext 0's limb 0
  size_t stride;   // doubles between ciphertexts
  int split;       // parity order
};
static DigitSrc digit_src(const nshe_ctx* c, const Ws& w) {
  // (the scale-and-round takes this stride from its template constants)
  if (parity_digits(c) && c->alpha == 3) return {w.acc, (size_t)2 * KS_of(c) * c->n, 1};
  return {w.dt + (size_t)2 * W_of(c) * c->n, (size_t)3 * W_of(c) * c->n, 0};
}

static int tensor_scale(nshe_ctx* c, const Ws& w, const double* fx_b, int n_ct, hipStream_t st,
                        const double* fx_a = nullptr, bool residues = false) {
  Dims d = dims(c, n_ct);
  {
    // the tensor product is formed while the inverse transform loads
    NttJob j{};
    j.base = w.dt;
    j.poly_stride = (size_t)W_of(c) * c->n;
    j.npoly = n_ct * 3;
    j.nlimb = W_of(c);
    j.limb_prime = c->lp_ext;
    j.count = j.npoly * j.nlimb;
    j.src = fx_a ? fx_a : w.fx;
    j.src_b = fx_b;
    j.src_ct_stride = (size_t)2 * W_of(c) * c->n;
    j.split_inv = d.fused;
    Prof pf(c, K_NTT_INV_TENSOR, st, ntt_work(c, j.count));
    HIPCHK(run_ntt(c->log2n, j, c->tb, 3, st));
  }
  {
    // a product kept as three components (residues) stays in dt
    const DigitSrc ds = digit_src(c, w);
    const bool own = !residues && ds.split;
    Prof pf(c, K_SCALE, st, 3.0 * n_ct * c->n);
    HIPCHK(run_scale(d, w.dt, c->tb, st, !residues && c->alpha > 1, own ? ds.p : nullptr));
  }
  return NSHE_OK;
}

static int digit_products(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, const double* key);
static int finish_relin(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, double* out,
                        bool lift_out, int64_t* finish_out, int64_t* i64_out, bool accumulate,
                        const WaveTab* finish_tab);

// Key-switch the third component in dt (limbs 0..L-1: canonical residues,
// or with several primes per digit each digit's mixed-radix digits) with
// `key` (the relinearization key unless given) and add the result to the
// first two: (c0 + k0, c1 + k1) into `out` (ext unless given), limbs 0..L-1.
// lift_out: also lift the result (limbs L..2L of out), for a squaring that
// follows at once (only with the split inverse).
// finish_out: write the result to this int64 buffer with the mask's finish
// instead (only with the split inverse); i64_out: write it there as it is.
// accumulate: add the result into out (limbs 0..L-1) instead of storing it.
// finish_tab: as finish_out, into a batched wave's ciphertexts (its table).
static int relin(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st,
                 const double* key = nullptr, double* out = nullptr, bool lift_out = false,
                 int64_t* finish_out = nullptr, int64_t* i64_out = nullptr,
                 bool accumulate = false, const WaveTab* finish_tab = nullptr) {
  if (!key) key = c->evk;
  if (!out) out = w.ext;
  if (ks_fused(c)) {
    NttJob j{};
    j.npoly = n_ct;
    j.digits = c->L;
    j.nlimb = c->L + 1;
    j.limb_prime = c->lp_ks;
    j.count = n_ct * c->L * (c->L + 1);
    j.src = w.dt + (size_t)2 * W_of(c) * c->n;
    j.src_ct_stride = (size_t)3 * W_of(c) * c->n;
    Prof pf(c, K_KS_FUSED, st, ntt_work(c, j.count));
    HIPCHK(run_ks_fused(j, key, w.acc, c->tb, st));
  } else {
    int rc0 = digit_products(c, w, n_ct, st, key);
    if (rc0) return rc0;
  }
  return finish_relin(c, w, n_ct, st, out, lift_out, finish_out, i64_out, accumulate,
                      finish_tab);
}

// The digits' transforms (written to w.dig) and their products with the
// key, summed into w.acc (two kernels).
static int digit_products(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, const double* key) {
  Dims d = dims(c, n_ct);
  const DigitSrc ds = digit_src(c, w);
  NttJob j{};
  j.split = c->tune.split_forward;
  // 2^15-point limbs with the split transforms: digit transforms by
  // coefficient parity, their last stage applied by the key-switch product
  j.parity = d.parity = parity_digits(c) ? 1 : 0;
  j.src_split = ds.split;
  j.base = w.dig;
  j.out = w.dig;
  j.poly_stride = (size_t)KS_of(c) * c->n;
  j.npoly = n_ct * c->dnum;
  j.nlimb = KS_of(c);
  j.limb_prime = c->lp_ks;
  j.count = j.npoly * j.nlimb;
  j.src = ds.p;
  j.src_ct_stride = ds.stride;
  j.digits = c->dnum;
  j.alpha = c->alpha;
  {
    // butterflies done: by parity, 14 of the 15 stages (the key-switch
    // product applies the last)
    const double work = j.parity ? (double)j.count * (c->n / 2) * (c->log2n - 1) : ntt_work(c, j.count);
    Prof pf(c, K_NTT_DIGIT, st, work);
    HIPCHK(run_ntt(c->log2n, j, c->tb, 2, st));
  }
  {
    Prof pf(c, K_KS_MAC, st, (double)n_ct * c->dnum * 2 * KS_of(c) * c->n);
    HIPCHK(run_ks_mac(d, w.dig, key, w.acc, c->tb, st));
  }
  return NSHE_OK;
}

// The key-switch sums in w.acc -> inverse transform -> mod-down (see relin).
static int finish_relin(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, double* out,
                        bool lift_out, int64_t* finish_out, int64_t* i64_out, bool accumulate,
                        const WaveTab* finish_tab) {
  Dims d = dims(c, n_ct);
  int rc = ntt_job_ks(c, w.acc, nullptr, n_ct * 2, 1, st, true);
  if (rc) return rc;
  if ((finish_out || finish_tab) && d.fused) {
    if (finish_tab) d.tab = *finish_tab;
    Prof pf(c, K_MODDOWN, st, 2.0 * n_ct * c->n);
    HIPCHK(run_moddown_finish(d, w.acc, w.dt, finish_out, c->tb, st, 1));
  } else if (i64_out && d.fused) {
    Prof pf(c, K_MODDOWN, st, 2.0 * n_ct * c->n);
    HIPCHK(run_moddown_finish(d, w.acc, w.dt, i64_out, c->tb, st, 0));
  } else if (lift_out && d.fused) {
    Prof pf(c, K_MODDOWN_LIFT, st, 2.0 * n_ct * c->n);
    HIPCHK(run_moddown_lift(d, w.acc, w.dt, out, c->tb, st));
  } else {
    Prof pf(c, K_MODDOWN, st, 2.0 * n_ct * c->n);
    HIPCHK(run_moddown(d, w.acc, w.dt, out, c->tb, st, accumulate ? 1 : 0));
  }
  return NSHE_OK;
}

// Relinearize and write the result to the int64 buffer out (canonical): the
// mod-down writes it directly after the split inverse, else a conversion
// pass follows.
static int relin_i64(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, int64_t* out) {
  Dims d = dims(c, n_ct);
  if (d.fused) return relin(c, w, n_ct, st, nullptr, nullptr, false, nullptr, out);
  int rc = relin(c, w, n_ct, st);
  if (rc) return rc;
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_polys_to_i64(d, w.ext, 2, 2 * W * N, W * N, out, 0, c->tb, st));
  return NSHE_OK;
}

// int64 ciphertexts -> lifted into ext ([n_ct][2][W][N]) -> transformed
// into fx: the conversion and the lift in one kernel.
static int prepare_i64(nshe_ctx* c, const int64_t* in, double* ext, double* fx, int n_ct,
                       hipStream_t st) {
  Dims d = dims(c, n_ct);
  {
    Prof pf(c, K_LIFT, st, 2.0 * n_ct * c->n);
    HIPCHK(run_i64_lift(d, in, ext, c->tb, st));
  }
  return ntt_job_ext(c, ext, fx, n_ct * 2, 0, st);
}

// One squaring level on the ciphertexts in ext.  In a chain of squarings
// (with the split inverse) each level but the last also lifts its result
// for the next (lift_out), which then skips its own lift (lifted).
static int square_level(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st,
                        bool lifted = false, bool lift_out = false,
                        int64_t* finish_out = nullptr, const WaveTab* finish_tab = nullptr) {
  const bool chain = split_inverse(c);
  int rc = prepare_operand(c, w.ext, w.fx, n_ct, st, lifted && chain);
  if (rc) return rc;
  rc = tensor_scale(c, w, nullptr, n_ct, st);
  if (rc) return rc;
  return relin(c, w, n_ct, st, nullptr, nullptr, lift_out && chain,
               chain ? finish_out : nullptr, nullptr, false, chain ? finish_tab : nullptr);
}

static int check_ctx(const nshe_ctx* c) {
  if (!c) return fail(NSHE_EINVAL, "context is null");
  return NSHE_OK;
}

static int check_key(const nshe_ctx* c) {
  if (!c->has_key) return fail(NSHE_ENOKEY, "relinearization key not set");
  return NSHE_OK;
}

static int set_device(const nshe_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return NSHE_OK;
}

}  // namespace nshe

// ---------------------------------------------------------- parameters

// The checks every parameter set must pass (shared by nshe_ctx_create and
// nshe_budget_of); fills q (the data primes).
static int check_params(const nshe_params* pr, std::vector<u64>* q_out) {
  if (!pr) return fail(NSHE_EINVAL, "null argument");
  if (pr->log2_n < NSHE_MIN_LOG2N || pr->log2_n > NSHE_MAX_LOG2N)
    return fail(NSHE_EINVAL, "log2_n out of range");
  if (pr->L < 1 || pr->L > NSHE_MAX_L) return fail(NSHE_EINVAL, "L out of range");
  {
    // the base-conversion kernels are instantiated for these prime counts
    static const int kSupportedL[] = {2, 3, 4, 8, 12, 15, 16, 17, 20, 24};
    bool ok = false;
    for (int v : kSupportedL) ok = ok || v == pr->L;
    if (!ok) return fail(NSHE_EINVAL, "L must be one of 2, 3, 4, 8, 12, 15, 16, 17, 20, 24");
  }
  if (!pr->q_host) return fail(NSHE_EINVAL, "q_host is null");
  if (pr->t < 3 || (pr->t & 1) == 0 || pr->t >= (1u << 24))
    return fail(NSHE_EINVAL, "t must be odd, 3 <= t < 2^24");
  const int alpha = pr->alpha == 0 ? 1 : pr->alpha;
  if (alpha < 1 || alpha > 3) return fail(NSHE_EINVAL, "alpha must be 1, 2 or 3");
  if (alpha == 2 && pr->L != 2 && pr->L != 4 && pr->L != 8 && pr->L != 16)
    return fail(NSHE_EINVAL, "with alpha = 2, L must be one of 2, 4, 8, 16");
  if (alpha == 3 && pr->L != 3 && pr->L != 12 && pr->L != 15)
    return fail(NSHE_EINVAL, "with alpha = 3, L must be one of 3, 12, 15");
  const int n = 1 << pr->log2_n;
  const u64 lo = 1ull << 48, hi = 1ull << 49;
  std::vector<u64> q(pr->q_host, pr->q_host + pr->L);
  std::vector<u64> qp = q;
  qp.push_back(pr->P);
  if (alpha >= 2) qp.push_back(pr->P1);
  if (alpha >= 3) qp.push_back(pr->P2);
  for (size_t i = 0; i < qp.size(); ++i) {
    const u64 x = qp[i];
    if (x < lo || x >= hi) return fail(NSHE_EINVAL, "every prime must lie in [2^48, 2^49)");
    if ((x - 1) % (2ull * n)) return fail(NSHE_EINVAL, "every prime must be 1 mod 2N");
    if (!is_prime(x)) return fail(NSHE_EINVAL, "modulus is not prime");
    if (x % pr->t == 0) return fail(NSHE_EINVAL, "t shares a factor with a prime");
    for (size_t k = 0; k < i; ++k)
      if (qp[k] == x) return fail(NSHE_EINVAL, "primes must be distinct");
  }
  *q_out = q;
  return NSHE_OK;
}

// Multiplicative depth of the comparison program (fresh z): levels[a] =
// z^(2^a) has depth a; babies and giants are products of earlier ones
// (as the program builds them); G_j = sum_i c_i B_i keeps the largest baby
// depth, g = G_0 + sum_j G_j W_j one product more, LT = max(K, depth(g) + 1).
static int lt_program_depth(int K, int k, int m) {
  auto split = [](int i) {
    int h = 1;
    while (h * 2 <= i) h *= 2;
    return h;
  };
  auto lg = [](int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
  };
  std::vector<int> bd(k, 0), gd(m, 0);
  if (k > 1) bd[1] = 1;
  for (int i = 2; i < k; ++i) {
    const int h = split(i), r = i - h;
    bd[i] = r == 0 ? lg(h) + 1 : std::max(bd[h], bd[r]) + 1;
  }
  if (m > 1) gd[1] = lg(k) + 1;
  for (int j = 2; j < m; ++j) {
    const int h = split(j), r = j - h;
    gd[j] = r == 0 ? lg(k) + lg(h) + 1 : std::max(gd[h], gd[r]) + 1;
  }
  const int dG = *std::max_element(bd.begin(), bd.end());
  int dg = dG;
  for (int j = 1; j < m; ++j) dg = std::max(dg, std::max(dG, gd[j]) + 1);
  return std::max(K, dg + 1);
}

// Noise budget of a parameter set, in bits of the invariant noise (the
// decryption error is below 1/2 while log2(Q / (2 |t c(s) - Q m|)) > 0;
// Sec. 2.1.2: every multiplication adds and amplifies noise).
//   fresh: a fresh encryption's error t e - [Q]_t m has |.| <= t (B + t),
//     B = 19 the error bound of the client's sampler (rounded Gaussian,
//     sigma 3.2, clipped at 6 sigma), so fresh = log2 Q - log2(2 t (B + t));
//   per multiplication with relinearization: the average-case (canonical
//     embedding) growth of a BFV product with a ternary secret is a factor
//     of about t N sqrt(8/3) on the larger operand noise; counted here as
//     log2 t + log2 N + 2 bits, one bit more, so that the model stays below
//     the exact noise the oracle measures (19-28 bits per squaring for
//     N = 64 .. 4096 at t = 65537, against 22-30 here);
//   the depth budget keeps MARGIN_BITS to spare after its last level.
constexpr double kErrBound = 19.0;
constexpr double kMarginBits = 8.0;

static nshe_budget budget_of(int log2n, u64 t, const std::vector<u64>& q) {
  double log2Q = 0.0;
  for (u64 x : q) log2Q += std::log2((double)x);
  const double td = (double)t;
  nshe_budget b{};
  b.fresh_bits = log2Q - std::log2(2.0 * td * (kErrBound + td));
  b.level_bits = std::log2(td) + log2n + 2.0;
  const double d = std::floor((b.fresh_bits - kMarginBits) / b.level_bits);
  b.depth_budget = d > 0 ? (int32_t)d : 0;
  b.lt_depth = -1;
  int K = 0;
  while ((1ull << K) + 1 < t) ++K;
  if ((1ull << K) + 1 == t && K >= 2 && is_prime(t)) {
    const int kb = K / 2;
    b.lt_depth = lt_program_depth(K, 1 << kb, 1 << (K - 1 - kb));
  }
  return b;
}

// Depth an operation adds to fresh inputs (the per-operator depths of
// Table table:noise_levels for this library's programs); -1 if the
// operation does not exist for these parameters.
//   LT/LE: the program depth plus one level for its scalar combination
//   (coefficients up to (p-1)/2 summed over k babies); BETWEEN one more;
//   IN: EQ plus one level for the k-way sum when k > 1 (the paper's
//   ceil(log(k)/p)); JOIN: EQ and one product, plus one level for the
//   plaintext product of Extract inside Broadcast.
static int op_depth(const nshe_ctx* c, int op, int arg) {
  switch (op) {
    case NSHE_OP_ADD: return 0;
    case NSHE_OP_MUL: return 1;
    case NSHE_OP_MUL_PLAIN: return 1;
    case NSHE_OP_EQ: return c->squarings;
    case NSHE_OP_IN: return c->squarings < 0 ? -1 : c->squarings + (arg > 1 ? 1 : 0);
    case NSHE_OP_LT: return c->lt_K ? c->lt_depth + 1 : -1;
    case NSHE_OP_BETWEEN: return c->lt_K ? c->lt_depth + 2 : -1;
    case NSHE_OP_JOIN: return c->squarings < 0 ? -1 : c->squarings + 2;
    default: return -1;
  }
}

// NSHE_EDEPTH when an operation on fresh inputs needs more levels than the
// context's budget.
static int depth_check(const nshe_ctx* c, int op, int arg, const char* what) {
  const int d = op_depth(c, op, arg);
  if (d > c->depth_budget)
    return fail(NSHE_EDEPTH, std::string(what) + " needs multiplicative depth " +
                                 std::to_string(d) + ", the parameters allow " +
                                 std::to_string(c->depth_budget));
  return NSHE_OK;
}

// Debug switch NSHE_DEBUG_CHECK_INPUTS: every residue of the listed int64
// polynomials ([polys][L][N]) must lie in [0, q_i); waits for the stream.
struct InSpan {
  const int64_t* p;
  size_t polys;
};

static int check_inputs(nshe_ctx* c, hipStream_t st, std::initializer_list<InSpan> ins) {
  if (!(c->debug & NSHE_DEBUG_CHECK_INPUTS)) return NSHE_OK;
  HIPCHK(run_fill_u64(c->tb.bad_input, 1, 0, st));
  for (const InSpan& a : ins)
    if (a.p) HIPCHK(run_check_residues(c->n, c->L, a.polys, a.p, c->tb, st));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->tb.bad_input, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return fail(NSHE_EINVAL, "an input residue lies outside [0, q_i)");
  return NSHE_OK;
}

// ------------------------------------------------- no-allocation scratch

// The scratch of nshe_eq_mask_noalloc: one ciphertext's workspace at the
// paper's size (N = 2^15, 17 primes: 153.9 MB) fits.  Each GPU the library
// runs on holds its own copy until the process ends.  In host code the name
// stands for the array only as a symbol: kernels get the device address
// that hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kScratchBytes = NSHE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device -> address of its copy

// This device's copy (`device` must be current), looked up once per device.
static int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NSHE_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(device, p).first;
  }
  *out = it->second;
  return NSHE_OK;
}

// =================================================================== ABI

extern "C" {

static void drop_graphs(nshe_ctx* c);

const char* nshe_last_error(void) { return g_err.c_str(); }

int nshe_ctx_create(const nshe_params* pr, int hip_device, nshe_ctx** out) {
  g_err.clear();
  if (!pr || !out) return fail(NSHE_EINVAL, "null argument");
  *out = nullptr;
  std::vector<u64> q;
  if (int rc0 = check_params(pr, &q)) return rc0;
  const int n = 1 << pr->log2_n;
  const u64 lo = 1ull << 48;
  const int alpha = pr->alpha == 0 ? 1 : pr->alpha;
  std::vector<u64> sp{pr->P};
  if (alpha >= 2) sp.push_back(pr->P1);
  if (alpha >= 3) sp.push_back(pr->P2);
  std::vector<u64> qp = q;
  qp.insert(qp.end(), sp.begin(), sp.end());
  // --- extension basis: L + 1 largest primes = 1 mod 2^16 below every q_i and P_k
  const int L = pr->L, LB = L + 1;
  u64 mn = *std::min_element(qp.begin(), qp.end());
  std::vector<u64> b;
  for (u64 k = (mn - 2) >> 16; (int)b.size() < LB && k > 0; --k) {
    u64 c = (k << 16) + 1;
    if (c >= mn || c < lo) continue;
    if (is_prime(c)) b.push_back(c);
  }
  if ((int)b.size() < LB) return fail(NSHE_EINVAL, "no room for the extension basis");
  double bits_q = 0, bits_b = 0;
  for (u64 x : q) bits_q += std::log2((double)x);
  for (u64 x : b) bits_b += std::log2((double)x);
  if (bits_b < bits_q + std::log2((double)pr->t) + pr->log2_n + 6)
    return fail(NSHE_EINVAL, "extension basis too small for exact products");

  nshe_ctx* c = new (std::nothrow) nshe_ctx();
  if (!c) return fail(NSHE_ENOMEM, "host allocation failed");
  c->device = hip_device;
  c->log2n = pr->log2_n;
  c->n = n;
  c->L = L;
  c->LB = LB;
  c->alpha = alpha;
  c->dnum = L / alpha;
  c->K = 2 * L + 1 + alpha;
  c->t = pr->t;
  {
    u64 e = pr->t - 1;
    int k = 0;
    while ((e & 1) == 0) {
      e >>= 1;
      ++k;
    }
    c->squarings = e == 1 ? k : -1;
  }
  c->primes = q;
  c->primes.insert(c->primes.end(), b.begin(), b.end());
  c->primes.insert(c->primes.end(), sp.begin(), sp.end());
  c->rounds = ntt_rounds(c->log2n, &c->loge, &c->r0);
  c->tw_len = 1 << c->loge;   // round 0's row
  const int K = c->K;
  const std::vector<u64>& P_ = c->primes;
  auto prime = [&](int i) { return P_[i]; };

  // --- host tables
  std::vector<double> h_p(K), h_pinv(K), h_ninv(K);
  for (int i = 0; i < K; ++i) {
    h_p[i] = (double)prime(i);
    h_pinv[i] = 1.0 / (double)prime(i);
    h_ninv[i] = bal(invmod((u64)n, prime(i)), prime(i));
  }
  std::vector<double> tw_f((size_t)K * c->tw_len, 0.0), tw_i((size_t)K * c->tw_len, 0.0);
  // Compact rows of rounds r >= 1: row u of round r holds, at slot k, the
  // first twiddle of the round's stage k, psi^brv(2^(s_r + k) + (u << k));
  // a round's 8 x 2^s_r entries are stored slot-major (slot k of row u at
  // k 2^s_r + u, so a wave's load of one slot is contiguous), rounds one
  // after the other (the device's layout).
  auto cmp_len_of = [](int rounds, int r0, int loge) {
    int len = 0;
    for (int r = 1; r < rounds; ++r) len += (1 << (r0 + (r - 1) * loge)) * 8;
    return len;
  };
  const int cmp_len = cmp_len_of(c->rounds, c->r0, c->loge);
  // N = 2^15: the two half-limb forward sub-transforms (2^14 points each,
  // the shape of the 2^14 transform, the full transform's twiddles)
  int h_loge = 0, h_r0 = 0, h_rounds = 0;
  if (c->log2n == 15) h_rounds = ntt_rounds(14, &h_loge, &h_r0);
  const int h_len = h_rounds ? 1 << h_loge : 0;
  const int cmp_h_len = h_rounds ? cmp_len_of(h_rounds, h_r0, h_loge) : 0;
  std::vector<double> tw_h((size_t)K * 2 * std::max(h_len, 1), 0.0), tw_h0(K, 0.0),
      tw_hi((size_t)K * 2 * std::max(h_len, 1), 0.0), tw_r1f((size_t)K * 2 * 512, 0.0),
      tw_r1i((size_t)K * 2 * 512, 0.0);
  std::vector<double> tw_cf((size_t)K * std::max(cmp_len, 1), 0.0),
      tw_ci((size_t)K * std::max(cmp_len, 1), 0.0),
      tw_ch((size_t)K * 2 * std::max(cmp_h_len, 1), 0.0),
      tw_chi((size_t)K * 2 * std::max(cmp_h_len, 1), 0.0), tw_kf((size_t)K * 32, 0.0),
      tw_ki((size_t)K * 32, 0.0);
  // N = 2^15: the parity sub-transforms' compact rows and round-1 rows, and
  // the last-stage twiddles of the key-switching basis (see Tables)
  const int KSn = L + alpha;
  std::vector<double> tw_cp((size_t)K * std::max(cmp_h_len, 1), 0.0),
      tw_r1p((size_t)K * 512, 0.0), tw_last(h_rounds ? (size_t)KSn * (n / 2) : 1, 0.0);
  // the inverse's last-stage twiddle of each prime (slot 1 of its round-0 row)
  std::vector<u64> w_last(K, 1);
  {
    std::vector<u64> pbr(n), pibr(n);
    for (int k = 0; k < K; ++k) {
      const u64 p = prime(k);
      const u64 psi = powmod(primitive_root(p), (p - 1) / (2ull * n), p);
      const u64 psi_inv = invmod(psi, p);
      std::vector<u64> pw(n), pwi(n);
      pw[0] = pwi[0] = 1;
      for (int i = 1; i < n; ++i) {
        pw[i] = mulmod(pw[i - 1], psi, p);
        pwi[i] = mulmod(pwi[i - 1], psi_inv, p);
      }
      for (int i = 0; i < n; ++i) {
        pbr[i] = pw[brv(i, c->log2n)];
        pibr[i] = pwi[brv(i, c->log2n)];
      }
      w_last[k] = pibr[1];
      // per-(stage, slot) constants omega_k^(+-brv_k(j)), omega_k = psi^(N/2^k)
      for (int kk = 1; kk < c->loge && kk < 5; ++kk) {
        const u64 om = powmod(psi, (u64)n >> kk, p), omi = invmod(om, p);
        for (int j = 1; j < (1 << kk); ++j) {
          tw_kf[(size_t)k * 32 + (1 << kk) + j] = bal(powmod(om, (u64)brv(j, kk), p), p);
          tw_ki[(size_t)k * 32 + (1 << kk) + j] = bal(powmod(omi, (u64)brv(j, kk), p), p);
        }
      }
      // round 0 (uniform) and the compact rows of the full transform
      for (int kk = 0; kk < c->r0; ++kk)
        for (int j = 0; j < (1 << kk); ++j) {
          tw_f[(size_t)k * c->tw_len + (1 << kk) + j] = bal(pbr[(1 << kk) + j], p);
          tw_i[(size_t)k * c->tw_len + (1 << kk) + j] = bal(pibr[(1 << kk) + j], p);
        }
      {
        size_t off = (size_t)k * cmp_len;
        for (int r = 1; r < c->rounds; ++r) {
          const int ss = c->r0 + (r - 1) * c->loge;
          for (int u = 0; u < (1 << ss); ++u)
            for (int kk = 0; kk < c->loge; ++kk) {
              const int idx = (1 << (ss + kk)) + (u << kk);
              tw_cf[off + ((size_t)kk << ss) + u] = bal(pbr[idx], p);
              tw_ci[off + ((size_t)kk << ss) + u] = bal(pibr[idx], p);
            }
          off += (size_t)8 << ss;
        }
      }
      // half-limb sub-transforms: sub-stage s' of half h is the full
      // transform's stage s' + 1 over the indices with top bit h
      if (h_rounds) {
        tw_h0[k] = bal(pbr[1], p);
        for (int hh = 0; hh < 2; ++hh) {
          for (int kk = 0; kk < h_r0; ++kk)
            for (int j = 0; j < (1 << kk); ++j) {
              tw_h[((size_t)k * 2 + hh) * h_len + (1 << kk) + j] =
                  bal(pbr[(1 << kk) * (2 + hh) + j], p);
              tw_hi[((size_t)k * 2 + hh) * h_len + (1 << kk) + j] =
                  bal(pibr[(1 << kk) * (2 + hh) + j], p);
            }
          // round 1 in full (16 rows x 32 slots), for the LDS copy
          {
            const int ss = h_r0;
            for (int u = 0; u < (1 << ss) && (1 << ss) * 32 == 512; ++u)
              for (int kk = 0; kk < h_loge; ++kk)
                for (int j = 0; j < (1 << kk); ++j) {
                  const int idx = (1 << (ss + kk)) * (2 + hh) + (u << kk) + j;
                  const size_t o = ((size_t)k * 2 + hh) * 512 + (size_t)u * 32 + (1 << kk) + j;
                  tw_r1f[o] = bal(pbr[idx], p);
                  tw_r1i[o] = bal(pibr[idx], p);
                }
          }
          size_t off = ((size_t)k * 2 + hh) * cmp_h_len;
          for (int r = 1; r < h_rounds; ++r) {
            const int ss = h_r0 + (r - 1) * h_loge;
            for (int u = 0; u < (1 << ss); ++u)
              for (int kk = 0; kk < h_loge; ++kk) {
                const int idx = (1 << (ss + kk)) * (2 + hh) + (u << kk);
                tw_ch[off + ((size_t)kk << ss) + u] = bal(pbr[idx], p);
                tw_chi[off + ((size_t)kk << ss) + u] = bal(pibr[idx], p);
              }
            off += (size_t)8 << ss;
          }
        }
        // parity sub-transforms: sub-stage s is the full transform's stage s
        // (slot 2^s + m), for either parity
        for (int u = 0; u < (1 << h_r0) && (1 << h_r0) * 32 == 512; ++u)
          for (int kk = 0; kk < h_loge; ++kk)
            for (int j = 0; j < (1 << kk); ++j)
              tw_r1p[(size_t)k * 512 + (size_t)u * 32 + (1 << kk) + j] =
                  bal(pbr[(1 << (h_r0 + kk)) + (u << kk) + j], p);
        size_t off = (size_t)k * cmp_h_len;
        for (int r = 1; r < h_rounds; ++r) {
          const int ss = h_r0 + (r - 1) * h_loge;
          for (int u = 0; u < (1 << ss); ++u)
            for (int kk = 0; kk < h_loge; ++kk)
              tw_cp[off + ((size_t)kk << ss) + u] = bal(pbr[(1 << (ss + kk)) + (u << kk)], p);
          off += (size_t)8 << ss;
        }
        // last stage, pairing standard indices 2k and 2k + 1: psi^brv(2^14 + k)
        // for k = 16 m + u at u 1024 + m
        const int ks = k < L ? k : (k > 2 * L ? L + (k - 2 * L - 1) : -1);
        if (ks >= 0 && n == (1 << 15))
          for (int u = 0; u < 16; ++u)
            for (int m = 0; m < 1024; ++m)
              tw_last[(size_t)ks * (n / 2) + (size_t)u * 1024 + m] =
                  bal(pbr[(n / 2) + 16 * m + u], p);
      }
    }
  }
  std::vector<u64> qv(q), bv(b);
  // Base-conversion matrices: each entry M (balanced mod m) split as M =
  // c1 2^24 + c0 (|c1| <= 2^24, |c0| <= 2^23) for exact FMA accumulation.
  auto split = [](double* d, u64 M, u64 m) {
    const double cb = bal(M, m);
    const double c1v = std::nearbyint(cb * 0x1p-24);
    d[0] = c1v;
    d[1] = cb - c1v * 0x1p24;
  };
  std::vector<double> q_hat_b_sp((size_t)LB * L * 2), c2_sp((size_t)LB * L * 2),
      b_hat_q_sp((size_t)L * LB * 2), two24(K), two48(K);
  for (int i = 0; i < K; ++i) {
    const u64 m = prime(i), t24 = (1ull << 24) % m;
    two24[i] = bal(t24, m);
    two48[i] = bal(mulmod(t24, t24, m), m);
  }
  // t_qhinv, t_q, c1: a second row times the inverse's last-stage twiddle
  std::vector<double> q_hat_inv(L), Q_b(LB), t_qhinv(2 * L), t_q(2 * L),
      c1(2 * LB), b_hat_inv(LB), B_q(L), P_inv_q(L), NP_inv_q(2 * L), ninv_P(2 * alpha),
      mr_q((size_t)std::max(alpha - 1, 1) * L, 0.0), delta_q(L), mrc_inv((size_t)L * L, 0.0),
      mrc_half(L), dig_c((size_t)(L / alpha) * (L + alpha) * std::max(alpha - 1, 1), 0.0);
  for (int k = 0; k < alpha; ++k) {
    const u64 Pp = sp[k], nP = invmod((u64)n % Pp, Pp);
    ninv_P[2 * k] = bal(nP, Pp);
    ninv_P[2 * k + 1] = bal(mulmod(nP, w_last[2 * L + 1 + k], Pp), Pp);
  }
  // alpha primes per digit: the special primes' Garner inverses
  // [P_0^-1]_{P_1}, [P_0^-1]_{P_2}, [P_1^-1]_{P_2}, and the mixed-radix
  // weights of digit j (first prime g = j alpha) modulo every prime of the
  // key-switching basis: [q_g]_{p_i}, [q_g q_{g+1}]_{p_i}
  double p_inv_p[3] = {0.0, 0.0, 0.0};
  if (alpha >= 2) p_inv_p[0] = bal(invmod(sp[0] % sp[1], sp[1]), sp[1]);
  if (alpha >= 3) {
    p_inv_p[1] = bal(invmod(sp[0] % sp[2], sp[2]), sp[2]);
    p_inv_p[2] = bal(invmod(sp[1] % sp[2], sp[2]), sp[2]);
  }
  if (alpha >= 2) {
    for (int j = 0; j < L / alpha; ++j)
      for (int i = 0; i < L + alpha; ++i) {
        const u64 m = i < L ? q[i] : sp[i - L];
        u64 w = 1;
        for (int k = 0; k + 1 < alpha; ++k) {
          w = mulmod(w, q[j * alpha + k] % m, m);
          dig_c[((size_t)j * (L + alpha) + i) * (alpha - 1) + k] = bal(w, m);
        }
      }
  }
  u64 Qmodt = 1;
  for (u64 x : qv) Qmodt = mulmod(Qmodt, x % c->t, c->t);
  for (int i = 0; i < L; ++i) {
    const u64 qi = qv[i];
    const u64 qhi = invmod(prod_mod(qv, i, qi), qi);
    q_hat_inv[i] = bal(qhi, qi);
    // inverse transforms return N times the coefficients: fold N^-1 here
    const u64 ninv_q = invmod((u64)n % qi, qi);
    const u64 tqh = mulmod(mulmod(c->t % qi, qhi, qi), ninv_q, qi), tq = mulmod(c->t % qi, ninv_q, qi);
    t_qhinv[i] = bal(tqh, qi);
    t_q[i] = bal(tq, qi);
    t_qhinv[L + i] = bal(mulmod(tqh, w_last[i], qi), qi);
    t_q[L + i] = bal(mulmod(tq, w_last[i], qi), qi);
    B_q[i] = bal(prod_mod(bv, -1, qi), qi);
    // P^-1 with P the product of the special primes
    u64 Pq = 1;
    for (u64 x : sp) Pq = mulmod(Pq, x % qi, qi);
    P_inv_q[i] = bal(invmod(Pq, qi), qi);
    // [(P_0 ... P_{k-1}) P^-1]_{q_i} for k = 1..alpha-1
    {
      u64 pre = 1;
      for (int k = 1; k < alpha; ++k) {
        pre = mulmod(pre, sp[k - 1] % qi, qi);
        mr_q[(size_t)(k - 1) * L + i] = bal(mulmod(pre, invmod(Pq, qi), qi), qi);
      }
    }
    const u64 npq = mulmod(invmod(Pq, qi), ninv_q, qi);
    NP_inv_q[i] = bal(npq, qi);
    NP_inv_q[L + i] = bal(mulmod(npq, w_last[i], qi), qi);
    // Delta = (Q - (Q mod t)) / t = -(Q mod t) * t^-1 (mod q_i)
    delta_q[i] = bal((qi - mulmod(Qmodt, invmod(c->t % qi, qi), qi)) % qi, qi);
    for (int k = 0; k < LB; ++k) split(&b_hat_q_sp[((size_t)i * LB + k) * 2], prod_mod(bv, k, qi), qi);
    for (int j = 0; j < i; ++j) mrc_inv[(size_t)j * L + i] = bal(invmod(qv[j] % qi, qi), qi);
  }
  for (int k = 0; k < LB; ++k) {
    const u64 bk = bv[k];
    const u64 Qb = prod_mod(qv, -1, bk);
    Q_b[k] = bal(Qb, bk);
    const u64 bhi = invmod(prod_mod(bv, k, bk), bk);
    b_hat_inv[k] = bal(bhi, bk);
    const u64 c1k = mulmod(mulmod(mulmod(c->t % bk, invmod(Qb, bk), bk), bhi, bk),
                           invmod((u64)n % bk, bk), bk);
    c1[k] = bal(c1k, bk);
    c1[LB + k] = bal(mulmod(c1k, w_last[L + k], bk), bk);
    for (int i = 0; i < L; ++i) {
      split(&q_hat_b_sp[((size_t)k * L + i) * 2], prod_mod(qv, i, bk), bk);
      split(&c2_sp[((size_t)k * L + i) * 2], mulmod(invmod(qv[i] % bk, bk), bhi, bk), bk);
    }
  }
  // mixed-radix digits of (Q-1)/2, whose residue mod q_i is (q_i - 1)/2
  {
    std::vector<u64> a(L);
    for (int i = 0; i < L; ++i) {
      const u64 qi = qv[i];
      u64 tv = (qi - 1) / 2;
      for (int j = 0; j < i; ++j) {
        const u64 diff = (tv + qi - a[j] % qi) % qi;
        tv = mulmod(diff, invmod(qv[j] % qi, qi), qi);
      }
      a[i] = tv;
      mrc_half[i] = (double)tv;
    }
  }
  // --- upload
  std::vector<std::pair<const std::vector<double>*, const double**>> parts = {
      {&h_p, &c->tb.p},           {&h_pinv, &c->tb.pinv},     {&h_pinv, &c->tb.recip},
      {&h_ninv, &c->tb.ninv},     {&tw_f, &c->tb.tw_fwd},     {&tw_i, &c->tb.tw_inv},
      {&q_hat_inv, &c->tb.q_hat_inv}, {&Q_b, &c->tb.Q_b},
      {&t_qhinv, &c->tb.t_qhinv}, {&t_q, &c->tb.t_q},         {&c1, &c->tb.c1},
      {&b_hat_inv, &c->tb.b_hat_inv},
      {&B_q, &c->tb.B_q},         {&P_inv_q, &c->tb.P_inv_q}, {&NP_inv_q, &c->tb.NP_inv_q},
      {&ninv_P, &c->tb.ninv_P},   {&mr_q, &c->tb.mr_q},       {&dig_c, &c->tb.dig_c},
      {&delta_q, &c->tb.delta_q},
      {&mrc_inv, &c->tb.mrc_inv}, {&mrc_half, &c->tb.mrc_half}, {&tw_h, &c->tb.tw_half},
      {&tw_h0, &c->tb.tw_half0},  {&tw_cf, &c->tb.tw_cmp_f},  {&tw_ci, &c->tb.tw_cmp_i},
      {&tw_ch, &c->tb.tw_cmp_h},  {&tw_kf, &c->tb.tw_cst_f},  {&tw_ki, &c->tb.tw_cst_i},
      {&q_hat_b_sp, &c->tb.q_hat_b_sp}, {&c2_sp, &c->tb.c2_sp}, {&b_hat_q_sp, &c->tb.b_hat_q_sp},
      {&two24, &c->tb.two24},     {&two48, &c->tb.two48},
      {&tw_hi, &c->tb.tw_half_inv}, {&tw_chi, &c->tb.tw_cmp_hi},
      {&tw_r1f, &c->tb.tw_r1_f},  {&tw_r1i, &c->tb.tw_r1_i},
      {&tw_cp, &c->tb.tw_cmp_par}, {&tw_r1p, &c->tb.tw_r1_par}, {&tw_last, &c->tb.tw_last}};
  size_t total = 0;
  std::vector<size_t> offs;
  for (auto& pp : parts) {
    offs.push_back(total);
    total += (pp.first->size() * sizeof(double) + 255) & ~size_t(255);
  }
  const size_t off_counters = total;
  total += 256;
  const size_t off_lp = total;
  total += ((size_t)(W_of(c) + L + alpha) * sizeof(int) + 255) & ~size_t(255);
  // comparison polynomial for a Fermat prime t
  std::vector<double> lt_coef;
  if (c->squarings >= 2 && is_prime(c->t)) {
    const int K = c->squarings, kb = K / 2;
    c->lt_K = K;
    c->lt_k = 1 << kb;
    c->lt_m = 1 << (K - 1 - kb);
    const std::vector<u64> cp = comparison_poly(c->t);
    lt_coef.resize((size_t)c->lt_m * c->lt_k);
    for (int j = 0; j < c->lt_m; ++j)
      for (int i = 0; i < c->lt_k; ++i)
        lt_coef[(size_t)j * c->lt_k + i] = centred_small(cp[2 * ((size_t)j * c->lt_k + i) + 1], c->t);
    c->lt_top = centred_small(cp[c->t - 1], c->t);
    lt_coef.push_back(c->lt_top);  // the z^(p-1) coefficient, after the matrix
    c->lt_depth = lt_program_depth(c->lt_K, c->lt_k, c->lt_m);
  }
  {
    const nshe_budget bud = budget_of(c->log2n, c->t, q);
    c->depth_budget = bud.depth_budget;
    c->fresh_bits = bud.fresh_bits;
    c->level_bits = bud.level_bits;
  }
  const size_t off_lt = total;
  total += (lt_coef.size() * sizeof(double) + 255) & ~size_t(255);
  int rc = NSHE_OK;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipMalloc(&c->dev_tables, total);
  if (e != hipSuccess) {
    delete c;
    return fail(NSHE_EDEVICE, std::string("table allocation: ") + hipGetErrorString(e));
  }
  char* base = static_cast<char*>(c->dev_tables);
  for (size_t i = 0; i < parts.size() && e == hipSuccess; ++i) {
    *parts[i].second = reinterpret_cast<const double*>(base + offs[i]);
    e = hipMemcpy(base + offs[i], parts[i].first->data(), parts[i].first->size() * sizeof(double),
                  hipMemcpyHostToDevice);
  }
  c->tb.tw_len = c->tw_len;
  c->tb.tw_half_len = h_len;
  c->tb.tw_cmp_len = cmp_len;
  c->tb.tw_cmp_h_len = cmp_h_len;
  if (!h_len) {
    c->tb.tw_half = nullptr;
    c->tb.tw_half0 = nullptr;
    c->tb.tw_half_inv = nullptr;
    c->tb.tw_cmp_par = nullptr;
    c->tb.tw_r1_par = nullptr;
    c->tb.tw_last = nullptr;
  }
  // counters: [MARGIN_COUNT] u64 event counts, the input-check flag at +128
  static_assert(MARGIN_COUNT * 8 <= 128, "counter area");
  c->tb.margin = reinterpret_cast<unsigned long long*>(base + off_counters);
  c->tb.bad_input = reinterpret_cast<int*>(base + off_counters + 128);
  c->tb.lift_edge = kLiftEdge;
  c->tb.ks_alpha = alpha;
  for (int k = 0; k < 3; ++k) c->tb.p_inv_p[k] = p_inv_p[k];
  if (e == hipSuccess) e = hipMemset(base + off_counters, 0, 256);
  std::vector<int> lp;
  for (int i = 0; i < W_of(c); ++i) lp.push_back(i);
  for (int i = 0; i < L; ++i) lp.push_back(i);
  for (int k = 0; k < alpha; ++k) lp.push_back(2 * L + 1 + k);
  c->lp_ext = reinterpret_cast<int*>(base + off_lp);
  c->lp_ks = c->lp_ext + W_of(c);
  if (e == hipSuccess)
    e = hipMemcpy(c->lp_ext, lp.data(), lp.size() * sizeof(int), hipMemcpyHostToDevice);
  if (!lt_coef.empty()) {
    c->lt_coef = reinterpret_cast<const double*>(base + off_lt);
    if (e == hipSuccess)
      e = hipMemcpy(base + off_lt, lt_coef.data(), lt_coef.size() * sizeof(double),
                    hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipFree(c->dev_tables);
    delete c;
    return fail(NSHE_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
  }
  if ((rc = scratch_address(hip_device, &c->scratch))) {
    (void)hipFree(c->dev_tables);
    delete c;
    return rc;
  }
  *out = c;
  return rc;
}

int nshe_ctx_destroy(nshe_ctx* c) {
  if (!c) return NSHE_OK;
  (void)hipSetDevice(c->device);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto& e : c->pool) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->half_stream) (void)hipStreamDestroy(c->half_stream);
  if (c->half_fork) (void)hipEventDestroy(c->half_fork);
  if (c->half_join) (void)hipEventDestroy(c->half_join);
  if (c->evk) (void)hipFree(c->evk);
  for (auto& kv : c->galois) (void)hipFree(kv.second);
  if (c->dev_tables) (void)hipFree(c->dev_tables);
  delete c;
  return NSHE_OK;
}

int nshe_ctx_info(const nshe_ctx* c, nshe_info* out) {
  if (check_ctx(c) || !out) return fail(NSHE_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->n = (uint32_t)c->n;
  out->L = c->L;
  out->L_ext = c->LB;
  out->squarings = c->squarings;
  for (int k = 0; k < c->LB && k < 32; ++k) out->ext_primes[k] = c->primes[c->L + k];
  out->ct_words = (size_t)2 * c->L * c->n;
  out->relin_key_words = (size_t)c->dnum * 2 * KS_of(c) * c->n;
  out->alpha = c->alpha;
  out->dnum = c->dnum;
  out->depth_budget = c->depth_budget;
  out->fresh_bits = c->fresh_bits;
  out->level_bits = c->level_bits;
  out->lt_depth = c->lt_K ? c->lt_depth : -1;
  return NSHE_OK;
}

int nshe_budget_of(const nshe_params* pr, nshe_budget* out) {
  g_err.clear();
  if (!pr || !out) return fail(NSHE_EINVAL, "null argument");
  std::vector<u64> q;
  if (int rc = check_params(pr, &q)) return rc;
  *out = budget_of((int)pr->log2_n, pr->t, q);
  return NSHE_OK;
}

int nshe_op_depth(const nshe_ctx* c, int op, int arg, int* depth) {
  g_err.clear();
  if (check_ctx(c) || !depth) return fail(NSHE_EINVAL, "null argument");
  if (op < NSHE_OP_ADD || op > NSHE_OP_JOIN) return fail(NSHE_EINVAL, "unknown operation");
  const int d = op_depth(c, op, arg);
  if (d < 0) return fail(NSHE_EUNSUPPORTED, "operation not available for these parameters");
  *depth = d;
  return NSHE_OK;
}

int nshe_depth_after(const nshe_ctx* c, int op, int arg, int in_depth, int* out_depth) {
  int d = 0;
  if (int rc = nshe_op_depth(c, op, arg, &d)) return rc;
  if (in_depth < 0) return fail(NSHE_EINVAL, "in_depth < 0");
  *out_depth = in_depth + d;
  if (in_depth + d > c->depth_budget)
    return fail(NSHE_EDEPTH, "depth " + std::to_string(in_depth + d) + " exceeds the budget " +
                                 std::to_string(c->depth_budget));
  return NSHE_OK;
}

int nshe_set_debug(nshe_ctx* c, uint32_t flags) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (flags & ~(uint32_t)(NSHE_DEBUG_WIDE_LIFT_WINDOW | NSHE_DEBUG_CHECK_INPUTS))
    return fail(NSHE_EINVAL, "unknown debug flag");
  c->debug = flags;
  c->tb.lift_edge = (flags & NSHE_DEBUG_WIDE_LIFT_WINDOW) ? kLiftEdgeWide : kLiftEdge;
  drop_graphs(c);  // captured kernels hold the tables by value
  return NSHE_OK;
}

size_t nshe_workspace_bytes(const nshe_ctx* c, int n_ct) {
  if (!c || n_ct <= 0) return 0;
  return ws_doubles(c, n_ct) * sizeof(double);
}

// Convert a switching key (int64 [dnum][2][L+alpha][N], coefficient
// domain) into *dst (NTT domain, allocated on first use); waits for the
// stream.
static int load_switch_key(nshe_ctx* c, const int64_t* key_dev, double** dst, hipStream_t st) {
  const size_t rows = (size_t)c->dnum * 2 * KS_of(c);
  if (!*dst) HIPCHK(hipMalloc(dst, rows * c->n * sizeof(double)));
  double* tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, rows * c->n * sizeof(double)));
  int rc = NSHE_OK;
  hipError_t e = run_i64_to_dbl_limbs(rows, c->n, key_dev, tmp, c->lp_ks, KS_of(c), c->tb, st);
  if (e != hipSuccess) rc = fail(NSHE_EDEVICE, std::string("key conversion: ") + hipGetErrorString(e));
  if (!rc) rc = ntt_job_ks(c, tmp, *dst, c->dnum * 2, 0, st);
  if (!rc) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(NSHE_EDEVICE, std::string("key transform: ") + hipGetErrorString(e));
  }
  (void)hipFree(tmp);
  return rc;
}

static size_t key_words(const nshe_ctx* c) {
  return (size_t)c->dnum * 2 * KS_of(c) * c->n;
}

int nshe_set_relin_key(nshe_ctx* c, const int64_t* evk_dev, size_t n_words, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (!evk_dev) return fail(NSHE_EINVAL, "evk is null");
  if (n_words != key_words(c)) return fail(NSHE_ESHAPE, "evk must hold dnum * 2 * (L+alpha) * N words");
  if (set_device(c)) return NSHE_EDEVICE;
  int rc = load_switch_key(c, evk_dev, &c->evk, static_cast<hipStream_t>(stream));
  if (rc) return rc;
  c->has_key = true;
  return NSHE_OK;
}

int nshe_set_galois_key(nshe_ctx* c, uint32_t g, const int64_t* key_dev, size_t n_words,
                        void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (!key_dev) return fail(NSHE_EINVAL, "key is null");
  if (n_words != key_words(c)) return fail(NSHE_ESHAPE, "key must hold dnum * 2 * (L+alpha) * N words");
  if (g % 2 == 0 || g >= 2u * (uint32_t)c->n) return fail(NSHE_EINVAL, "g must be odd and below 2N");
  if (set_device(c)) return NSHE_EDEVICE;
  double*& slot = c->galois[g];
  int rc = load_switch_key(c, key_dev, &slot, static_cast<hipStream_t>(stream));
  if (rc) {
    if (slot) (void)hipFree(slot);
    c->galois.erase(g);
  }
  return rc;
}

int nshe_sub(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out, int n_ct,
             void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0) return fail(NSHE_ESHAPE, "n_ct < 0");
  if (n_ct == 0) return NSHE_OK;
  if (!x || !y || !out) return fail(NSHE_EINVAL, "null buffer");
  if (set_device(c)) return NSHE_EDEVICE;
  Dims d = dims(c, n_ct);
  const size_t np = (size_t)n_ct * 2;
  if (int rc = check_inputs(c, static_cast<hipStream_t>(stream), {{x, np}, {y, np}})) return rc;
  HIPCHK(run_sub_i64(d, x, y, out, c->tb, static_cast<hipStream_t>(stream)));
  return NSHE_OK;
}

int nshe_add(nshe_ctx* c, const int64_t* a, const int64_t* b, int64_t* out, int n_ct,
             void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0) return fail(NSHE_ESHAPE, "n_ct < 0");
  if (n_ct == 0) return NSHE_OK;
  if (!a || !b || !out) return fail(NSHE_EINVAL, "null buffer");
  if (set_device(c)) return NSHE_EDEVICE;
  const size_t np = (size_t)n_ct * 2;
  if (int rc = check_inputs(c, static_cast<hipStream_t>(stream), {{a, np}, {b, np}})) return rc;
  HIPCHK(run_sum_i64(dims(c, n_ct), a, b, 0, 1, out, c->tb, static_cast<hipStream_t>(stream)));
  return NSHE_OK;
}

int nshe_sum(nshe_ctx* c, const int64_t* in, int k, int64_t* out, int n_ct, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0 || k < 0) return fail(NSHE_ESHAPE, "n_ct < 0 or k < 0");
  if (n_ct == 0) return NSHE_OK;
  if (!out || (k > 0 && !in)) return fail(NSHE_EINVAL, "null buffer");
  if (set_device(c)) return NSHE_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = check_inputs(c, st, {{in, (size_t)k * n_ct * 2}})) return rc;
  const size_t words = (size_t)n_ct * 2 * c->L * c->n;
  if (k == 0) {
    HIPCHK(run_fill_u64(out, words, 0, st));  // the encryption (0, 0)
    return NSHE_OK;
  }
  HIPCHK(run_sum_i64(dims(c, n_ct), in, in + words, words, k - 1, out, c->tb, st));
  return NSHE_OK;
}

static int common_checks(nshe_ctx* c, int n_ct, void* ws, size_t ws_bytes, bool need_key) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0) return fail(NSHE_ESHAPE, "n_ct < 0");
  if (n_ct > 0) {
    int rc = check_ws(c, ws, ws_bytes, n_ct);
    if (rc) return rc;
  }
  if (need_key && check_key(c)) return NSHE_ENOKEY;
  if (set_device(c)) return NSHE_EDEVICE;
  return NSHE_OK;
}

int nshe_square_relin(nshe_ctx* c, const int64_t* in, int64_t* out, int n_ct, void* ws,
                      size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, true);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in || !out) return fail(NSHE_EINVAL, "null buffer");
  if ((rc = depth_check(c, NSHE_OP_MUL, 0, "a multiplication"))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  rc = prepare_i64(c, in, w.ext, w.fx, n_ct, st);
  if (rc) return rc;
  rc = tensor_scale(c, w, nullptr, n_ct, st);
  if (rc) return rc;
  return relin_i64(c, w, n_ct, st, out);
}

// The second operand's transform sits in the digit region after its lift.
static double* fx_second(const nshe_ctx* c, const Ws& w, int n_ct) {
  return w.dig + (size_t)n_ct * 2 * W_of(c) * c->n;
}

static int load_two(nshe_ctx* c, const Ws& w, const int64_t* a, const int64_t* b, int n_ct,
                    hipStream_t st) {
  int rc = prepare_i64(c, a, w.ext, w.fx, n_ct, st);
  if (rc) return rc;
  return prepare_i64(c, b, w.dig, fx_second(c, w, n_ct), n_ct, st);
}

int nshe_mul_relin(nshe_ctx* c, const int64_t* a, const int64_t* b, int64_t* out, int n_ct,
                   void* ws, size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, true);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!a || !b || !out) return fail(NSHE_EINVAL, "null buffer");
  if ((rc = depth_check(c, NSHE_OP_MUL, 0, "a multiplication"))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{a, (size_t)n_ct * 2}, {b, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  rc = load_two(c, w, a, b, n_ct, st);
  if (rc) return rc;
  rc = tensor_scale(c, w, fx_second(c, w, n_ct), n_ct, st);
  if (rc) return rc;
  return relin_i64(c, w, n_ct, st, out);
}

int nshe_multiply(nshe_ctx* c, const int64_t* a, const int64_t* b, int64_t* out3, int n_ct,
                  void* ws, size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, false);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!a || !b || !out3) return fail(NSHE_EINVAL, "null buffer");
  if ((rc = depth_check(c, NSHE_OP_MUL, 0, "a multiplication"))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{a, (size_t)n_ct * 2}, {b, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  rc = load_two(c, w, a, b, n_ct, st);
  if (rc) return rc;
  rc = tensor_scale(c, w, fx_second(c, w, n_ct), n_ct, st, nullptr, true);
  if (rc) return rc;
  HIPCHK(run_polys_to_i64(d, w.dt, 3, 3 * W * N, W * N, out3, 0, c->tb, st));
  return NSHE_OK;
}

int nshe_relinearize(nshe_ctx* c, const int64_t* in3, int64_t* out, int n_ct, void* ws,
                     size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, true);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in3 || !out) return fail(NSHE_EINVAL, "null buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in3, (size_t)n_ct * 3}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_i64_to_polys(d, in3, 3, w.dt, 3 * W * N, W * N, 2, c->tb, st));
  const DigitSrc ds = digit_src(c, w);
  if (ds.split) HIPCHK(run_digit_split(d, w.dt, ds.p, ds.stride, st));
  if (c->alpha > 1) HIPCHK(run_digit_mrc(d, ds.p, ds.stride, c->tb, st));
  rc = relin(c, w, n_ct, st);
  if (rc) return rc;
  HIPCHK(run_polys_to_i64(d, w.ext, 2, 2 * W * N, W * N, out, 0, c->tb, st));
  return NSHE_OK;
}

// The EQ chain on ciphertexts already differenced into w.ext.
// finish_out (with the split inverse): the last level writes the mask to it;
// finish_tab: to a batched wave's ciphertexts, through its table.
static int eq_levels(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st,
                     bool first_lifted = false, int64_t* finish_out = nullptr,
                     const WaveTab* finish_tab = nullptr) {
  for (int k = 0; k < c->squarings; ++k) {
    const bool last = k + 1 == c->squarings;
    int rc = square_level(c, w, n_ct, st, k > 0 || first_lifted, !last,
                          last ? finish_out : nullptr, last ? finish_tab : nullptr);
    if (rc) return rc;
  }
  return NSHE_OK;
}

static int eq_run(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out, int n_ct,
                  int y_broadcast, void* ws, hipStream_t st);

// Whether st is known not to be capturing into a graph (a second stream
// joins only then).
static bool stream_idle_capture(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusNone;
}

// Whether an EQ or rotate-and-add call runs as two halves on two streams
// (tuning streams = 2):
// at least 32 ciphertexts (16 per half keep the key-switch product's key
// reads at one per 16 ciphertexts), not profiling (each launch's own time),
// not the no-allocation scratch, not while st is being captured, and only
// where the second half's share of the workspace starts 256-byte aligned.
static bool two_halves(nshe_ctx* c, int n_ct, const void* ws, hipStream_t st) {
  if (c->tune.streams != 2 || n_ct < 32 || c->prof || ws == c->scratch) return false;
  if (ws_doubles(c, n_ct / 2) * sizeof(double) % 256) return false;
  return stream_idle_capture(st);
}

// The context's second stream and its fork and join events, made on first use.
static int half_stream_ready(nshe_ctx* c) {
  if (!c->half_stream) HIPCHK(hipStreamCreateWithFlags(&c->half_stream, hipStreamNonBlocking));
  if (!c->half_fork) HIPCHK(hipEventCreateWithFlags(&c->half_fork, hipEventDisableTiming));
  if (!c->half_join) HIPCHK(hipEventCreateWithFlags(&c->half_join, hipEventDisableTiming));
  return NSHE_OK;
}

// run(first ciphertext, count, workspace share, stream) for the two halves
// of n_ct ciphertexts: the first half on st, the second on the context's
// second stream, each in its own share of the workspace (the workspace is
// linear in n_ct, so the two shares fill it).  The second stream starts
// after the work already on st, and st waits for it at the end.
static int run_two_halves(nshe_ctx* c, int n_ct, void* ws, hipStream_t st,
                          const std::function<int(int, int, void*, hipStream_t)>& run) {
  const int h = n_ct / 2;
  int rc = half_stream_ready(c);
  if (rc) return rc;
  HIPCHK(hipEventRecord(c->half_fork, st));
  HIPCHK(hipStreamWaitEvent(c->half_stream, c->half_fork, 0));
  rc = run(0, h, ws, st);
  if (!rc) rc = run(h, n_ct - h, static_cast<double*>(ws) + ws_doubles(c, h), c->half_stream);
  HIPCHK(hipEventRecord(c->half_join, c->half_stream));
  HIPCHK(hipStreamWaitEvent(st, c->half_join, 0));
  return rc;
}

static int eq_mask_impl(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out,
                        int n_ct, int y_broadcast, void* ws, size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, true);
  if (rc) return rc;
  if (c->squarings < 0) return fail(NSHE_EUNSUPPORTED, "t - 1 is not a power of two");
  if ((rc = depth_check(c, NSHE_OP_EQ, 0, "EQ"))) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!x || !y || !out) return fail(NSHE_EINVAL, "null buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{x, (size_t)n_ct * 2},
                                 {y, y_broadcast ? (size_t)2 : (size_t)n_ct * 2}})))
    return rc;
  if (two_halves(c, n_ct, ws, st)) {
    const size_t ctw = (size_t)2 * c->L * c->n;
    return run_two_halves(c, n_ct, ws, st, [&](int c0, int cnt, void* wsh, hipStream_t s) {
      return eq_run(c, x + c0 * ctw, y_broadcast ? y : y + c0 * ctw, out + c0 * ctw, cnt,
                    y_broadcast, wsh, s);
    });
  }
  return eq_run(c, x, y, out, n_ct, y_broadcast, ws, st);
}

// The EQ chain itself on n_ct ciphertexts (checked by the caller), on st.
static int eq_run(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out, int n_ct,
                  int y_broadcast, void* ws, hipStream_t st) {
  int rc = NSHE_OK;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  // with the split inverse the subtraction also lifts (the first squaring's
  // operand), like every later level's mod-down
  const bool chain = split_inverse(c);
  {
    Prof pf(c, K_SUB, st, 2.0 * n_ct * c->L * c->n);
    if (chain)
      HIPCHK(run_sub_lift(d, x, y, y_broadcast ? 1 : 0, w.ext, c->tb, st));
    else
      HIPCHK(run_sub_to_ext(d, x, y, y_broadcast ? 1 : 0, w.ext, c->tb, st));
  }
  rc = eq_levels(c, w, n_ct, st, chain, chain ? out : nullptr);
  if (rc) return rc;
  if (!chain) {
    Prof pf(c, K_CONVERT, st, 2.0 * n_ct * c->L * c->n);
    HIPCHK(run_polys_to_i64(d, w.ext, 2, 2 * W * N, W * N, out, 1, c->tb, st));
  }
  return NSHE_OK;
}

int nshe_eq_mask(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out, int n_ct,
                 int y_broadcast, void* ws, size_t ws_bytes, void* stream) {
  return eq_mask_impl(c, x, y, out, n_ct, y_broadcast, ws, ws_bytes, stream);
}

int nshe_eq_mask_noalloc(nshe_ctx* c, const int64_t* x, const int64_t* y, int64_t* out,
                         int n_ct, int y_broadcast, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0) return fail(NSHE_ESHAPE, "n_ct < 0");
  const size_t need = ws_doubles(c, n_ct) * sizeof(double);
  if (need > kScratchBytes)
    return fail(NSHE_ENOMEM, std::to_string(n_ct) + " ciphertexts need " + std::to_string(need) +
                                 " bytes of scratch; nshe_eq_mask_noalloc has " +
                                 std::to_string(kScratchBytes) +
                                 " (split the call, or use nshe_eq_mask with a workspace)");
  if (!c->scratch) return fail(NSHE_EDEVICE, "no scratch on this device");
  // profiling records would create events: none in this call
  const bool prof = c->prof;
  c->prof = false;
  const int rc = eq_mask_impl(c, x, y, out, n_ct, y_broadcast, c->scratch, kScratchBytes, stream);
  c->prof = prof;
  return rc;
}

// Batched waves.  The caller's workspace holds, after the ciphertext area
// of one wave, a wave counter (256 bytes) and a table of per-ciphertext
// pointers ([wave][wave_ct] entries); the kernels that read inputs and write outputs look
// up their wave there, so one captured graph serves every wave of a size.
static size_t table_entries(int wave_ct, long long total) { return (size_t)(total + wave_ct); }

static size_t batched_ws_bytes(const nshe_ctx* c, int wave_ct, long long total) {
  const size_t cts = (ws_doubles(c, wave_ct) * sizeof(double) + 255) & ~(size_t)255;
  const size_t tab = (table_entries(wave_ct, total) * sizeof(CtPtrs) + 255) & ~(size_t)255;
  return cts + tab + 256;
}

struct BatchArea {
  CtPtrs* table;
  int* counter;
};

static BatchArea batch_area(const nshe_ctx* c, void* ws, int wave_ct, long long total) {
  char* p = static_cast<char*>(ws);
  const size_t cts = (ws_doubles(c, wave_ct) * sizeof(double) + 255) & ~(size_t)255;
  (void)total;
  return BatchArea{reinterpret_cast<CtPtrs*>(p + cts + 256), reinterpret_cast<int*>(p + cts)};
}

// One wave of cnt ciphertexts: x - y, the 16 levels and the mask's finish,
// the wave's ciphertexts read and written through its table; then advance
// the wave counter by `step` (the number of streams taking turns over the
// table's waves).  With the split inverse the ends are the plain chain's
// fused kernels (subtraction + first lift, last mod-down + finish), else a
// gather, the levels and a scatter.
static int enqueue_wave(nshe_ctx* c, int cnt, int stride, int step, const BatchArea& a,
                        const Ws& w, hipStream_t st) {
  Dims d = dims(c, cnt);
  const WaveTab wt{a.table, a.counter, stride};
  if (split_inverse(c)) {
    d.tab = wt;
    {
      Prof pf(c, K_SUB, st, 2.0 * cnt * c->L * c->n);
      HIPCHK(run_sub_lift(d, nullptr, nullptr, 0, w.ext, c->tb, st));
    }
    int rc = eq_levels(c, w, cnt, st, true, nullptr, &wt);
    if (rc) return rc;
  } else {
    {
      Prof pf(c, K_SUB, st, 2.0 * cnt * c->L * c->n);
      HIPCHK(run_gather_sub(d, stride, a.table, a.counter, w.ext, c->tb, st));
    }
    int rc = eq_levels(c, w, cnt, st);
    if (rc) return rc;
    {
      Prof pf(c, K_CONVERT, st, 2.0 * cnt * c->L * c->n);
      HIPCHK(run_scatter_mask(d, stride, a.table, a.counter, w.ext, c->tb, st));
    }
  }
  HIPCHK(run_bump_counter(a.counter, step, st));
  return NSHE_OK;
}

size_t nshe_batched_workspace_bytes(const nshe_ctx* c, int wave_ct, long long total_ct) {
  if (check_ctx(c) || wave_ct < 1 || total_ct < 0) return 0;
  return batched_ws_bytes(c, wave_ct, total_ct);
}

int nshe_eq_mask_batched(nshe_ctx* c, const nshe_item* items, int n_items, int wave_ct,
                         int use_graph, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_items < 0 || (n_items > 0 && !items)) return fail(NSHE_EINVAL, "bad item list");
  if (c->squarings < 0) return fail(NSHE_EUNSUPPORTED, "t - 1 is not a power of two");
  if (int rc0 = depth_check(c, NSHE_OP_EQ, 0, "EQ")) return rc0;
  if (check_key(c)) return NSHE_ENOKEY;
  if (wave_ct < 0) return fail(NSHE_EINVAL, "wave_ct < 0");
  long long total = 0;
  for (int i = 0; i < n_items; ++i) {
    if (items[i].n_ct < 0) return fail(NSHE_ESHAPE, "item with n_ct < 0");
    if (items[i].n_ct > 0 && (!items[i].x_dev || !items[i].y_dev || !items[i].out_dev))
      return fail(NSHE_EINVAL, "item with a null buffer");
    total += items[i].n_ct;
  }
  if (total == 0) return NSHE_OK;
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  if (wave_ct == 0) {
    // the tuned wave if it fits, else the largest that does
    const size_t per_ct = ws_doubles(c, 1) * sizeof(double) + sizeof(CtPtrs);
    const size_t fixed = (size_t)total * sizeof(CtPtrs) + 1024;
    const long long fit = ws_bytes > fixed ? (long long)((ws_bytes - fixed) / per_ct) : 0;
    wave_ct = (int)std::min<long long>(fit, 1 << 20);
    if (c->tune.wave_ct > 0) wave_ct = std::min(wave_ct, c->tune.wave_ct);
    while (wave_ct > 1 &&
           batched_ws_bytes(c, (int)std::min<long long>(wave_ct, total), total) > ws_bytes)
      --wave_ct;
    if (wave_ct < 1) return fail(NSHE_ENOMEM, "workspace smaller than one wave");
  }
  if (wave_ct > total) wave_ct = (int)total;
  if (ws_bytes < batched_ws_bytes(c, wave_ct, total))
    return fail(NSHE_ENOMEM, "workspace smaller than nshe_batched_workspace_bytes(ctx, wave_ct, total)");
  if (set_device(c)) return NSHE_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const BatchArea area = batch_area(c, ws, wave_ct, total);
  const size_t ctw = (size_t)2 * c->L * c->n;

  // Two streams (tuning streams = 2): half-waves of wave_ct / 2 ciphertexts
  // alternate between st and the context's second stream.  Each stream has
  // its own share of the wave's ciphertext area (the two shares fill it)
  // and its own wave counter (128 bytes apart), which starts at the
  // stream's first wave and steps by two, so that one stream's kernels and
  // graphs never touch the other's.  (Units: the waves the table is laid out
  // in, half-waves with two streams.)
  const int hw = wave_ct / 2;
  const bool two = c->tune.streams == 2 && hw >= 16 && total > hw && !c->prof &&
                   ws_doubles(c, hw) * sizeof(double) % 256 == 0 && stream_idle_capture(st);
  const int unit = two ? hw : wave_ct;
  const int n_seq = two ? 2 : 1;
  const long long n_units = (total + unit - 1) / unit;
  const BatchArea seq[2] = {area, BatchArea{area.table, area.counter + 32}};
  char* const share[2] = {static_cast<char*>(ws),
                          static_cast<char*>(ws) + ws_doubles(c, hw) * sizeof(double)};

  // per-ciphertext pointers, unit by unit (unit u at entries u * unit; at
  // most total + wave_ct entries)
  for (int q = 0; q < n_seq; ++q) HIPCHK(run_set_counter(seq[q].counter, q, st));
  TableChunk ch{};
  ch.first = 0;
  ch.n = 0;
  auto flush = [&]() -> int {
    if (ch.n == 0) return NSHE_OK;
    HIPCHK(run_fill_table(ch, area.table, st));
    ch.first += ch.n;
    ch.n = 0;
    return NSHE_OK;
  };
  for (int i = 0; i < n_items; ++i) {
    const nshe_item& it = items[i];
    for (int j = 0; j < it.n_ct; ++j) {
      CtPtrs e;
      e.x = it.x_dev + (size_t)j * ctw;
      e.y = it.y_broadcast ? it.y_dev : it.y_dev + (size_t)j * ctw;
      e.out = it.out_dev + (size_t)j * ctw;
      ch.e[ch.n++] = e;
      if (ch.n == TableChunk::CAP) {
        int rc = flush();
        if (rc) return rc;
      }
    }
  }
  int rc = flush();
  if (rc) return rc;

  if (two) {
    if ((rc = half_stream_ready(c))) return rc;
    HIPCHK(hipEventRecord(c->half_fork, st));
    HIPCHK(hipStreamWaitEvent(c->half_stream, c->half_fork, 0));
  }
  for (long long u = 0; u < n_units && !rc; ++u) {
    const int q = (int)(u % n_seq);
    hipStream_t su = q ? c->half_stream : st;
    const int cnt = (int)std::min<long long>(unit, total - u * unit);
    Ws w = carve(c, share[q], cnt);
    if (!use_graph) {
      rc = enqueue_wave(c, cnt, unit, n_seq, seq[q], w, su);
      continue;
    }
    const std::vector<uintptr_t> key = {reinterpret_cast<uintptr_t>(share[q]), (uintptr_t)cnt,
                                        (uintptr_t)unit, (uintptr_t)n_seq,
                                        reinterpret_cast<uintptr_t>(seq[q].counter)};
    const bool prof_saved = c->prof;
    c->prof = false;  // no event records inside a captured graph
    struct Restore {
      nshe_ctx* c;
      bool v;
      ~Restore() { c->prof = v; }
    } restore{c, prof_saved};
    auto found = c->graphs.find(key);
    if (found == c->graphs.end()) {
      // Capture on a context-owned stream (nothing executes during capture);
      // the instantiated graph is then launched on the unit's stream.
      if (!c->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
          rc = fail(NSHE_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
          break;
        }
      }
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        rc = fail(NSHE_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        break;
      }
      rc = enqueue_wave(c, cnt, unit, n_seq, seq[q], w, c->cap_stream);
      e = hipStreamEndCapture(c->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        break;
      }
      if (e != hipSuccess) {
        rc = fail(NSHE_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        break;
      }
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        rc = fail(NSHE_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e));
        break;
      }
      if (c->graphs.size() >= 16) drop_graphs(c);
      found = c->graphs.emplace(key, nshe_ctx::GraphEntry{ex}).first;
    }
    hipError_t e = hipGraphLaunch(found->second.exec, su);
    if (e != hipSuccess) rc = fail(NSHE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  }
  if (two) {
    // st waits for the second stream's units whatever happened above
    HIPCHK(hipEventRecord(c->half_join, c->half_stream));
    HIPCHK(hipStreamWaitEvent(st, c->half_join, 0));
  }
  return rc;
}

// bytes of an int64 ciphertext array, rounded up to 256
static size_t ct_bytes(const nshe_ctx* c, int n_ct) {
  return ((size_t)n_ct * 2 * c->L * c->n * sizeof(int64_t) + 255) & ~(size_t)255;
}

// ------------------------------------------------------------- rotations

// Galois elements of the rotate-and-add sum, in order: 3^(N/4), ..., 3^1
// (rotations of each half of the slots by N/4, ..., 1), then 2N - 1 (swap).
static std::vector<uint32_t> sum_elements(const nshe_ctx* c) {
  std::vector<uint32_t> out;
  const uint64_t two_n = 2ull * c->n;
  for (int r = c->n / 4; r >= 1; r /= 2) {
    uint64_t g = 1;
    for (int k = 0; k < r; ++k) g = g * 3 % two_n;
    out.push_back((uint32_t)g);
  }
  out.push_back((uint32_t)(two_n - 1));
  return out;
}

static unsigned inv_mod_2n(const nshe_ctx* c, uint32_t g) {
  const uint64_t two_n = 2ull * c->n;
  uint64_t x = 1;
  for (uint64_t k = 1; k < two_n; ++k) {
    x = x * g % two_n;
    if (x == 1) {
      // g^k = 1, so g^(k-1) = g^-1
      uint64_t r = 1;
      for (uint64_t m = 0; m + 1 < k; ++m) r = r * g % two_n;
      return (unsigned)r;
    }
  }
  return 1;
}

// One rotation of the ciphertexts in w.ext by Galois element g into `out`
// ([ct][2][W][N] limbs 0..L-1).
static int rotate_ext(nshe_ctx* c, const Ws& w, int n_ct, uint32_t g, const double* key,
                      double* out, hipStream_t st, bool accumulate = false) {
  Dims d = dims(c, n_ct);
  {
    Prof pf(c, K_AUTOMORPH, st, 2.0 * n_ct * c->L * c->n);
    const DigitSrc ds = digit_src(c, w);
    HIPCHK(run_automorph(d, inv_mod_2n(c, g), w.ext, w.dt, c->tb, st, ds.split ? ds.p : nullptr,
                         ds.stride, ds.split));
    if (c->alpha > 1) HIPCHK(run_digit_mrc(d, ds.p, ds.stride, c->tb, st));
  }
  return relin(c, w, n_ct, st, key, out, false, nullptr, nullptr, accumulate);
}

// ct <- ct + rot_g(ct) over the sum elements, on the ciphertexts in w.ext
static int sum_slots_ext(nshe_ctx* c, const Ws& w, int n_ct, const std::vector<uint32_t>& els,
                         const std::vector<const double*>& keys, hipStream_t st) {
  // the rotation's mod-down adds its result into the running sum in ext
  // (the automorphism has read ext before)
  for (size_t k = 0; k < els.size(); ++k) {
    int rc = rotate_ext(c, w, n_ct, els[k], keys[k], w.ext, st, true);
    if (rc) return rc;
  }
  return NSHE_OK;
}

// The Galois keys of the sum elements (NSHE_ENOKEY naming a missing one).
static int sum_keys(nshe_ctx* c, std::vector<uint32_t>* els, std::vector<const double*>* keys) {
  *els = sum_elements(c);
  keys->clear();
  for (uint32_t g : *els) {
    auto k = c->galois.find(g);
    if (k == c->galois.end()) return fail(NSHE_ENOKEY, "no Galois key for g = " + std::to_string(g));
    keys->push_back(k->second);
  }
  return NSHE_OK;
}

int nshe_galois_elements(const nshe_ctx* c, uint32_t* out, int max_out, int* n_out) {
  g_err.clear();
  if (check_ctx(c) || !n_out || (max_out > 0 && !out)) return fail(NSHE_EINVAL, "null argument");
  const std::vector<uint32_t> e = sum_elements(c);
  *n_out = (int)e.size();
  for (int i = 0; i < (int)e.size() && i < max_out; ++i) out[i] = e[i];
  return NSHE_OK;
}

int nshe_rotate(nshe_ctx* c, const int64_t* in, uint32_t g, int64_t* out, int n_ct, void* ws,
                size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, false);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in || !out) return fail(NSHE_EINVAL, "null buffer");
  auto key = c->galois.find(g);
  if (key == c->galois.end()) return fail(NSHE_ENOKEY, "no Galois key for g = " + std::to_string(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_i64_to_polys(d, in, 2, w.ext, 2 * W * N, W * N, 2, c->tb, st));
  rc = rotate_ext(c, w, n_ct, g, key->second, w.fx, st);
  if (rc) return rc;
  HIPCHK(run_polys_to_i64(d, w.fx, 2, 2 * W * N, W * N, out, 0, c->tb, st));
  return NSHE_OK;
}

int nshe_sum_slots(nshe_ctx* c, const int64_t* in, int64_t* out, int n_ct, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, false);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in || !out) return fail(NSHE_EINVAL, "null buffer");
  std::vector<uint32_t> els;
  std::vector<const double*> keys;
  rc = sum_keys(c, &els, &keys);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in, (size_t)n_ct * 2}}))) return rc;
  // the rotate-and-add of cnt ciphertexts from ciphertext c0, on s
  auto run = [&](int c0, int cnt, void* wsh, hipStream_t s) -> int {
    const size_t ctw = (size_t)2 * c->L * c->n;
    Ws w = carve(c, wsh, cnt);
    Dims d = dims(c, cnt);
    const size_t W = W_of(c), N = c->n;
    HIPCHK(run_i64_to_polys(d, in + c0 * ctw, 2, w.ext, 2 * W * N, W * N, 2, c->tb, s));
    int rc1 = sum_slots_ext(c, w, cnt, els, keys, s);
    if (rc1) return rc1;
    HIPCHK(run_polys_to_i64(d, w.ext, 2, 2 * W * N, W * N, out + c0 * ctw, 0, c->tb, s));
    return NSHE_OK;
  };
  // (with the tuning's two streams: the two halves of the ciphertexts on two
  // streams, as the EQ call)
  if (two_halves(c, n_ct, ws, st)) return run_two_halves(c, n_ct, ws, st, run);
  return run(0, n_ct, ws, st);
}

// ------------------------------------------------------ plaintext products

// ct (in w.ext, data limbs) times the plaintext pt (int64 [N] in [0, t)) into
// w.fx's data limbs: forward transforms of ct and of the plaintext's limbs
// (times N^-1, in w.dt), pointwise products, inverse transform.
static int mul_plain_ext(nshe_ctx* c, const Ws& w, const int64_t* pt, int n_ct, hipStream_t st) {
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_plain_limbs(d, (int64_t)c->t, pt, w.dt, c->tb, st));
  NttJob j{};
  j.split = c->tune.split_forward;
  j.base = w.dt;
  j.out = w.dt + W * N;
  j.poly_stride = W * N;
  j.npoly = 1;
  j.nlimb = c->L;
  j.limb_prime = c->lp_ext;
  j.count = c->L;
  {
    Prof pf(c, K_NTT_FWD, st, ntt_work(c, j.count));
    HIPCHK(run_ntt(c->log2n, j, c->tb, 0, st));
  }
  j.base = w.ext;
  j.out = w.fx;
  j.npoly = 2 * n_ct;
  j.count = j.npoly * c->L;
  {
    Prof pf(c, K_NTT_FWD, st, ntt_work(c, j.count));
    HIPCHK(run_ntt(c->log2n, j, c->tb, 0, st));
  }
  HIPCHK(run_pointwise_plain(d, w.fx, w.dt + W * N, c->tb, st));
  j.base = w.fx;
  j.out = nullptr;
  {
    Prof pf(c, K_NTT_INV, st, ntt_work(c, j.count));
    HIPCHK(run_ntt(c->log2n, j, c->tb, 1, st));
  }
  return NSHE_OK;
}

// The basis plaintext of `slot` (slot order of the 2 x N/2 layout) into out.
static int basis_plain(nshe_ctx* c, int slot, int64_t* out, hipStream_t st) {
  const u64 t = c->t, two_n = 2ull * c->n;
  const u64 psi = powmod(primitive_root(t), (t - 1) / two_n, t);
  const int half = c->n / 2;
  u64 e = 1;
  for (int s = 0; s < slot % half; ++s) e = e * 3 % two_n;
  if (slot >= half) e = two_n - e;
  const u64 zinv = powmod(psi, two_n - e, t);   // psi^-e
  HIPCHK(run_basis_plain(c->n, t, zinv, invmod((u64)c->n % t, t), out, st));
  return NSHE_OK;
}

int nshe_mul_plain(nshe_ctx* c, const int64_t* in, const int64_t* pt, int64_t* out, int n_ct,
                   void* ws, size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, false);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in || !pt || !out) return fail(NSHE_EINVAL, "null buffer");
  if ((c->t - 1) % (2ull * c->n))
    return fail(NSHE_EUNSUPPORTED, "plaintext slots need t = 1 mod 2N");
  if ((rc = depth_check(c, NSHE_OP_MUL_PLAIN, 0, "a plaintext product"))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_i64_to_polys(d, in, 2, w.ext, 2 * W * N, W * N, 2, c->tb, st));
  rc = mul_plain_ext(c, w, pt, n_ct, st);
  if (rc) return rc;
  HIPCHK(run_polys_to_i64(d, w.fx, 2, 2 * W * N, W * N, out, 0, c->tb, st));
  return NSHE_OK;
}

// Extract (broadcast = 0) or Broadcast (1) of one slot, ciphertexts in w.ext
// -> w.ext.
static int extract_ext(nshe_ctx* c, const Ws& w, int slot, int n_ct, int bcast, hipStream_t st) {
  int64_t* pt = reinterpret_cast<int64_t*>(w.acc);
  int rc = basis_plain(c, slot, pt, st);
  if (rc) return rc;
  rc = mul_plain_ext(c, w, pt, n_ct, st);
  if (rc) return rc;
  const size_t W = W_of(c), N = c->n;
  HIPCHK(hipMemcpyAsync(w.ext, w.fx, (size_t)n_ct * 2 * W * N * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
  if (!bcast) return NSHE_OK;
  std::vector<uint32_t> els;
  std::vector<const double*> keys;
  rc = sum_keys(c, &els, &keys);
  if (rc) return rc;
  return sum_slots_ext(c, w, n_ct, els, keys, st);
}

int nshe_extract(nshe_ctx* c, const int64_t* in, int slot, int broadcast, int64_t* out,
                 int n_ct, void* ws, size_t ws_bytes, void* stream) {
  int rc = common_checks(c, n_ct, ws, ws_bytes, false);
  if (rc) return rc;
  if (n_ct == 0) return NSHE_OK;
  if (!in || !out) return fail(NSHE_EINVAL, "null buffer");
  if (slot < 0 || slot >= c->n) return fail(NSHE_EINVAL, "slot out of range");
  if ((c->t - 1) % (2ull * c->n))
    return fail(NSHE_EUNSUPPORTED, "plaintext slots need t = 1 mod 2N");
  if ((rc = depth_check(c, NSHE_OP_MUL_PLAIN, 0, "a plaintext product"))) return rc;
  if (broadcast) {
    std::vector<uint32_t> els;
    std::vector<const double*> keys;
    rc = sum_keys(c, &els, &keys);
    if (rc) return rc;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = check_inputs(c, st, {{in, (size_t)n_ct * 2}}))) return rc;
  Ws w = carve(c, ws, n_ct);
  Dims d = dims(c, n_ct);
  const size_t W = W_of(c), N = c->n;
  HIPCHK(run_i64_to_polys(d, in, 2, w.ext, 2 * W * N, W * N, 2, c->tb, st));
  rc = extract_ext(c, w, slot, n_ct, broadcast ? 1 : 0, st);
  if (rc) return rc;
  HIPCHK(run_polys_to_i64(d, w.ext, 2, 2 * W * N, W * N, out, 0, c->tb, st));
  return NSHE_OK;
}

// ------------------------------------------------------------------ JOIN

size_t nshe_join_workspace_bytes(const nshe_ctx* c, int n_ct) {
  if (check_ctx(c) || n_ct < 0) return 0;
  return 3 * ct_bytes(c, n_ct) + 2 * ct_bytes(c, 1) + ws_doubles(c, std::max(n_ct, 1)) * sizeof(double);
}

int nshe_join_sum(nshe_ctx* c, const int64_t* a_key, const int64_t* b_key, const int64_t* b_attr,
                  const int32_t* rows, int n_rows, int64_t* out, int n_ct, void* ws,
                  size_t ws_bytes, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0 || n_rows < 0) return fail(NSHE_ESHAPE, "n_ct or n_rows < 0");
  if (n_ct == 0) return NSHE_OK;
  if (!a_key || !b_key || !b_attr || !out || (n_rows > 0 && !rows))
    return fail(NSHE_EINVAL, "null buffer");
  if (c->squarings < 0) return fail(NSHE_EUNSUPPORTED, "t - 1 is not a power of two");
  if ((c->t - 1) % (2ull * c->n))
    return fail(NSHE_EUNSUPPORTED, "plaintext slots need t = 1 mod 2N");
  if (int rc0 = depth_check(c, NSHE_OP_JOIN, 0, "JOIN")) return rc0;
  for (int r = 0; r < n_rows; ++r)
    if (rows[r] < 0 || rows[r] >= c->n) return fail(NSHE_EINVAL, "row index out of range");
  if (check_key(c)) return NSHE_ENOKEY;
  {
    std::vector<uint32_t> els;
    std::vector<const double*> keys;
    int rc = sum_keys(c, &els, &keys);
    if (rc) return rc;
  }
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < nshe_join_workspace_bytes(c, n_ct))
    return fail(NSHE_ENOMEM, "workspace smaller than nshe_join_workspace_bytes(ctx, n_ct)");
  if (set_device(c)) return NSHE_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc0 = check_inputs(c, st, {{a_key, (size_t)n_ct * 2}, {b_key, 2}, {b_attr, 2}}))
    return rc0;
  if (n_rows == 0) return nshe_sum(c, nullptr, 0, out, n_ct, stream);
  const size_t cb = ct_bytes(c, n_ct), cb1 = ct_bytes(c, 1);
  char* p = static_cast<char*>(ws);
  int64_t* mask = reinterpret_cast<int64_t*>(p);
  int64_t* term = reinterpret_cast<int64_t*>(p + cb);
  int64_t* rep = reinterpret_cast<int64_t*>(p + 2 * cb);
  int64_t* bk = reinterpret_cast<int64_t*>(p + 3 * cb);
  int64_t* ba = reinterpret_cast<int64_t*>(p + 3 * cb + cb1);
  void* mws = p + 3 * cb + 2 * cb1;
  const size_t mws_bytes = ws_bytes - (3 * cb + 2 * cb1);
  const size_t ctw = (size_t)2 * c->L * c->n;
  Dims d = dims(c, n_ct);
  for (int r = 0; r < n_rows; ++r) {
    int rc = nshe_extract(c, b_key, rows[r], 1, bk, 1, mws, mws_bytes, stream);
    if (!rc) rc = nshe_extract(c, b_attr, rows[r], 1, ba, 1, mws, mws_bytes, stream);
    if (!rc) rc = nshe_eq_mask(c, a_key, bk, mask, n_ct, 1, mws, mws_bytes, stream);
    if (rc) return rc;
    for (int k = 0; k < n_ct; ++k)
      HIPCHK(hipMemcpyAsync(rep + k * ctw, ba, ctw * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    rc = nshe_mul_relin(c, mask, rep, r == 0 ? out : term, n_ct, mws, mws_bytes, stream);
    if (rc) return rc;
    if (r > 0) HIPCHK(run_sum_i64(d, out, term, 0, 1, out, c->tb, st));
  }
  return NSHE_OK;
}

// ------------------------------------------------------------ comparisons

static int ilog2(int x) {
  int r = 0;
  while ((1 << (r + 1)) <= x) ++r;
  return r;
}

// Ciphertext-array slots of the comparison workspace (then the multiply
// workspace): chain levels 1..K (slot 0 unused), babies, giants, 16
// linear combinations, the core's g, T, S, and the callers' z, LT, and two
// comparison results (the last four).
static int cmp_slots(const nshe_ctx* c) { return c->lt_K + 1 + c->lt_k + c->lt_m + 16 + 3 + 4; }

// one operand's transform, [n_ct][2][W][N] doubles
static size_t fx_bytes(const nshe_ctx* c, int n_ct) {
  return ((size_t)n_ct * 2 * W_of(c) * c->n * sizeof(double) + 255) & ~(size_t)255;
}

// the summed tensor, [n_ct][3][W][N] doubles
static size_t dacc_bytes(const nshe_ctx* c, int n_ct) {
  return ((size_t)n_ct * 3 * W_of(c) * c->n * sizeof(double) + 255) & ~(size_t)255;
}

size_t nshe_compare_workspace_bytes(const nshe_ctx* c, int n_ct) {
  if (check_ctx(c) || n_ct < 0 || c->lt_K == 0) return 0;
  return (size_t)cmp_slots(c) * ct_bytes(c, n_ct) + fx_bytes(c, n_ct) + dacc_bytes(c, n_ct) +
         ws_doubles(c, n_ct) * sizeof(double);
}

struct CmpArea {
  int64_t* slot0;
  size_t U;       // int64 words per slot
  double* fx;     // a shared operand's transform (mul_shared)
  double* dacc;   // the giants' products' summed tensor
  void* mws;      // multiply workspace
  size_t mws_bytes;
  int64_t* slot(int i) const { return slot0 + (size_t)i * U; }
};

// A product a * b relinearized (as nshe_mul_relin) whose first operand's
// lift and transform are kept in the area's fx and reused while the next
// product has the same first operand (`held`): the babies' and giants'
// products share their power-of-two factor.  Same arithmetic, so the same
// result as nshe_mul_relin.
static int mul_shared(nshe_ctx* c, const CmpArea& a, const int64_t** held, const int64_t* x,
                      const int64_t* y, int64_t* out, int n_ct, hipStream_t st) {
  Ws w = carve(c, a.mws, n_ct);
  if (*held != x) {
    int rc = prepare_i64(c, x, w.ext, a.fx, n_ct, st);
    if (rc) return rc;
    *held = x;
  }
  int rc = prepare_i64(c, y, w.dig, fx_second(c, w, n_ct), n_ct, st);
  if (rc) return rc;
  rc = tensor_scale(c, w, fx_second(c, w, n_ct), n_ct, st, a.fx);
  if (rc) return rc;
  return relin_i64(c, w, n_ct, st, out);
}

// LT of the differences z (int64, n_ct ciphertexts, not in the area) into
// out: the baby-step giant-step program of the comparison polynomial
// (its odd part in w = z^2, powers of two of w from the squaring chain).
// On return slot `one` holds the trivial encryption of 1.
static int lt_core(nshe_ctx* c, const int64_t* z, int64_t* out, int n_ct, const CmpArea& a,
                   int* one_slot, hipStream_t st) {
  const int K = c->lt_K, k = c->lt_k, m = c->lt_m;
  void* stv = st;
  const int s_lev = 0, s_bab = K + 1, s_gi = s_bab + k, s_G = s_gi + m, s_g = s_G + 16,
            s_T = s_g + 1, s_S = s_g + 2;
  Dims d = dims(c, n_ct);
  std::vector<const int64_t*> lev(K + 1);
  lev[0] = z;
  for (int i = 1; i <= K; ++i) {
    int rc = nshe_square_relin(c, lev[i - 1], a.slot(s_lev + i), n_ct, a.mws, a.mws_bytes, stv);
    if (rc) return rc;
    lev[i] = a.slot(s_lev + i);
  }
  BabyPtrs bp{};
  HIPCHK(run_fill_one(d, a.slot(s_bab), c->tb, st));
  bp.p[0] = a.slot(s_bab);
  bp.p[1] = lev[1];
  const int64_t* held = nullptr;   // the operand whose transform a.fx holds
  for (int i = 2; i < k; ++i) {
    const int h = 1 << ilog2(i), r = i - h;
    if (r == 0) {
      bp.p[i] = lev[ilog2(i) + 1];
    } else {
      int rc = mul_shared(c, a, &held, bp.p[h], bp.p[r], a.slot(s_bab + i), n_ct, st);
      if (rc) return rc;
      bp.p[i] = a.slot(s_bab + i);
    }
  }
  std::vector<const int64_t*> gi(m, nullptr);
  if (m > 1) gi[1] = lev[ilog2(k) + 1];
  for (int j = 2; j < m; ++j) {
    const int h = 1 << ilog2(j), r = j - h;
    if (r == 0) {
      gi[j] = lev[ilog2(k) + ilog2(j) + 1];
    } else {
      int rc = mul_shared(c, a, &held, gi[h], gi[r], a.slot(s_gi + j), n_ct, st);
      if (rc) return rc;
      gi[j] = a.slot(s_gi + j);
    }
  }
  // g = G_0 + sum_{j>=1} G_j W_j, G_j = sum_i c_(2(jk+i)+1) B_i in chunks of
  // 16.  The products' tensors are summed in the extended basis (exact: Q B
  // exceeds m N Q^2), then scaled, rounded and relinearized once.
  int64_t* g = a.slot(s_g);
  Ws w = carve(c, a.mws, n_ct);
  for (int j0 = 0; j0 < m; j0 += 16) {
    const int J = std::min(16, m - j0);
    {
      Prof pf(c, K_LINCOMB, st, (double)J * k * n_ct * 2 * c->L * c->n);
      HIPCHK(run_lincomb(d, k, bp, c->lt_coef + (size_t)j0 * k, J, a.slot(s_G), a.U, c->tb, st));
    }
    for (int jj = 0; jj < J; ++jj) {
      const int j = j0 + jj;
      const int64_t* Gj = a.slot(s_G + jj);
      if (j == 0) {
        HIPCHK(run_sum_i64(d, Gj, nullptr, 0, 0, g, c->tb, st));
        continue;
      }
      int rc = load_two(c, w, Gj, gi[j], n_ct, st);
      if (rc) return rc;
      Prof pf(c, K_TENSOR_MAC, st, 3.0 * n_ct * W_of(c) * c->n);
      HIPCHK(run_tensor_mac(d, w.fx, fx_second(c, w, n_ct), a.dacc, j == 1 ? 1 : 0, c->tb, st));
    }
  }
  if (m > 1) {
    NttJob j{};
    j.base = a.dacc;
    j.out = w.dt;
    j.poly_stride = (size_t)W_of(c) * c->n;
    j.npoly = n_ct * 3;
    j.nlimb = W_of(c);
    j.limb_prime = c->lp_ext;
    j.count = j.npoly * j.nlimb;
    j.split_inv = d.fused;
    {
      Prof pf(c, K_NTT_INV, st, ntt_work(c, j.count));
      HIPCHK(run_ntt(c->log2n, j, c->tb, 4, st));
    }
    {
      const DigitSrc ds = digit_src(c, w);
      Prof pf(c, K_SCALE, st, 3.0 * n_ct * c->n);
      HIPCHK(run_scale(d, w.dt, c->tb, st, c->alpha > 1, ds.split ? ds.p : nullptr));
    }
    int rc = relin_i64(c, w, n_ct, st, a.slot(s_T));
    if (rc) return rc;
    HIPCHK(run_sum_i64(d, g, a.slot(s_T), 0, 1, g, c->tb, st));
  }
  // out = c_(p-1) z^(p-1) + z g
  int rc = nshe_mul_relin(c, lev[0], g, a.slot(s_T), n_ct, a.mws, a.mws_bytes, stv);
  if (rc) return rc;
  BabyPtrs top{};
  top.p[0] = lev[K];
  {
    Prof pf(c, K_LINCOMB, st, (double)n_ct * 2 * c->L * c->n);
    HIPCHK(run_lincomb(d, 1, top, c->lt_coef + (size_t)m * k, 1, a.slot(s_S), a.U, c->tb, st));
  }
  HIPCHK(run_sum_i64(d, a.slot(s_S), a.slot(s_T), 0, 1, out, c->tb, st));
  *one_slot = s_bab;
  return NSHE_OK;
}

static int cmp_checks(nshe_ctx* c, int n_ct, void* ws, size_t ws_bytes, CmpArea* a, int op) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (c->lt_K == 0) return fail(NSHE_EUNSUPPORTED, "comparisons need t = 2^K + 1 prime");
  if (int rc0 = depth_check(c, op, 0, op == NSHE_OP_LT ? "LT" : "BETWEEN")) return rc0;
  if (n_ct < 0) return fail(NSHE_ESHAPE, "n_ct < 0");
  if (check_key(c)) return NSHE_ENOKEY;
  if (n_ct == 0) return NSHE_OK;
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < nshe_compare_workspace_bytes(c, n_ct))
    return fail(NSHE_ENOMEM, "workspace smaller than nshe_compare_workspace_bytes(ctx, n_ct)");
  if (set_device(c)) return NSHE_EDEVICE;
  const size_t cb = ct_bytes(c, n_ct);
  a->slot0 = static_cast<int64_t*>(ws);
  a->U = cb / sizeof(int64_t);
  a->fx = reinterpret_cast<double*>(static_cast<char*>(ws) + (size_t)cmp_slots(c) * cb);
  a->dacc = reinterpret_cast<double*>(reinterpret_cast<char*>(a->fx) + fx_bytes(c, n_ct));
  const size_t used = (size_t)cmp_slots(c) * cb + fx_bytes(c, n_ct) + dacc_bytes(c, n_ct);
  a->mws = static_cast<char*>(ws) + used;
  a->mws_bytes = ws_bytes - used;
  return NSHE_OK;
}

// z = sign (x - y) into the area's last slot, then LT (op 0) or 1 - LT (op 1)
static int compare_into(nshe_ctx* c, const int64_t* x, const int64_t* y, int y_bcast, int op,
                        int64_t* out, int n_ct, const CmpArea& a, hipStream_t st) {
  Dims d = dims(c, n_ct);
  int64_t* z = a.slot(cmp_slots(c) - 1);
  // LT(x, y) takes z = x - y; LE(x, y) = 1 - LT(y, x) takes z = y - x
  HIPCHK(run_diff_i64(d, x, y, y_bcast, op == 1 ? 1 : 0, z, c->tb, st));
  int one = 0;
  if (op == 0) return lt_core(c, z, out, n_ct, a, &one, st);
  int64_t* lt = a.slot(cmp_slots(c) - 2);
  int rc = lt_core(c, z, lt, n_ct, a, &one, st);
  if (rc) return rc;
  HIPCHK(run_diff_i64(d, a.slot(one), lt, 0, 0, out, c->tb, st));
  return NSHE_OK;
}

int nshe_compare(nshe_ctx* c, const int64_t* x, const int64_t* y, int y_broadcast, int op,
                 int64_t* out, int n_ct, void* ws, size_t ws_bytes, void* stream) {
  CmpArea a{};
  int rc = cmp_checks(c, n_ct, ws, ws_bytes, &a, NSHE_OP_LT);
  if (rc || n_ct == 0) return rc;
  if (op != 0 && op != 1) return fail(NSHE_EINVAL, "op must be 0 (LT) or 1 (LE)");
  if (!x || !y || !out) return fail(NSHE_EINVAL, "null buffer");
  if ((rc = check_inputs(c, static_cast<hipStream_t>(stream),
                         {{x, (size_t)n_ct * 2}, {y, y_broadcast ? (size_t)2 : (size_t)n_ct * 2}})))
    return rc;
  return compare_into(c, x, y, y_broadcast ? 1 : 0, op, out, n_ct, a,
                      static_cast<hipStream_t>(stream));
}

int nshe_between(nshe_ctx* c, const int64_t* x, const int64_t* lo, const int64_t* hi,
                 int bounds_broadcast, int64_t* out, int n_ct, void* ws, size_t ws_bytes,
                 void* stream) {
  CmpArea a{};
  int rc = cmp_checks(c, n_ct, ws, ws_bytes, &a, NSHE_OP_BETWEEN);
  if (rc || n_ct == 0) return rc;
  if (!x || !lo || !hi || !out) return fail(NSHE_EINVAL, "null buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    const size_t nb = bounds_broadcast ? (size_t)2 : (size_t)n_ct * 2;
    if ((rc = check_inputs(c, st, {{x, (size_t)n_ct * 2}, {lo, nb}, {hi, nb}}))) return rc;
  }
  Dims d = dims(c, n_ct);
  const int bc = bounds_broadcast ? 1 : 0;
  int64_t* ge = a.slot(cmp_slots(c) - 3);   // [lo <= x] = 1 - LT(x, lo)
  int64_t* z = a.slot(cmp_slots(c) - 1);
  HIPCHK(run_diff_i64(d, x, lo, bc, 0, z, c->tb, st));
  int one = 0;
  int64_t* lt = a.slot(cmp_slots(c) - 2);
  rc = lt_core(c, z, lt, n_ct, a, &one, st);
  if (rc) return rc;
  HIPCHK(run_diff_i64(d, a.slot(one), lt, 0, 0, ge, c->tb, st));
  // [x <= hi] = 1 - LT(hi, x), z = hi - x
  HIPCHK(run_diff_i64(d, x, hi, bc, 1, z, c->tb, st));
  rc = lt_core(c, z, lt, n_ct, a, &one, st);
  if (rc) return rc;
  int64_t* le = a.slot(cmp_slots(c) - 4);
  HIPCHK(run_diff_i64(d, a.slot(one), lt, 0, 0, le, c->tb, st));
  return nshe_mul_relin(c, ge, le, out, n_ct, a.mws, a.mws_bytes, stream);
}

// ------------------------------------------------------------ IN / GROUP BY

static int in_wave(const nshe_ctx* c, int wave_ct, long long total) {
  if (wave_ct <= 0) wave_ct = c->tune.wave_ct > 0 ? c->tune.wave_ct : 32;
  return (int)std::min<long long>(wave_ct, total);
}

static size_t in_masks_bytes(const nshe_ctx* c, int n_ct, int k) {
  return ((size_t)k * n_ct * 2 * c->L * c->n * sizeof(int64_t) + 255) & ~(size_t)255;
}

size_t nshe_in_workspace_bytes(const nshe_ctx* c, int n_ct, int k, int wave_ct) {
  if (check_ctx(c) || n_ct < 0 || k < 0 || wave_ct < 0) return 0;
  const long long total = (long long)k * n_ct;
  if (total == 0) return 256;
  return in_masks_bytes(c, n_ct, k) + batched_ws_bytes(c, in_wave(c, wave_ct, total), total);
}

int nshe_in_mask(nshe_ctx* c, const int64_t* x, const int64_t* set, int k, int64_t* out, int n_ct,
                 int wave_ct, int use_graph, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (n_ct < 0 || k < 0 || wave_ct < 0) return fail(NSHE_ESHAPE, "n_ct, k or wave_ct < 0");
  if (n_ct == 0) return NSHE_OK;
  if (!x || !out || (k > 0 && !set)) return fail(NSHE_EINVAL, "null buffer");
  if (c->squarings < 0) return fail(NSHE_EUNSUPPORTED, "t - 1 is not a power of two");
  if (int rc0 = depth_check(c, NSHE_OP_IN, k, "IN")) return rc0;
  if (k == 0) return nshe_sum(c, nullptr, 0, out, n_ct, stream);
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  const long long total = (long long)k * n_ct;
  const int wave = in_wave(c, wave_ct, total);
  const size_t mb = in_masks_bytes(c, n_ct, k);
  if (ws_bytes < mb + batched_ws_bytes(c, wave, total))
    return fail(NSHE_ENOMEM, "workspace smaller than nshe_in_workspace_bytes(ctx, n_ct, k, wave_ct)");
  const size_t ctw = (size_t)2 * c->L * c->n;
  int64_t* masks = static_cast<int64_t*>(ws);
  std::vector<nshe_item> items((size_t)k);
  for (int j = 0; j < k; ++j)
    items[j] = nshe_item{x, set + (size_t)j * ctw, masks + (size_t)j * n_ct * ctw, n_ct, 1};
  int rc = nshe_eq_mask_batched(c, items.data(), k, wave, use_graph, static_cast<char*>(ws) + mb,
                                ws_bytes - mb, stream);
  if (rc) return rc;
  return nshe_sum(c, masks, k, out, n_ct, stream);
}

// ---------------------------------------------------------------- tuning

static bool tuning_valid(const nshe_tuning& t) {
  const bool ks = t.ks_chunk == 4 || t.ks_chunk == 8 || t.ks_chunk == 16 || t.ks_chunk == 32;
  const bool blk = t.ew_block == 64 || t.ew_block == 128 || t.ew_block == 256;
  return ks && blk && (t.split_forward == 0 || t.split_forward == 1) && t.wave_ct >= 0 &&
         (t.ks_fused == 0 || t.ks_fused == 1) && (t.streams == 1 || t.streams == 2);
}

static void drop_graphs(nshe_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
}

int nshe_get_tuning(nshe_ctx* c, nshe_tuning* out) {
  g_err.clear();
  if (check_ctx(c) || !out) return fail(NSHE_EINVAL, "null argument");
  *out = c->tune;
  return NSHE_OK;
}

int nshe_set_tuning(nshe_ctx* c, const nshe_tuning* in) {
  g_err.clear();
  if (check_ctx(c) || !in) return fail(NSHE_EINVAL, "null argument");
  if (!tuning_valid(*in)) return fail(NSHE_EINVAL, "tuning value out of range");
  if (set_device(c)) return NSHE_EDEVICE;
  drop_graphs(c);
  c->tune = *in;
  return NSHE_OK;
}

namespace {

// Per-kind event time of the records taken since the last call (waits).
static int drain_records(nshe_ctx* c, double ms[K_COUNT]) {
  for (int i = 0; i < K_COUNT; ++i) ms[i] = 0.0;
  for (auto& r : c->recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.kind] += t;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return NSHE_OK;
}

// Fill the first n_ct ciphertext slots of ext from the sample, cyclically.
static int load_sample(nshe_ctx* c, const Ws& w, const int64_t* sample, int n_sample, int n_ct,
                       hipStream_t st) {
  const size_t W = W_of(c), N = c->n, ctw = (size_t)2 * c->L * N;
  for (int k = 0; k < n_ct; k += n_sample) {
    const int m = std::min(n_sample, n_ct - k);
    HIPCHK(run_i64_to_polys(dims(c, m), sample, 2, w.ext + (size_t)k * 2 * W * N, 2 * W * N,
                            W * N, 2, c->tb, st));
  }
  (void)ctw;
  return NSHE_OK;
}

// Per-kind times of `reps` squaring levels on n_ct ciphertexts (after one
// untimed level) under tuning t.
static int time_kinds(nshe_ctx* c, const nshe_tuning& t, const Ws& w, int n_ct, int reps,
                      hipStream_t st, double ms[K_COUNT]) {
  c->tune = t;
  c->prof = false;
  int rc = square_level(c, w, n_ct, st);
  if (rc) return rc;
  c->prof = true;
  for (int i = 0; i < reps; ++i) {
    rc = square_level(c, w, n_ct, st);
    if (rc) return rc;
  }
  c->prof = false;
  return drain_records(c, ms);
}

// Wall time of one squaring level on n_ct ciphertexts (after one untimed).
static int time_level(nshe_ctx* c, const Ws& w, int n_ct, hipStream_t st, double* ms) {
  int rc = square_level(c, w, n_ct, st);
  if (rc) return rc;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return fail(NSHE_EDEVICE, "event creation failed");
  HIPCHK(hipEventRecord(a, st));
  rc = square_level(c, w, n_ct, st);
  if (rc) return rc;
  HIPCHK(hipEventRecord(b, st));
  HIPCHK(hipEventSynchronize(b));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, a, b));
  c->pool.push_back(a);
  c->pool.push_back(b);
  *ms = t;
  return NSHE_OK;
}

}  // namespace

int nshe_autotune(nshe_ctx* c, const int64_t* sample, int n_sample, int max_wave_ct, void* ws,
                  size_t ws_bytes, void* stream, nshe_tuning* out, double* ms_per_ct) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (!sample || n_sample < 1) return fail(NSHE_EINVAL, "empty sample");
  if (max_wave_ct < 0) return fail(NSHE_EINVAL, "max_wave_ct < 0");
  if (check_key(c)) return NSHE_ENOKEY;
  if (!ws) return fail(NSHE_EINVAL, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NSHE_EINVAL, "workspace not 256-byte aligned");
  const size_t per_ct = ws_doubles(c, 1) * sizeof(double);
  int fit = (int)std::min<size_t>(ws_bytes / per_ct, 1 << 20);
  if (max_wave_ct > 0) fit = std::min(fit, max_wave_ct);
  if (fit < 1) return fail(NSHE_ENOMEM, "workspace smaller than one ciphertext's");
  if (set_device(c)) return NSHE_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);

  // the caller's profiling records and flag are set aside meanwhile
  std::vector<nshe_ctx::Rec> saved_recs;
  saved_recs.swap(c->recs);
  const bool saved_prof = c->prof;
  const nshe_tuning start = c->tune;
  struct Restore {
    nshe_ctx* c;
    std::vector<nshe_ctx::Rec>& recs;
    bool prof;
    ~Restore() {
      for (auto& r : c->recs) {
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
      }
      c->recs.swap(recs);
      c->prof = prof;
    }
  } restore{c, saved_recs, saved_prof};

  // 1. launch shapes, one parameter at a time (each moves only its own
  // kernels' times), on up to 32 ciphertexts
  const int n_t = std::min(fit, 32);
  Ws w = carve(c, ws, n_t);
  int rc = load_sample(c, w, sample, n_sample, n_t, st);
  if (rc) { c->tune = start; return rc; }
  nshe_tuning best = start;
  double ms[K_COUNT];
  {
    const int cand[] = {4, 8, 16, 32};
    double tbest = 1e300;
    for (int v : cand) {
      nshe_tuning t = best;
      t.ks_chunk = v;
      rc = time_kinds(c, t, w, n_t, 2, st, ms);
      if (rc) { c->tune = start; return rc; }
      if (ms[K_KS_MAC] < tbest) { tbest = ms[K_KS_MAC]; best.ks_chunk = v; }
    }
  }
  if (c->log2n == 15) {
    double tbest = 1e300;
    for (int v = 0; v < 2; ++v) {
      nshe_tuning t = best;
      t.split_forward = v;
      rc = time_kinds(c, t, w, n_t, 2, st, ms);
      if (rc) { c->tune = start; return rc; }
      // the split changes the key-switch product too (parity digits)
      const double tt = ms[K_NTT_FWD] + ms[K_NTT_DIGIT] + ms[K_KS_MAC];
      if (tt < tbest) { tbest = tt; best.split_forward = v; }
    }
  }
  // (the fused key switch exists for one-prime digits only)
  if (c->log2n == 15 && best.split_forward && c->alpha == 1) {
    double tt[2];
    for (int v = 0; v < 2; ++v) {
      nshe_tuning t = best;
      t.ks_fused = v;
      rc = time_kinds(c, t, w, n_t, 2, st, ms);
      if (rc) { c->tune = start; return rc; }
      tt[v] = v ? ms[K_KS_FUSED] : ms[K_NTT_DIGIT] + ms[K_KS_MAC];
    }
    best.ks_fused = tt[1] < tt[0] ? 1 : 0;
  }
  {
    const int cand[] = {64, 128, 256};
    double tbest = 1e300;
    for (int v : cand) {
      nshe_tuning t = best;
      t.ew_block = v;
      rc = time_kinds(c, t, w, n_t, 2, st, ms);
      if (rc) { c->tune = start; return rc; }
      const double tt = ms[K_LIFT] + ms[K_SCALE] + ms[K_MODDOWN];
      if (tt < tbest) { tbest = tt; best.ew_block = v; }
    }
  }
  c->tune = best;

  // 2. wave size: per-ciphertext time of a level for 1, 2, 4, ... up to
  // `fit` ciphertexts; the smallest wave within 1% of the best rate (a
  // wave half as large costs about 2% of the rate, measured)
  std::vector<std::pair<int, double>> rates;
  for (int n = 1;; n = std::min(2 * n, fit)) {
    Ws wn = carve(c, ws, n);
    rc = load_sample(c, wn, sample, n_sample, n, st);
    if (rc) { c->tune = start; return rc; }
    double t = 0.0;
    rc = time_level(c, wn, n, st, &t);
    if (rc) { c->tune = start; return rc; }
    rates.emplace_back(n, t / n);
    if (n == fit) break;
  }
  double rbest = 1e300;
  for (auto& r : rates) rbest = std::min(rbest, r.second);
  for (auto& r : rates)
    if (r.second <= 1.01 * rbest) { best.wave_ct = r.first; break; }
  // two streams: waves of at least 32 where the workspace holds them, so
  // that the batched call's half-waves (16 or more) take turns on them
  if (best.streams == 2 && fit >= 32) best.wave_ct = std::max(best.wave_ct, 32);
  drop_graphs(c);
  c->tune = best;
  if (out) *out = best;
  if (ms_per_ct) *ms_per_ct = rbest;
  return NSHE_OK;
}

int nshe_ntt(nshe_ctx* c, const int64_t* in, int64_t* out, int n_poly, int inverse, void* ws,
             size_t ws_bytes, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (!in || !out || !ws) return fail(NSHE_EINVAL, "null buffer");
  if (n_poly < 0) return fail(NSHE_ESHAPE, "n_poly < 0");
  if (n_poly == 0) return NSHE_OK;
  const size_t need = 2 * (size_t)n_poly * c->L * c->n * sizeof(double);
  if (ws_bytes < need) return fail(NSHE_ENOMEM, "workspace too small (2 n_poly L N doubles)");
  if (inverse) return fail(NSHE_EINVAL, "inverse debug transform not provided");
  if (set_device(c)) return NSHE_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* buf = static_cast<double*>(ws);
  HIPCHK(run_i64_to_dbl_limbs((size_t)n_poly * c->L, c->n, in, buf, c->lp_ext, c->L, c->tb, st));
  double* res = buf + (size_t)n_poly * c->L * c->n;
  NttJob j{};
  j.split = c->tune.split_forward;
  j.base = buf;
  j.out = res;
  j.poly_stride = (size_t)c->L * c->n;
  j.npoly = n_poly;
  j.nlimb = c->L;
  j.limb_prime = c->lp_ext;
  j.count = n_poly * c->L;
  HIPCHK(run_ntt(c->log2n, j, c->tb, 0, st));
  HIPCHK(run_ntt_order(c->log2n, (size_t)n_poly * c->L, res, out, c->lp_ext, c->L, 1, c->tb, st));
  return NSHE_OK;
}

int nshe_profile(nshe_ctx* c, int enable) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  for (auto& r : c->recs) {
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  c->prof = enable != 0;
  return NSHE_OK;
}

int nshe_profile_read(nshe_ctx* c, nshe_kernel_stat* out, int max_stats, int* n_stats) {
  g_err.clear();
  if (check_ctx(c) || !out || !n_stats) return fail(NSHE_EINVAL, "null argument");
  if (set_device(c)) return NSHE_EDEVICE;
  nshe_kernel_stat acc[K_COUNT];
  std::memset(acc, 0, sizeof(acc));
  for (auto& r : c->recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    acc[r.kind].launches += 1;
    acc[r.kind].total_ms += ms;
    acc[r.kind].work += r.work;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  int k = 0;
  for (int i = 0; i < K_COUNT && k < max_stats; ++i) {
    if (!acc[i].launches) continue;
    out[k] = acc[i];
    std::strncpy(out[k].name, kKindName[i], sizeof(out[k].name) - 1);
    ++k;
  }
  *n_stats = k;
  return NSHE_OK;
}

// Reads the counter area (waits for the stream).
static int read_counters(nshe_ctx* c, hipStream_t st, unsigned long long (&h)[MARGIN_COUNT]) {
  HIPCHK(hipMemcpyAsync(h, c->tb.margin, sizeof(h), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h[MARGIN_FAULT]) return fail(NSHE_EDEVICE, "extension-basis lift left its proven range");
  return NSHE_OK;
}

int nshe_margin_events(nshe_ctx* c, uint64_t* count, void* stream) {
  g_err.clear();
  if (check_ctx(c) || !count) return fail(NSHE_EINVAL, "null argument");
  if (set_device(c)) return NSHE_EDEVICE;
  unsigned long long h[MARGIN_COUNT] = {};
  if (int rc = read_counters(c, static_cast<hipStream_t>(stream), h)) return rc;
  uint64_t sum = 0;
  for (int i = 0; i < MARGIN_SITES; ++i) sum += h[i];
  *count = sum;
  return NSHE_OK;
}

int nshe_margin_sites(nshe_ctx* c, uint64_t* counts, int max_counts, int* n_counts,
                      void* stream) {
  g_err.clear();
  if (check_ctx(c) || !counts || !n_counts) return fail(NSHE_EINVAL, "null argument");
  if (set_device(c)) return NSHE_EDEVICE;
  unsigned long long h[MARGIN_COUNT] = {};
  if (int rc = read_counters(c, static_cast<hipStream_t>(stream), h)) return rc;
  const int k = std::min(max_counts, (int)NSHE_MARGIN_SITES);
  static_assert(NSHE_MARGIN_SITES == MARGIN_SITES, "site list");
  for (int i = 0; i < k; ++i) counts[i] = h[i];
  *n_counts = k < 0 ? 0 : k;
  return NSHE_OK;
}

int nshe_reset_margin_events(nshe_ctx* c, void* stream) {
  g_err.clear();
  if (check_ctx(c)) return NSHE_EINVAL;
  if (set_device(c)) return NSHE_EDEVICE;
  HIPCHK(run_fill_u64(c->tb.margin, MARGIN_COUNT, 0, static_cast<hipStream_t>(stream)));
  return NSHE_OK;
}

}  // extern "C"
