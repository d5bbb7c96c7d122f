/*
 * nshe.h - C ABI of the MI355X (gfx950) library for the NSHEDB equality-mask
 * hot path: word-level BFV ciphertext arithmetic on batch-encoded columns.
 *
 * What the calls compute (NSHEDB, arXiv 2602.24271):
 *   - BFV subtraction of two ciphertexts (Sec. 2.1.6, BFV operations);
 *   - one ciphertext multiplication followed by relinearization (Sec. 2.1.6;
 *     Sec. 2.1.2 notes relinearization after each multiplication, and that a
 *     product's depth is max(depth(A), depth(B)) + 1);
 *   - the equality mask EQ(x, y) = 1 - (x - y)^(p-1) (Eq. eq:equality),
 *     evaluated by exponentiation by squaring with ceil(log2(p-1))
 *     multiplications (Sec. 4.3.1, equality checks; Table table:noise_levels).
 *     For the paper's p = t = 65537 (Sec. 5.1) this is 16 squarings.
 *
 * Every result is an exact integer function of the inputs (the textbook
 * BFV evaluation):
 *   multiply     lift both operands' coefficients to (-Q/2, Q/2), form
 *                d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 exactly in
 *                Z[X]/(X^N + 1), output c_k = [round(t d_k / Q)]_Q;
 *   relinearize  digits D_j = [c2]_{Q_j} in [0, Q_j), u_b = sum_j D_j evk_j[b],
 *                output [c_b + round(u_b / P)]_Q, where digit j covers alpha
 *                consecutive data primes (Q_j their product; Q_j = q_j when
 *                alpha = 1) and P is the product of the alpha special
 *                primes (hybrid key switching, Han and Ki, CT-RSA 2020);
 *   EQ           z = [x - y]_Q, z <- relin(z * z) (t - 1 = 2^k times k),
 *                out = ([-z0 + Delta e_0]_Q, [-z1]_Q) with Delta = floor(Q/t)
 *                (the trivial encryption of the constant 1, minus z).
 * The device never holds the secret key (the trusted-client split of
 * Sec. 3, system overview): keys are generated and data encrypted and
 * decrypted by the caller.
 *
 * Data layout (the exchange format):
 *   ciphertext  int64 [n_ct][2][L][N]  residues in [0, q_i), coefficient
 *               domain, natural coefficient order, limb i belongs to q_i;
 *   relin key   int64 [dnum][2][L+alpha][N]  digit j < dnum = L / alpha,
 *               component b (b = 0 is [-a_j s + e_j + P g_j s^2]_{PQ},
 *               g_j = (Q/Q_j) [(Q/Q_j)^-1]_{Q_j}; b = 1 is a_j), limbs in
 *               the order q_0 .. q_{L-1}, P_0 .. P_{alpha-1}; coefficient
 *               domain.
 * Pointers named *_dev are device memory of the context's HIP device;
 * pointers named *_host are host memory.  The caller owns every buffer
 * passed in; the library borrows it for the duration of the work enqueued
 * on the given stream and keeps no reference afterwards (except the relin
 * key, which is copied).  The library owns only its context (tables and the
 * transformed relinearization key).
 *
 * Workspace: calls that take (ws_dev, ws_bytes) need a caller-allocated
 * device scratch area of at least nshe_workspace_bytes(ctx, n_ct) bytes,
 * 256-byte aligned; the library allocates nothing on these paths.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  All work is
 * enqueued asynchronously; results are valid after the stream synchronises.
 *
 * Errors: every int-returning call returns NSHE_OK (0) or a negative code;
 * nshe_last_error() gives a message for the calling thread.  Arguments are
 * validated on the host before any work is enqueued (null pointers, sizes,
 * alignment, parameter ranges, the depth budget); a rejected call enqueues
 * nothing.  Residues are range-checked on the device only under the debug
 * switch NSHE_DEBUG_CHECK_INPUTS (otherwise residues outside [0, q_i) give
 * undefined - but memory-safe - results).  Asynchronous device faults are
 * reported by the next synchronising HIP call.  No C++ exception crosses
 * the ABI.  Calls on one context from several host threads must not
 * overlap.
 */
#ifndef NSHE_H
#define NSHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSHE_OK 0
#define NSHE_EINVAL -1   /* bad argument (null pointer, bad size, bad prime) */
#define NSHE_ESHAPE -2   /* sizes inconsistent with the context */
#define NSHE_ENOMEM -3   /* workspace too small, or context allocation failed */
#define NSHE_EDEVICE -4  /* a HIP runtime call failed */
#define NSHE_EDEPTH -5   /* the operation's multiplicative depth exceeds the
                            context's depth budget (see nshe_budget) */
#define NSHE_ENOKEY -6   /* relinearization (or Galois) key not set */
#define NSHE_EUNSUPPORTED -7 /* not defined for these parameters: EQ needs
                            t - 1 = 2^k, comparisons a prime t = 2^K + 1,
                            slot operations t = 1 (mod 2N) */

#define NSHE_MAX_L 24        /* data primes */
#define NSHE_MAX_LOG2N 15    /* ring degree up to 32768 */
#define NSHE_MIN_LOG2N 3

typedef struct nshe_ctx nshe_ctx;

/* BFV parameters (Sec. 5.1: n = 32768, log Q = 881, t = 65537).
 *   log2_n  ring degree N = 2^log2_n, NSHE_MIN_LOG2N..NSHE_MAX_LOG2N;
 *   t       plaintext modulus, odd, 2 < t < 2^24, coprime to every prime;
 *   L       number of data primes: 2, 3, 4, 8, 12, 15, 16, 17, 20 or 24 (the
 *           counts the base-conversion kernels are built for; the paper's
 *           18-prime modulus gives 17, 16 or 15 with 1, 2 or 3 special
 *           primes);
 *   q_host  L distinct primes, each in [2^48, 2^49) and = 1 (mod 2N);
 *   P       the (first) special prime, same constraints, distinct from the q_i;
 *   alpha   data primes per key-switching digit = number of special primes:
 *           1 (0 reads as 1: one digit per data prime, a single special
 *           prime), 2 (L one of 2, 4, 8 or 16) or 3 (L one of 3, 12 or 15);
 *   P1, P2  the second and third special primes when alpha >= 2, 3
 *           (ignored otherwise).
 * Q = prod q_i, P = P P1 P2 (as many as alpha).  The library picks its own
 * extension basis (primes of the same form below every q_i and special
 * prime) large enough for exact products. */
typedef struct {
  uint32_t log2_n;
  uint64_t t;
  int32_t L;
  const uint64_t* q_host;
  uint64_t P;
  int32_t alpha;
  uint64_t P1;
  uint64_t P2;
} nshe_params;

/* Read-only description of a context (sizes for the caller's buffers). */
typedef struct {
  uint32_t n;            /* ring degree N */
  int32_t L;             /* data primes */
  int32_t L_ext;         /* extension primes chosen by the library */
  int32_t squarings;     /* k with t - 1 = 2^k, or -1 */
  uint64_t ext_primes[32];
  size_t ct_words;       /* int64 words of one ciphertext: 2 * L * N */
  size_t relin_key_words;/* int64 words of the relin key (and of a Galois
                            key): dnum * 2 * (L+alpha) * N */
  int32_t depth_budget;  /* multiplications a fresh ciphertext takes (nshe_budget) */
  int32_t lt_depth;      /* depth of the comparison program, -1 without one */
  double fresh_bits;     /* noise budget of a fresh encryption, bits */
  double level_bits;     /* bits one multiplication costs (the model's) */
  int32_t alpha;         /* data primes per key-switching digit (special primes) */
  int32_t dnum;          /* key-switching digits, L / alpha */
} nshe_info;

/* Noise budget and multiplicative depth (Sec. 2.1.2: every multiplication
 * adds and amplifies noise, and depth(A x B) = max(depth(A), depth(B)) + 1;
 * Table table:noise_levels gives each operator's depth).  A ciphertext
 * decrypts correctly while log2(Q / (2 |t (c0 + c1 s) - Q m|)) > 0.  The
 * library's model (an average-case estimate, not a worst-case bound):
 *   fresh_bits = log2 Q - log2(2 t (19 + t))   (client errors |e| <= 19:
 *                a rounded Gaussian of sigma 3.2 clipped at 6 sigma, and a
 *                ternary secret);
 *   level_bits = log2 t + log2 N + 2           per multiplication with
 *                relinearization (one bit above the canonical-embedding
 *                growth t N sqrt(8/3));
 *   depth_budget = floor((fresh_bits - 8) / level_bits), >= 0.
 * It stays below the exact noise the test oracle measures at every level
 * of the EQ chain.  At the paper's parameters (Sec. 5.1) it gives 799.1,
 * 33 and 23.  nshe_budget_of needs no device (host arithmetic only). */
typedef struct {
  int32_t depth_budget;
  int32_t lt_depth;      /* depth of the comparison program, -1 without one */
  double fresh_bits;
  double level_bits;
} nshe_budget;
int nshe_budget_of(const nshe_params* params, nshe_budget* out_host);

/* Depth an operation adds to its inputs (for fresh inputs, the whole
 * result's depth):
 *   NSHE_OP_ADD        sub, add, sum, rotate, sum_slots: 0 (rotations'
 *                      key switching adds noise, not depth);
 *   NSHE_OP_MUL        multiply, square_relin, mul_relin (SELECT): 1;
 *   NSHE_OP_MUL_PLAIN  mul_plain, extract (a plaintext product with
 *                      coefficients up to t/2): 1;
 *   NSHE_OP_EQ         eq_mask, eq_mask_batched (GROUP BY): k, t - 1 = 2^k;
 *   NSHE_OP_IN         in_mask with arg = k members: EQ + 1 if k > 1 (the
 *                      k-way sum, the paper's ceil(log(k)/p));
 *   NSHE_OP_LT         compare (LT, LE): the program's depth (lt_depth,
 *                      18 at p = 65537) + 1 for its scalar combination;
 *   NSHE_OP_BETWEEN    between: LT + 1;
 *   NSHE_OP_JOIN       join_sum: EQ + 1 (Table table:noise_levels) + 1 for
 *                      the plaintext product inside Broadcast.
 * Every call with a fixed depth (all but the additions) returns
 * NSHE_EDEPTH, enqueuing nothing, when that depth on fresh inputs exceeds
 * the budget.  The library cannot see an input's history: a caller that
 * chains calls keeps a depth per ciphertext and asks nshe_depth_after,
 * which returns NSHE_EDEPTH (and still sets *out_depth) when
 * in_depth + the operation's depth exceeds the budget.  NSHE_EUNSUPPORTED
 * names an operation these parameters do not have. */
#define NSHE_OP_ADD 0
#define NSHE_OP_MUL 1
#define NSHE_OP_MUL_PLAIN 2
#define NSHE_OP_EQ 3
#define NSHE_OP_IN 4
#define NSHE_OP_LT 5
#define NSHE_OP_BETWEEN 6
#define NSHE_OP_JOIN 7

/* Create a context on HIP device `hip_device`: validates the parameters,
 * selects the extension basis and uploads its tables (this call allocates
 * device memory; none of the evaluation calls below do). */
int nshe_ctx_create(const nshe_params* params, int hip_device, nshe_ctx** out);
int nshe_ctx_destroy(nshe_ctx* ctx);
int nshe_ctx_info(const nshe_ctx* ctx, nshe_info* out);
int nshe_op_depth(const nshe_ctx* ctx, int op, int arg, int* depth_host);
int nshe_depth_after(const nshe_ctx* ctx, int op, int arg, int in_depth, int* out_depth_host);

/* Install the relinearization key (Sec. 2.1.2).  Copies and transforms
 * `evk_dev` (layout above; n_words must be dnum * 2 * (L+alpha) * N, else
 * NSHE_ESHAPE) into context-owned memory on `stream` and waits for it;
 * `evk_dev` may be freed on return.  Allocates the context-owned key store
 * on first use and a temporary of the same size during the call (set-up,
 * not the evaluation path). */
int nshe_set_relin_key(nshe_ctx* ctx, const int64_t* evk_dev, size_t n_words, void* stream);

/* Device scratch needed by the evaluation calls for n_ct ciphertexts. */
size_t nshe_workspace_bytes(const nshe_ctx* ctx, int n_ct);

/* out = [x - y]_Q, component-wise, for n_ct ciphertext pairs (Sec. 2.1.6).
 * out may alias x or y. */
int nshe_sub(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* y_dev,
             int64_t* out_dev, int n_ct, void* stream);

/* out = relin(in * in): one squaring level of the EQ chain (Sec. 4.3.1).
 * out may alias in. */
int nshe_square_relin(nshe_ctx* ctx, const int64_t* in_dev, int64_t* out_dev,
                      int n_ct, void* ws_dev, size_t ws_bytes, void* stream);

/* out = relin(a * b) (Sec. 2.1.6 multiplication; SELECT and AND, Eq.
 * eq:select and Table tab:operator-support, are this call). */
int nshe_mul_relin(nshe_ctx* ctx, const int64_t* a_dev, const int64_t* b_dev,
                   int64_t* out_dev, int n_ct, void* ws_dev, size_t ws_bytes,
                   void* stream);

/* The three-component product before relinearization: out3 is int64
 * [n_ct][3][L][N] = ([round(t d_k / Q)]_Q)_{k=0,1,2}. */
int nshe_multiply(nshe_ctx* ctx, const int64_t* a_dev, const int64_t* b_dev,
                  int64_t* out3_dev, int n_ct, void* ws_dev, size_t ws_bytes,
                  void* stream);

/* Relinearization alone: in3 int64 [n_ct][3][L][N] -> out [n_ct][2][L][N]. */
int nshe_relinearize(nshe_ctx* ctx, const int64_t* in3_dev, int64_t* out_dev,
                     int n_ct, void* ws_dev, size_t ws_bytes, void* stream);

/* EQ(x, y) = 1 - (x - y)^(t-1) (Eq. eq:equality) for n_ct ciphertexts:
 * x is [n_ct][2][L][N]; y is the same shape, or one ciphertext broadcast to
 * every x when y_broadcast != 0 (an encrypted predicate constant).  Requires
 * t - 1 = 2^k (k squarings).  out may alias x (not y when broadcast).
 * From 32 ciphertexts on, the call runs its two halves on two streams
 * (tuning streams, see nshe_tuning); it stays ordered on `stream`. */
int nshe_eq_mask(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* y_dev,
                 int64_t* out_dev, int n_ct, int y_broadcast, void* ws_dev,
                 size_t ws_bytes, void* stream);

/* EQ for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as nshe_eq_mask, with the library's own scratch,
 * a file-scope device array of NSHE_NOALLOC_SCRATCH_BYTES (160 MiB) that
 * each GPU the library runs on holds until the process ends.  It holds
 * n_ct ciphertexts' workspace when n_ct * nshe_workspace_bytes(ctx, 1) fits
 * in it (one ciphertext at N = 32768 with 17 primes, eight at N = 4096);
 * larger calls return NSHE_ENOMEM before any work.  The caller passes inputs
 * and outputs only.  Every call on one GPU, from any context, uses that
 * GPU's one scratch, so calls that overlap on a GPU race: serialise them
 * (one stream, or events between streams).  Nothing in the scratch needs to
 * start at zero (every value is written before it is read); it keeps the
 * last call's contents.  The call makes no hipMalloc, hipFree or other
 * allocating call and records no profiling events. */
#define NSHE_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
int nshe_eq_mask_noalloc(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* y_dev,
                         int64_t* out_dev, int n_ct, int y_broadcast, void* stream);

/* Batched EQ over instances of uneven size: item i has n_ct ciphertexts.
 * The items' ciphertexts are processed together, in waves of at most
 * `wave_ct` ciphertexts, with one
 * shared pass over the relinearization key per squaring and wave.  When
 * use_graph != 0 the whole chain of a wave is captured once into a HIP graph
 * and replayed; the graph reads its wave's ciphertext pointers from a table
 * in the workspace (filled by small kernels at the start of the call), so
 * one graph per wave size serves every wave and every later call with the
 * same workspace and wave size.  Capture runs on a context-owned stream and
 * the graph is launched on `stream` (with tuning streams = 2 and waves of at
 * least 32: half-waves, on `stream` and the context's second stream in
 * turn, one graph per stream and half-wave size).  ws_bytes must cover
 * nshe_batched_workspace_bytes(ctx, wave size, total ciphertexts); with
 * wave_ct = 0 the wave is the tuned one, capped by what ws_bytes holds. */
typedef struct {
  const int64_t* x_dev;
  const int64_t* y_dev;
  int64_t* out_dev;
  int32_t n_ct;
  int32_t y_broadcast;
} nshe_item;

/* Workspace bytes for nshe_eq_mask_batched with waves of wave_ct
 * ciphertexts over total_ct ciphertexts in all: one wave's ciphertext
 * workspace, a wave counter and a table of 24-byte per-ciphertext pointers
 * (total_ct + wave_ct entries).  0 on a bad argument. */
size_t nshe_batched_workspace_bytes(const nshe_ctx* ctx, int wave_ct, long long total_ct);

int nshe_eq_mask_batched(nshe_ctx* ctx, const nshe_item* items_host,
                         int n_items, int wave_ct, int use_graph, void* ws_dev,
                         size_t ws_bytes, void* stream);

/* BFV addition (Sec. 2.1.6): out = [a + b]_Q per residue, int64
 * [n_ct][2][L][N] canonical residues.  No workspace. */
int nshe_add(nshe_ctx* ctx, const int64_t* a_dev, const int64_t* b_dev,
             int64_t* out_dev, int n_ct, void* stream);

/* Sum of k ciphertext arrays: in_dev is int64 [k][n_ct][2][L][N], out_dev
 * [n_ct][2][L][N] = [sum_j in[j]]_Q.  k = 0 writes the encryption (0, 0).
 * BFV addition is exact per residue, so the order of the sum does not
 * change the result. */
int nshe_sum(nshe_ctx* ctx, const int64_t* in_dev, int k, int64_t* out_dev,
             int n_ct, void* stream);

/* Set membership, IN(x, S) = sum over y in S of EQ(x, y) (Eq. eq:in,
 * Sec. 4.2.2, range and set queries): x_dev is one column of n_ct
 * ciphertexts, set_dev holds the k members as k single ciphertexts
 * (int64 [k][2][L][N], each broadcast over the column).  With distinct
 * members out_dev decrypts to the indicator [x in S]; a member given twice
 * counts twice.  The k equality masks run as one batched call (waves of
 * wave_ct ciphertexts, 0 = the tuned wave else 32; use_graph as for
 * nshe_eq_mask_batched) into the workspace, then are summed.  GROUP BY
 * (one mask per group value, Sec. 4.2.2) is nshe_eq_mask_batched with items
 * (x, value_j, out_j, n_ct, y_broadcast = 1).  ws_bytes must cover
 * nshe_in_workspace_bytes(ctx, n_ct, k, wave_ct). */
size_t nshe_in_workspace_bytes(const nshe_ctx* ctx, int n_ct, int k, int wave_ct);
int nshe_in_mask(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* set_dev, int k,
                 int64_t* out_dev, int n_ct, int wave_ct, int use_graph,
                 void* ws_dev, size_t ws_bytes, void* stream);

/* Range comparisons (Eq. eq:inequality; BETWEEN, Sec. 4.2.2).  LT(x, y) is
 * the sum over a in A = {-(p-1)/2, ..., -1} of 1 - (x - y - a)^(p-1), i.e.
 * the encrypted indicator of x - y in the negative half of Z_p: [x < y] when
 * |x - y| <= (p-1)/2 (larger differences wrap around).  It is evaluated as
 * one polynomial f(z) = c_(p-1) z^(p-1) + z g(z^2), z = x - y, whose
 * coefficients the context derives from t (a prime 2^K + 1, else
 * NSHE_EDEPTH), by a fixed program every result follows exactly:
 *   levels[a] = z^(2^a) by K squarings (a = 0..K);
 *   w = levels[1]; k = 2^floor(K/2) babies B_i = w^i (B_0 = (Delta, 0),
 *   powers of two from the levels, others B_h * B_(i-h) with h the largest
 *   power of two below i); m = 2^(K-1)/k giants W_j = w^(k j) (powers of
 *   two from the levels, others W_h * W_(j-h));
 *   G_j = sum_i c_(2(jk+i)+1) B_i with centred coefficients (scalar
 *   products, exact mod Q); g = G_0 + sum_{j>=1} G_j * W_j;
 *   LT = c_(p-1) levels[K] + z * g,
 * every product a multiplication followed by relinearization (as
 * nshe_mul_relin / nshe_square_relin), except that the m - 1 products
 * G_j * W_j have their exact tensors added and their sum scaled, rounded
 * and relinearized once.  op 0 gives LT(x, y); op 1 gives
 * LE(x, y) = (Delta, 0) - LT(y, x).  nshe_between gives
 * LE(lo, x) * LE(x, hi) (one more multiplication).  y (or lo and hi) may be
 * one ciphertext broadcast over the column.  Workspace:
 * nshe_compare_workspace_bytes(ctx, n_ct) (about K + k + m + 27 ciphertext
 * arrays, one operand's transform, one summed tensor and the multiply
 * workspace; 0 if the context has no comparison polynomial). */
#define NSHE_CMP_LT 0
#define NSHE_CMP_LE 1
size_t nshe_compare_workspace_bytes(const nshe_ctx* ctx, int n_ct);
int nshe_compare(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* y_dev, int y_broadcast,
                 int op, int64_t* out_dev, int n_ct, void* ws_dev, size_t ws_bytes,
                 void* stream);
int nshe_between(nshe_ctx* ctx, const int64_t* x_dev, const int64_t* lo_dev,
                 const int64_t* hi_dev, int bounds_broadcast, int64_t* out_dev, int n_ct,
                 void* ws_dev, size_t ws_bytes, void* stream);

/* Plaintext products, Extract and Broadcast (the derived operations of
 * Sec. 2.1.6) and the fused equi-join aggregation (Sec. 4.2.2, JOIN).
 *   nshe_mul_plain  out = ([c0 m]_Q, [c1 m]_Q) for the plaintext polynomial
 *                   m (int64 [N], coefficients in [0, t), taken as centred
 *                   representatives), exact in Z[X]/(X^N + 1);
 *   nshe_extract    the product with the basis plaintext of `slot` (slot
 *                   order as for rotations: its polynomial is
 *                   N^-1 zeta^-i mod t, zeta the slot's root psi^(+-3^s));
 *                   with broadcast != 0 followed by nshe_sum_slots, which
 *                   puts that slot's value in every slot (needs the Galois
 *                   keys);
 *   nshe_join_sum   for the fact-table key column a_key (n_ct ciphertexts)
 *                   and one reference ciphertext each of keys and of an
 *                   attribute: sum over the given reference rows j of
 *                   EQ(a_key, bcast(b_key, j)) * bcast(b_attr, j); with
 *                   unique reference keys each fact row decrypts to the
 *                   attribute of its matching row among them, else 0.
 * All need t = 1 (mod 2N) (the batched slots).  Workspace:
 * nshe_workspace_bytes(ctx, n_ct) for the first two,
 * nshe_join_workspace_bytes(ctx, n_ct) for the join. */
int nshe_mul_plain(nshe_ctx* ctx, const int64_t* in_dev, const int64_t* pt_dev,
                   int64_t* out_dev, int n_ct, void* ws_dev, size_t ws_bytes, void* stream);
int nshe_extract(nshe_ctx* ctx, const int64_t* in_dev, int slot, int broadcast,
                 int64_t* out_dev, int n_ct, void* ws_dev, size_t ws_bytes, void* stream);
size_t nshe_join_workspace_bytes(const nshe_ctx* ctx, int n_ct);
int nshe_join_sum(nshe_ctx* ctx, const int64_t* a_key_dev, const int64_t* b_key_dev,
                  const int64_t* b_attr_dev, const int32_t* rows_host, int n_rows,
                  int64_t* out_dev, int n_ct, void* ws_dev, size_t ws_bytes, void* stream);

/* Slot rotations and the rotate-and-add aggregation (COUNT and SUM,
 * Sec. 4.2.2, aggregation).  Slots follow the 2 x N/2 layout: slot s < N/2 is
 * the plaintext's value at psi^(3^s), slot N/2 + s at psi^(-3^s) (psi a
 * primitive 2N-th root of unity mod t), so the automorphism X -> X^g with
 * g = 3^r mod 2N rotates each half left by r and g = 2N - 1 swaps the
 * halves.  A rotation applies X -> X^g to both components and switches the
 * second from sigma_g(s) back to s with the Galois key of g:
 *   key_g  int64 [dnum][2][L+alpha][N], digit j = ([-a_j s + e_j + P g_j
 *          sigma_g(s)]_{PQ}, a_j) (the relin key's format with sigma_g(s)
 *          in place of s^2, n_words as for the relin key); copied and
 *          transformed into context memory (waits for `stream`; allocates
 *          on the first key for g);
 *   out    = ([sigma_g(c0) + round(sum_j D_j b_j / P)]_Q,
 *             [round(sum_j D_j a_j / P)]_Q), D_j = [sigma_g(c1)]_{Q_j}.
 * nshe_sum_slots replaces each ciphertext by ct + rot(ct) for the Galois
 * elements nshe_galois_elements lists (rotations by N/4, ..., 1, then the
 * swap): every slot of the result holds the sum of all slots.  COUNT is
 * nshe_sum_slots of a 0/1 mask, SUM nshe_sum_slots of a column times the
 * mask (nshe_mul_relin).  Workspace: nshe_workspace_bytes(ctx, n_ct).
 * NSHE_ENOKEY names a missing Galois key.  nshe_sum_slots runs the two
 * halves of 32 or more ciphertexts on two streams (tuning streams). */
int nshe_set_galois_key(nshe_ctx* ctx, uint32_t g, const int64_t* key_dev, size_t n_words,
                        void* stream);
int nshe_galois_elements(const nshe_ctx* ctx, uint32_t* out_host, int max_out, int* n_out_host);
int nshe_rotate(nshe_ctx* ctx, const int64_t* in_dev, uint32_t g, int64_t* out_dev,
                int n_ct, void* ws_dev, size_t ws_bytes, void* stream);
int nshe_sum_slots(nshe_ctx* ctx, const int64_t* in_dev, int64_t* out_dev, int n_ct,
                   void* ws_dev, size_t ws_bytes, void* stream);

/* Launch shapes and the autotuner.  Results never depend on the tuning
 * (every kernel computes the same exact integers); only the speed does.
 *   ks_chunk       ciphertexts accumulated per pass over the relinearization
 *                  key in the key-switch inner product: 4, 8, 16 or 32
 *                  (at most 16 are used with digit transforms by parity);
 *   split_forward  1: each 2^15-point forward transform runs as two
 *                  workgroups: one per output half, and for the key-switch
 *                  digits one per coefficient parity (two 2^14-point
 *                  transforms whose last radix-2 stage the key-switch
 *                  product applies); 0: one workgroup per limb (ignored
 *                  for smaller N);
 *   ew_block       threads per workgroup of the per-coefficient kernels
 *                  (base lift, scale-and-round, mod-down): 64, 128 or 256;
 *   wave_ct        ciphertexts per wave of nshe_eq_mask_batched when its
 *                  wave_ct argument is 0 (0: as many as the workspace holds);
 *   ks_fused       1: at N = 32768 with split_forward, the key-switch
 *                  product runs fused with the digit transforms (one
 *                  kernel; the digits' transforms are never written),
 *                  0: digit transforms, then the product (two kernels);
 *   streams        2: nshe_eq_mask and nshe_sum_slots with at least 32
 *                  ciphertexts run the first half of them on `stream` and
 *                  the second half on a second stream the context owns
 *                  (non-blocking, default priority), each in its own half
 *                  of the workspace, so
 *                  that one half's kernels fill the GPU while the other's
 *                  drain; nshe_eq_mask_batched with waves of at least 32
 *                  runs half-waves, taking turns between the two streams
 *                  (each with its own half of the wave's workspace).  The
 *                  second stream starts after the work already on `stream`
 *                  and `stream` waits for it at the end (events), so the
 *                  call stays ordered on `stream`.  Not while profiling,
 *                  while `stream` is being captured into a graph, or in
 *                  nshe_eq_mask_noalloc.  1: one stream.
 * A new context starts at {32, 1, 128, 0, 0, 2}.  nshe_set_tuning validates the
 * values (NSHE_EINVAL otherwise) and drops the batched call's cached graphs.
 *
 * nshe_autotune measures, on the caller's sample ciphertexts (int64
 * [n_sample][2][L][N], repeated cyclically to fill larger trials), squaring
 * levels of the EQ chain with HIP events: first ks_chunk, split_forward,
 * ks_fused and ew_block one at a time (each judged by the event time of the
 * kernels it shapes, on min(32, wave limit) ciphertexts), then the per-ciphertext
 * time of a level at 1, 2, 4, ... ciphertexts up to the wave limit
 * (max_wave_ct if > 0, and what ws_bytes holds), keeping the smallest wave
 * within 1% of the best rate (with streams = 2, at least 32 where that many
 * fit: the batched call's half-waves).  The result becomes the context's tuning and
 * is copied to *out_host (if not NULL); *ms_per_ct_host (if not NULL)
 * receives the best per-ciphertext level time in ms.  Needs the relin key.
 * The workspace contents are overwritten; the sample is only read.  The
 * call synchronises `stream` several times; profiling records and the
 * profiling flag of the caller are kept aside and restored. */
typedef struct {
  int32_t ks_chunk;
  int32_t split_forward;
  int32_t ew_block;
  int32_t wave_ct;
  int32_t ks_fused;
  int32_t streams;
} nshe_tuning;

int nshe_get_tuning(nshe_ctx* ctx, nshe_tuning* out_host);
int nshe_set_tuning(nshe_ctx* ctx, const nshe_tuning* in_host);
int nshe_autotune(nshe_ctx* ctx, const int64_t* sample_dev, int n_sample,
                  int max_wave_ct, void* ws_dev, size_t ws_bytes, void* stream,
                  nshe_tuning* out_host, double* ms_per_ct_host);

/* Negacyclic NTT (debug/parity entry): for each of n_poly polynomials of L
 * data-prime limbs (int64 [n_poly][L][N], residues in [0, q_i)), out holds
 * the evaluations at psi_i^(2j+1), j = 0..N-1, in natural j order, where
 * psi_i = g^((q_i - 1) / 2N) for the smallest primitive root g of q_i.
 * The workspace must hold 2 * n_poly * L * N doubles.  Only the forward
 * transform is exposed: inverse != 0 returns NSHE_EINVAL. */
int nshe_ntt(nshe_ctx* ctx, const int64_t* in_dev, int64_t* out_dev,
             int n_poly, int inverse, void* ws_dev, size_t ws_bytes,
             void* stream);

/* Exactness monitor.  The centred lift between residue bases decides an
 * overflow count from a floating-point estimate; when the estimate falls
 * within its proven error bound of a decision boundary the library takes
 * an exact mixed-radix comparison instead and counts the event here.
 * Results are exact either way.  (Synchronises `stream` to read.) */
int nshe_margin_events(nshe_ctx* ctx, uint64_t* count_host, void* stream);
int nshe_reset_margin_events(nshe_ctx* ctx, void* stream);

/* The same events per call site of the lift (counts_host[i] for site i,
 * min(max_counts, NSHE_MARGIN_SITES) entries, *n_counts_host set):
 *   0  a squaring's operand lift not fused into the kernel before it
 *      (k_lift: the levels without the split transforms)
 *   1  the scale-and-round's lift of [t d]_Q
 *   2  the same after the split inverse (N = 2^15)
 *   3  the mod-down fused with the next squaring's lift
 *   4  the subtraction fused with the first squaring's lift
 *   5  the lift of a product's int64 operands
 * (Synchronises `stream`.) */
#define NSHE_MARGIN_SITES 6
int nshe_margin_sites(nshe_ctx* ctx, uint64_t* counts_host, int max_counts, int* n_counts_host,
                      void* stream);

/* Test and debugging switches (off in a new context; not for production):
 *   NSHE_DEBUG_WIDE_LIFT_WINDOW  the lift takes its exact decision whenever
 *     its estimate S lies within 1/4 of a half-integer instead of 2^-40:
 *     floor(S) is still exact there, so results do not change, and about
 *     half of all coefficients go through the exact path (and are counted);
 *   NSHE_DEBUG_CHECK_INPUTS  every call that reads int64 ciphertexts first
 *     checks on the device that each residue lies in [0, q_i) and returns
 *     NSHE_EINVAL, enqueuing nothing more, if one does not (synchronises
 *     the stream; keys and plaintexts are not checked).
 * Setting the switches drops the batched call's captured graphs. */
#define NSHE_DEBUG_WIDE_LIFT_WINDOW 1u
#define NSHE_DEBUG_CHECK_INPUTS 2u
int nshe_set_debug(nshe_ctx* ctx, uint32_t flags);

/* Kernel timing.  nshe_profile(ctx, 1) starts recording a pair of HIP
 * events on the call's stream around every kernel launch of subsequent
 * non-graph calls (clearing earlier records); nshe_profile(ctx, 0) stops.
 * nshe_profile_read waits for the recorded events and returns, per kernel
 * kind, the launch count, the summed event time and the summed algorithmic
 * work: butterflies for the transform kinds (ntt_fwd, ntt_inv, ntt_digit;
 * N/2 log2 N per limb), coefficient-limbs or coefficients for the others.
 * Reading clears the records. */
typedef struct {
  char name[24];
  uint64_t launches;
  double total_ms;
  double work;
} nshe_kernel_stat;

int nshe_profile(nshe_ctx* ctx, int enable);
int nshe_profile_read(nshe_ctx* ctx, nshe_kernel_stat* stats_host, int max_stats,
                      int* n_stats_host);

/* Message for the last error on the calling thread ("" if none). */
const char* nshe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NSHE_H */
