/*
 * montexp.h -- C ABI of libmontexp.so: batched Montgomery modular
 * multiplication / squaring with truncated reduction and constant-time
 * fixed-window modular exponentiation on AMD MI355X (gfx950).
 *
 * Paper: "Truncated multiplication and batch software SIMD AVX512
 * implementation for faster Montgomery multiplications and modular
 * exponentiation" (Didier, El Mrabet, Glandus, Robert).
 *
 * Conventions for every entry point:
 *  - Multiprecision values are little-endian arrays of uint64_t words (the
 *    GMP mpn order the paper's exponentiation takes, Section 6, Algorithm 7).
 *    Instance i of a batch starts at ptr + i * words.
 *  - Operand pointers are DEVICE pointers unless the name says _host.
 *    `stream` is a hipStream_t (NULL = the default stream).  Batch calls
 *    only enqueue work: results are valid after the stream synchronises.
 *  - Size classes: bits in {64, 128, 256, 512, 1024, 2048, 3072, 4096}.  A
 *    class uses n limbs of 28 bits, n = ceil((bits + 2) / 28) rounded up to a
 *    multiple of 37 above 2048 bits, and R = 2^(28 n) >= 4 * 2^bits (r_bits =
 *    28 n, reported by mont_ctx_query), so products of values below 2N reduce
 *    to values below 2N with no final subtraction (Section 4).
 *  - Canonical values (< N) use words = ceil(bits / 64); Montgomery-domain
 *    values (< 2N) use mont_words = ceil(r_bits / 64).
 *  - The caller owns all operand buffers and the stream; the library owns
 *    context memory and the context's workspace.  Only mont_ctx_init,
 *    mont_ctx_reserve, the mixed plan's create call and the autotuner
 *    allocate device memory; the batch calls never allocate and never wait
 *    for the device.
 *  - Streams: a context's constants are read-only once initialised.  Calls
 *    that use its library workspace (block-kernel single operations,
 *    modexp_batch, rsa_crt_batch on ctx_p) may come from several host
 *    threads and streams:
 *    each makes its stream wait for the workspace's previous user (an event),
 *    so they take turns on the device.  Calls with a caller workspace
 *    (modexp_batch_ws, rsa_crt_batch_ws) are independent of each other.
 *  - Errors: host-checkable arguments give MX_EINVAL synchronously (also a
 *    launch refused before it is enqueued because the workspace does not hold
 *    its tiles); launch or device errors give MX_EDEVICE; mont_last_error()
 *    returns a thread-local message for the last non-OK status.  No call
 *    aborts.
 *  - Device-data preconditions (a, b < 2N; base < N) are checked only on
 *    request (MX_CHECK_INPUTS, a debugging aid); unchecked, a violation gives
 *    an unspecified value, never an out-of-bounds access.  ctx_idx entries
 *    >= the context count are replaced by 0.
 *  - Compared with the call list of the hot path: mont_ctx_query also
 *    returns the limb width, mont_ctx_export also returns R mod N, and the
 *    mixed-size launch is a plan (mx_mixed_plan_*) built once and launched
 *    or replayed from a HIP graph, in place of one call over caller-built
 *    job descriptors.
 */
#ifndef MONTEXP_H
#define MONTEXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mont_ctx mont_ctx; /* opaque, device-resident, immutable after init */

typedef enum {
  MX_OK = 0,
  MX_EINVAL = 1,
  MX_ENOMEM = 2,
  MX_EDEVICE = 3,
  MX_EUNSUPPORTED = 4
} mx_status;

/* flags for the batch calls (OR-ed) */
enum {
  MX_REDC_TRUNC = 0, /* truncated reduction, Section 5 Algorithm 6 (default)  */
  MX_REDC_PLAIN = 1, /* full q*N product, Section 4 Algorithm 3 (B_fma)        */
  MX_IMPL_BLOCK = 2, /* block-level schoolbook over 37-limb blocks for the
                        1024/2048 classes (the only kernels above 2048 bits);
                        same results, MX_EUNSUPPORTED where not built        */
  MX_MUL_KARATSUBA = 4, /* block kernels whose product (A*B or A^2) is one-level
                           Karatsuba over half-size block numbers (Section 3):
                           2048 and 4096 bits; same results                  */
  MX_ONE_LANE = 8,     /* exponentiation with the block kernels: one lane per
                          instance even for batches of at most 32768 (which
                          otherwise run four lanes per instance: lower
                          latency, more lanes); for loaded devices where the
                          other work fills the SIMDs; same results           */
  MX_REDC_CIOS = 16,   /* word-interleaved Montgomery multiplication (Section
                          4, Algorithm 4, CIOS): for each limb a_i, Y += a_i B,
                          q_i = Y_0 N'_0 mod 2^28, Y = (Y + q_i N) / 2^28;
                          same results.  The register-resident classes (<=
                          2048 bits, their default kernels); above 2048 bits
                          the same steps with 37-limb blocks as the words, one
                          lane per instance (MX_TWO_LANES, MX_FOUR_LANES:
                          MX_EUNSUPPORTED); with MX_REDC_PLAIN, MX_EINVAL; not
                          in the mixed launch                                */
  MX_TWO_LANES = 32,   /* exponentiation with the block kernels: at most two
                          lanes per instance (batches of at most 32768 would
                          otherwise run four); with MX_ONE_LANE, MX_EINVAL;
                          same results                                       */
  MX_MUL_KARATSUBA2 = 128, /* mp_mul_batch only: Karatsuba at two levels         */
  MX_FOUR_LANES = 512, /* exponentiation with the block schoolbook kernels: four
                          lanes per instance at any batch size (the default
                          only up to 32768), the lanes' arrays in LDS; in the
                          mixed launch, 3072- and 4096-bit tiles of 16
                          instances; with MX_ONE_LANE or MX_TWO_LANES,
                          MX_EINVAL; same results                            */
  MX_CHECK_INPUTS = 256, /* debugging: before the work, check the device-data
                          preconditions (a, b < 2N for mont_mul_batch and
                          mont_sqr_batch; base < N for the modexp_batch calls)
                          with a small kernel; the call then waits for the
                          stream, and gives MX_EINVAL naming the count and the
                          first offending instance, launching nothing else.
                          The check branches on the data: not for secrets   */
  MX_REDC_KARATSUBA = 64 /* the truncated high half of q N formed by one-level
                          Karatsuba (Section 5, Karatsuba paragraph) from
                          limb-wise half sums, so that every column is the
                          schoolbook's; same results.  Single operations and
                          exponentiation of the register-resident classes
                          (<= 2048 bits) and of the block kernels with an
                          even block count (2048 with MX_IMPL_BLOCK or
                          MX_MUL_KARATSUBA, 4096; one lane per instance,
                          MX_TWO_LANES refused), else MX_EUNSUPPORTED; with
                          another MX_REDC_ flag, MX_EINVAL; not in the mixed
                          launch or rsa_crt_batch                            */
};

/* Montgomery contexts for `count` moduli of size class `bits` (Section 4:
 * N' = (-N)^{-1} mod R, R^2 mod N for conversion into Montgomery form, and
 * R mod N, the Montgomery form of 1).  moduli_host: count * ceil(bits/64)
 * words in host memory; each modulus odd, >= 3 and below 2^bits, else
 * MX_EINVAL (the offending index is in mont_last_error()).  The constants
 * are computed on the device; the call blocks until they are resident.
 * It also allocates the context's workspace: enough for one launch of
 * `count` instances at the class's default window (at most 256 MiB).
 * *out receives the context (NULL on failure); free with mont_ctx_destroy. */
mx_status mont_ctx_init(mont_ctx **out, const uint64_t *moduli_host, uint32_t bits, uint32_t count,
                        void *stream);

/* Grows the context's workspace to at least `bytes` (modexp_ws_bytes,
 * mont_ws_bytes or rsa_crt_ws_bytes give the size a call needs for one
 * launch).  Allocates device memory; first waits for the work already
 * queued on the old workspace (this context's only).  A no-op when the
 * workspace is already large enough.  Not for use during stream capture. */
mx_status mont_ctx_reserve(mont_ctx *ctx, size_t bytes);

/* Size class, r_bits (log2 R), limb bits (28), context count and device bytes.
 * Any output pointer may be NULL. */
mx_status mont_ctx_query(const mont_ctx *ctx, uint32_t *bits, uint32_t *r_bits, uint32_t *limb_bits,
                         uint32_t *count, size_t *device_bytes);

/* Copies context `idx` to host memory as mont_words words each: N' mod R,
 * R^2 mod N and R mod N.  Synchronous; any output pointer may be NULL. */
mx_status mont_ctx_export(const mont_ctx *ctx, uint32_t idx, uint64_t *nprime_host, uint64_t *r2_host,
                          uint64_t *r1_host);

/* Frees the context.  The caller guarantees no queued work still uses it. */
void mont_ctx_destroy(mont_ctx *ctx);

/* out[i] = REDC(a[i] * b[i]) = (a b + q N) / R exactly, q = -a b N^{-1} mod R
 * (Algorithm 5's value; Algorithms 3 and 6 compute it, Theorem 1).  Values
 * are mont_words wide; precondition a, b < 2N, result < 2N.  MX_REDC_TRUNC
 * and MX_REDC_PLAIN return identical bits.  ctx_idx (device, n entries) picks
 * the context of each instance; NULL means instance i uses context i (then
 * n <= count).  out may alias a or b.  n = 0 is a no-op.  The block kernels
 * (MX_IMPL_BLOCK, MX_MUL_KARATSUBA, classes above 2048 bits) keep their
 * operands in the context's workspace: n is done in as many launches as it
 * holds (mont_ws_bytes gives one launch's size); MX_ENOMEM if it holds
 * fewer than 64 instances. */
mx_status mont_mul_batch(const mont_ctx *ctx, const uint32_t *ctx_idx, const uint64_t *a, const uint64_t *b,
                         uint64_t *out, uint32_t n, uint32_t flags, void *stream);

/* out[i] = REDC(a[i]^2), as mont_mul_batch with b = a (squaring, Algorithm 2). */
mx_status mont_sqr_batch(const mont_ctx *ctx, const uint32_t *ctx_idx, const uint64_t *a, uint64_t *out,
                         uint32_t n, uint32_t flags, void *stream);

/* out[i] = base[i]^exp[i] mod N, canonical in [0, N), by the constant-time
 * left-to-right fixed-window exponentiation of Algorithm 7 (table of 2^w
 * Montgomery powers, full masked table scan per window).  base: words wide,
 * base < N.  exp: ceil(exp_bits / 64) words per instance; exp_bits is public
 * and leading zeros are processed; bits above exp_bits are ignored.
 * exp_bits = 0 gives 1 (also 0^0 = 1).  window in 1..8, 0 = library choice.
 * The window table and working arrays live in the context's workspace
 * (modexp_ws_bytes): n is done in as many launches as it holds, MX_ENOMEM if
 * it holds fewer than 64 instances (mont_ctx_reserve grows it).  Calls on one
 * context take turns on that workspace (see Streams above); modexp_batch_ws
 * lets them overlap.  out may alias base. */
mx_status modexp_batch(const mont_ctx *ctx, const uint32_t *ctx_idx, const uint64_t *base, const uint64_t *exp,
                       uint32_t exp_bits, uint32_t window, uint64_t *out, uint32_t n, uint32_t flags,
                       void *stream);

/* As modexp_batch, with a caller-owned device workspace of ws_bytes bytes
 * instead of the context's: no allocation and no lock, so calls on one
 * context may overlap on different streams as long as each has its own
 * workspace.  A workspace smaller than modexp_ws_bytes(ctx, n, ...) is used
 * for n in several launches (MX_EINVAL if it cannot hold 64 instances). */
mx_status modexp_batch_ws(const mont_ctx *ctx, const uint32_t *ctx_idx, const uint64_t *base, const uint64_t *exp,
                          uint32_t exp_bits, uint32_t window, uint64_t *out, uint32_t n, uint32_t flags, void *ws,
                          size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): modexp_batch with
 * its workspace in a fixed array of 64 MiB that the library holds on each GPU
 * it runs on until the process ends; the call itself allocates nothing.  The
 * batch runs in one launch: MX_EINVAL, before anything is enqueued, if its
 * workspace (modexp_ws_bytes) exceeds 64 MiB -- at window 5, 8064 instances
 * of 2048 bits, 15872 of 1024 bits.  Every call on one GPU uses that GPU's
 * array, whatever the context or stream: calls that overlap on the device
 * race on it, so issue them on one stream (or order their streams).  The
 * array's address is looked up when the first context is made on a device. */
mx_status modexp_batch_noalloc(const mont_ctx *ctx, const uint32_t *ctx_idx, const uint64_t *base,
                               const uint64_t *exp, uint32_t exp_bits, uint32_t window, uint64_t *out, uint32_t n,
                               uint32_t flags, void *stream);

/* Workspace bytes a single launch of n instances needs for this window and
 * flags (larger batches than one 2 GiB launch holds: the bytes of one such
 * launch). */
mx_status modexp_ws_bytes(const mont_ctx *ctx, uint32_t n, uint32_t window, uint32_t flags, size_t *bytes);

/* The same for mont_mul_batch / mont_sqr_batch (0 for the register-resident
 * kernels, which need no workspace). */
mx_status mont_ws_bytes(const mont_ctx *ctx, uint32_t n, uint32_t flags, size_t *bytes);

/* ---- raw products --------------------------------------------------------------
 * out[i] = a[i] * b[i], or a[i]^2 when b is NULL: the full product of two
 * values of `bits` bits (1 <= bits <= 4256), without reduction -- the batch
 * multiplication the paper measures on its own (Section 2, Algorithms 1 and 2;
 * Section 3, Karatsuba; Table 6 goes to 4108 bits by schoolbook and 4154 by
 * Karatsuba).  flags: 0 schoolbook (block product scanning), MX_MUL_KARATSUBA
 * one level of Karatsuba above it, MX_MUL_KARATSUBA2 two levels; every method
 * gives the same integers.  a, b: ceil(bits / 64) words per instance, only
 * their low `bits` bits are used; out: ceil(2 bits / 64) words per instance.
 * Operands are held as 148 limbs of 28 bits up to 4144 bits, else 152 (four
 * blocks of 37 or 38 limbs; Karatsuba splits at block boundaries).  ws: a
 * caller-owned device workspace of ws_bytes; n is done in as many launches as
 * it holds (mp_mul_ws_bytes gives one launch's size; MX_EINVAL if it holds
 * fewer than 64 instances).  Allocates nothing.  out must not alias a or b. */
mx_status mp_mul_batch(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t bits, uint32_t n,
                       uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes of one mp_mul_batch launch over n instances. */
mx_status mp_mul_ws_bytes(uint32_t bits, uint32_t n, uint32_t flags, size_t *bytes);

/* ---- RSA private-key operations by the Chinese remainder theorem -----------
 * The application the paper's batched exponentiation is built for (Section
 * 1): out[i] = c[i]^d mod p q for a key given as dp = d mod (p-1),
 * dq = d mod (q-1) and qinv = q^{-1} mod p.  Computed as
 *   m1 = (c mod p)^dp mod p,  m2 = (c mod q)^dq mod q   (modexp_batch),
 *   h = qinv (m1 - m2) mod p,  out = m2 + h q            (Garner),
 * with c mod p = REDC(REDC(c) R^2 mod p) and h by one Montgomery product.
 * ctx_p, ctx_q: contexts of the primes, one size class (1024 bits for
 * RSA-2048, 2048 bits for RSA-4096, else MX_EUNSUPPORTED); key k is context k
 * of each.  Each prime has exactly `bits` bits (top bit set) and p != q;
 * otherwise the values are unspecified.  key_idx (device, n entries) picks
 * each instance's key; NULL means instance i uses key i.  c: 2 W words per
 * instance (W = bits/64), c < p q; dp, dq, qinv: W words each, dp < p, dq < q,
 * qinv < p; the exponents have exp_bits = bits.  out: 2 W words per
 * instance, canonical (< p q).  window and flags (MX_REDC_PLAIN or
 * MX_REDC_CIOS) apply to the two exponentiations.  out may alias c but not
 * dp, dq or qinv.  The two intermediates (n W words each) and the
 * exponentiations' table live in ctx_p's workspace (rsa_crt_ws_bytes gives
 * the size of one launch over both halves; a smaller workspace runs them one
 * after the other, in several launches if needed; MX_ENOMEM if it cannot
 * hold the intermediates and one 64-instance tile). */
mx_status rsa_crt_batch(const mont_ctx *ctx_p, const mont_ctx *ctx_q, const uint32_t *key_idx, const uint64_t *c,
                        const uint64_t *dp, const uint64_t *dq, const uint64_t *qinv, uint32_t window,
                        uint64_t *out, uint32_t n, uint32_t flags, void *stream);

/* As rsa_crt_batch with a caller-owned device workspace of ws_bytes bytes
 * (MX_EINVAL if it cannot hold the intermediates and one tile): no lock, so
 * calls with their own workspaces may overlap on different streams. */
mx_status rsa_crt_batch_ws(const mont_ctx *ctx_p, const mont_ctx *ctx_q, const uint32_t *key_idx,
                           const uint64_t *c, const uint64_t *dp, const uint64_t *dq, const uint64_t *qinv,
                           uint32_t window, uint64_t *out, uint32_t n, uint32_t flags, void *ws, size_t ws_bytes,
                           void *stream);

/* Workspace bytes of rsa_crt_batch over n instances as one paired launch
 * (where the class has it) for this window and flags. */
mx_status rsa_crt_ws_bytes(const mont_ctx *ctx_p, uint32_t n, uint32_t window, uint32_t flags, size_t *bytes);

/* ---- mixed sizes in one persistent launch ----------------------------------
 * For callers that hold batches of several size classes at once (not a
 * construct of the paper, which exponentiates one size per call; this plan
 * takes the place of a single mixed-launch call over job descriptors): the
 * instances of all batches are cut into 64-instance tiles, ordered by
 * decreasing cost and consumed by one persistent grid (one wavefront per
 * SIMD) through a device work counter.  The truncated reduction is used.
 * Supported classes: 1024, 2048 (optionally MX_IMPL_BLOCK or
 * MX_MUL_KARATSUBA), 3072, 4096 (optionally MX_MUL_KARATSUBA). */
typedef struct mx_batch_desc {
  const mont_ctx *ctx;      /* contexts of this batch's class                         */
  const uint32_t *ctx_idx;  /* device, n entries, or NULL: instance i uses context i  */
  const uint64_t *base;     /* device, n x ceil(bits/64) words, base < N              */
  const uint64_t *exp;      /* device, n x ceil(exp_bits/64) words                    */
  uint64_t *out;            /* device, n x ceil(bits/64) words                        */
  uint32_t n;
  uint32_t exp_bits;
  uint32_t window;          /* 1..8, 0 = library choice                               */
  uint32_t flags;           /* 0, MX_IMPL_BLOCK or MX_MUL_KARATSUBA                   */
  float tile_cost;          /* relative cost of one 64-instance tile, 0 = estimate    */
} mx_batch_desc;

typedef struct mx_mixed_plan mx_mixed_plan;

/* Validates the batches and allocates the job list, the work counter and one
 * workspace slot per persistent wave and batch (2^w r_bits/8 bytes per lane,
 * plus the working arrays of the block kernels).  The descriptors' device
 * pointers are captured: every launch of the plan reads and writes them.
 * MX_EUNSUPPORTED if a batch's workspace would exceed 2 GiB (smaller window). */
mx_status mx_mixed_plan_create(mx_mixed_plan **out, const mx_batch_desc *batches, uint32_t nbatch);

/* Enqueues a counter-reset kernel and the persistent kernel on `stream`.
 * Allocates nothing.  Launches of one plan must not overlap. */
mx_status mx_mixed_plan_launch(mx_mixed_plan *plan, void *stream);

/* As mx_mixed_plan_launch, through a HIP graph captured on the first call
 * and replayed afterwards. */
mx_status mx_mixed_plan_launch_graph(mx_mixed_plan *plan, void *stream);

/* Job (tile) count, persistent waves, and the window chosen for each batch. */
mx_status mx_mixed_plan_query(const mx_mixed_plan *plan, uint32_t *njobs, uint32_t *nslots, uint32_t *windows);

/* Frees the plan (after its launches have completed). */
void mx_mixed_plan_destroy(mx_mixed_plan *plan);

/* ---- autotuning --------------------------------------------------------------
 * Times modexp_batch on n seeded sample instances of ctx (bases below
 * 2^(bits-1), uniform exp_bits-bit exponents) for each candidate window, and
 * for the block and Karatsuba kernels too when try_block and the class has
 * them; returns
 * the fastest window and flags, and its time per 64-instance tile (the best
 * of `reps` runs, in ms).  Allocates its sample buffers. */
mx_status mx_tune_modexp(const mont_ctx *ctx, uint32_t n, uint32_t exp_bits, const uint32_t *windows,
                         uint32_t nwin, uint32_t try_block, uint32_t reps, uint32_t *best_window,
                         uint32_t *best_flags, float *best_ms, void *stream);

/* Thread-local message for the last non-OK status of this thread. */
const char *mont_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MONTEXP_H */
