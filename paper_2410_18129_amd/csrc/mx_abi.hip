// C ABI of libmontexp.so (declared in include/montexp.h): argument checks,
// context ownership, workspace management and kernel launches.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <memory>
#include <mutex>

#include "../../include/montexp.h"
#include "mx_internal.h"
#include "mx_ctx.h"

// ---- scratch of the allocation-free exponentiation (modexp_batch_noalloc) ----------------------
// The entry point keeps its window table and working arrays in this file-scope device array instead
// of a workspace that it allocates.  Each GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code the array's name is only a host-side stand-in for
// the symbol, never a device address: the address of a device's copy comes from
// hipGetSymbolAddress, looked up once per device, with that device current, by the first
// mont_ctx_init on it, and only that address is passed to kernels.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace mx {
// CRT-RSA steps around the two half-size exponentiations (mx_crt.hip, one object per prime class)
#define MX_DECL_CRT(B)                                                                                                \
  hipError_t crt_reduce_##B(const CtxDev& ctxp, const CtxDev& ctxq, const uint32_t* kidx, const uint64_t* c,         \
                            uint64_t* cp, uint64_t* cq, uint32_t count, uint32_t coff, hipStream_t st);             \
  hipError_t crt_garner_##B(const CtxDev& ctxp, const CtxDev& ctxq, const uint32_t* kidx, const uint64_t* m1,       \
                            const uint64_t* m2, const uint64_t* qinv, uint64_t* out, uint32_t count, uint32_t coff, \
                            hipStream_t st);
MX_DECL_CRT(1024)
MX_DECL_CRT(2048)
#undef MX_DECL_CRT
// batched raw products (mx_mul.hip)
uint32_t mul_raw_rows(uint32_t bits, int levels);
hipError_t mul_raw(int levels, const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t bits, uint32_t win,
                   uint32_t wout, uint32_t count, uint32_t* ws, uint32_t ws_bytes, hipStream_t st);
}  // namespace mx

namespace {

thread_local char g_err[512] = "";

mx_status fail(mx_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

mx_status dev_fail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? MX_ENOMEM : MX_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Per-device addresses of `scratch` (see its definition above).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Looks up the current device's copy of `scratch` (the current device is `dev`), once per device.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  if (e == hipSuccess && p) g_scratch_ptr[dev] = p;
}

// The device address of `dev`'s copy of `scratch` (nullptr before its lookup or if it failed).
void* scratch_of(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

// A launcher's error: hipErrorInvalidValue is its own refusal of a launch whose tiles the
// workspace does not hold (nothing was enqueued); anything else comes from the runtime.
mx_status launch_fail(hipError_t e, const char* where) {
  if (e == hipErrorInvalidValue)
    return fail(MX_EINVAL, "%s: launch refused: the workspace is smaller than the launch's tiles", where);
  return dev_fail(e, where);
}

uint32_t words_for(uint32_t bits) { return (bits + 63) / 64; }
uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

uint32_t default_window(uint32_t bits) {
  if (bits <= 128) return 3;
  if (bits <= 512) return 4;
  if (bits <= 2048) return 3;  // measured best at 2048 bits: the table stays in the last-level cache
  if (bits <= 3072) return 5;
  return 6;
}

// Switches to `dev` for the lifetime of the guard when it is not current.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

mx_status mx_fail(mx_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}



// Instances per launch for a workspace of `avail` bytes with `rows` 32-bit words per instance:
// whole 64-instance tiles, at most n, and under the 2 GiB one buffer descriptor spans.  0 when one
// tile does not fit.
static uint32_t fit_instances(uint32_t rows, uint32_t n, size_t avail) {
  if (rows == 0) return n;
  const size_t cap = avail < mx::kMaxWsBytes ? avail : mx::kMaxWsBytes;
  uint64_t c = (cap / ((uint64_t)rows * sizeof(uint32_t))) / 64 * 64;
  if (c > n) c = n;
  return (uint32_t)c;
}

// Bytes of workspace one launch over `cnt` instances uses (whole tiles).
static size_t launch_bytes(uint32_t rows, uint32_t cnt) { return (size_t)rows * round_up(cnt, 64) * sizeof(uint32_t); }

// Takes a context's library workspace for a batch call: holds its lock and, on construction,
// makes `stream` wait for the work last enqueued on it (possibly from another stream); on
// release, records that this call's work is now the last.
struct WsTurn {
  mont_ctx* ctx;
  hipStream_t st;
  std::unique_lock<std::mutex> lk;
  hipError_t err = hipSuccess;
  WsTurn(mont_ctx* c, hipStream_t s) : ctx(c), st(s), lk(c->ws_mu) {
    err = hipStreamWaitEvent(st, ctx->ws_done, 0);
  }
  hipError_t done() { return hipEventRecord(ctx->ws_done, st); }
};

// More than one of MX_ONE_LANE, MX_TWO_LANES and MX_FOUR_LANES.
static bool lane_flags_conflict(uint32_t flags) {
  const uint32_t l = flags & (uint32_t)(MX_ONE_LANE | MX_TWO_LANES | MX_FOUR_LANES);
  return (l & (l - 1)) != 0;
}

// Kernel family for the flags: 0 register-resident, 1 block, 2 block + Karatsuba, 3 block with one
// lane per instance whatever the batch size (MX_ONE_LANE), 4 block with at most two lanes per
// instance (MX_TWO_LANES), 5 block with four lanes per instance at any batch size (MX_FOUR_LANES);
// -1 if not built.
static int impl_of(const mont_ctx* ctx, uint32_t flags) {
  if (flags & MX_MUL_KARATSUBA) return ctx->ops->has_kara ? 2 : -1;
  const int blk = (flags & MX_ONE_LANE) ? 3 : (flags & MX_TWO_LANES) ? 4 : (flags & MX_FOUR_LANES) ? 5 : 1;
  if (flags & MX_IMPL_BLOCK) return ctx->ops->has_block ? blk : -1;
  return ctx->bits > 2048 && blk != 1 ? blk : 0;
}

// Reduction of the flags (mx::Redc); -1 if more than one of MX_REDC_PLAIN, MX_REDC_CIOS and
// MX_REDC_KARATSUBA is set.
static int redc_of(uint32_t flags) {
  const uint32_t r = flags & (uint32_t)(MX_REDC_PLAIN | MX_REDC_CIOS | MX_REDC_KARATSUBA);
  if (r & (r - 1)) return -1;
  return (flags & MX_REDC_CIOS) ? mx::kRedcCios : (flags & MX_REDC_KARATSUBA) ? mx::kRedcKara
       : (flags & MX_REDC_PLAIN) ? mx::kRedcPlain : mx::kRedcTrunc;
}

// Checks the reduction flags against the kernel family; MX_OK or the failure status.
static mx_status check_redc(const char* name, const mont_ctx* ctx, int impl, int redc) {
  if (redc < 0)
    return fail(MX_EINVAL, "%s: MX_REDC_PLAIN, MX_REDC_CIOS and MX_REDC_KARATSUBA exclude each other", name);
  const bool regcls = ctx->bits <= 2048;  // the classes with register-resident kernels
  if (redc == mx::kRedcCios) {
    // register-resident kernels; above 2048 bits the block-word CIOS, one lane per instance
    const bool reg = regcls && impl == 0;
    const bool blk = !regcls && (impl == 0 || impl == 1 || impl == 3);
    if (!ctx->ops->has_cios || (!reg && !blk))
      return fail(MX_EUNSUPPORTED, "%s: MX_REDC_CIOS is built for the register-resident kernels (<= 2048 bits) and "
                  "the block classes with one lane per instance", name);
  }
  if (redc == mx::kRedcKara) {
    const bool reg = regcls && impl == 0;
    // block kernels (the only ones above 2048 bits), one lane per instance, an even block count
    const bool blk = (impl >= 1 || !regcls) && impl != 4 && impl != 5 && ctx->ops->has_kara;
    if (!reg && !blk)
      return fail(MX_EUNSUPPORTED, "%s: MX_REDC_KARATSUBA is built for the register-resident kernels and the block "
                  "kernels with an even block count (2048, 4096 bits), one lane per instance", name);
  }
  return MX_OK;
}

// ---- device-data preconditions, checked on request (MX_CHECK_INPUTS) ------------------------
// flag[0] counts the instances whose value v is not below mult * N of their context, flag[1] is the
// first of them.  A debugging aid: unlike the method's kernels, this check branches on the data.
__global__ void k_check_clear(uint32_t* flag) {
  if (threadIdx.x == 0) flag[0] = 0u;
  if (threadIdx.x == 1) flag[1] = 0xFFFFFFFFu;
}

__global__ void k_check_below(mx::CtxDev ctx, const uint32_t* __restrict__ cidx, const uint64_t* __restrict__ v,
                              uint32_t words, uint32_t limbs, uint32_t mult, uint32_t count, uint32_t coff,
                              uint32_t* flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c = cidx ? cidx[i] : i + coff;
  c = c < ctx.count ? c : 0u;
  const uint64_t* x = v + (size_t)i * words;
  // v - mult N over the limbs of N, low to high; a negative final carry means v < mult N
  int64_t carry = 0;
  for (uint32_t k = 0; k < limbs; ++k) {
    const uint32_t bit = 28u * k, wd = bit >> 6, off = bit & 63u;
    uint64_t t = wd < words ? x[wd] >> off : 0ull;
    if (off > 36u && wd + 1 < words) t |= x[wd + 1] << (64u - off);
    const int64_t d = (int64_t)(t & 0xFFFFFFFull) - (int64_t)mult * (int64_t)ctx.n[(size_t)k * ctx.stride + c] + carry;
    carry = d >> 28;  // arithmetic shift: floor division
  }
  bool high = false;  // bits of v above the limbs
  const uint32_t top = 28u * limbs;
  for (uint32_t wd = top >> 6; wd < words; ++wd) high |= (wd == (top >> 6) ? x[wd] >> (top & 63u) : x[wd]) != 0ull;
  if (carry >= 0 || high) {
    atomicAdd(&flag[0], 1u);
    atomicMin(&flag[1], i);
  }
}

// Checks that the n values at v (words each) are below mult * N of their contexts, with 8 bytes of
// device memory at `flag`; waits for the stream.  MX_EINVAL names the violations.
static mx_status check_inputs(const char* name, const mont_ctx* ctx, const uint32_t* cidx, const uint64_t* v,
                              uint32_t words, uint32_t mult, uint32_t n, void* flag, hipStream_t st, const char* what) {
  uint32_t* f = (uint32_t*)flag;
  hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, st, f);
  hipLaunchKernelGGL(k_check_below, dim3((n + 255) / 256), dim3(256), 0, st, ctx->dev, cidx, v, words, ctx->limbs, mult,
                     n, 0u, f);
  hipError_t e = hipGetLastError();
  uint32_t h[2] = {0u, 0u};
  if (e == hipSuccess) e = hipMemcpyAsync(h, f, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return dev_fail(e, name);
  if (h[0]) return fail(MX_EINVAL, "%s: %u of %u instances violate %s (first: instance %u)", name, h[0], n, what, h[1]);
  return MX_OK;
}

// Library workspace a context reserves at init: one launch over its moduli at the default window,
// up to this size.
constexpr size_t kInitWsBytes = 256ull << 20;

extern "C" {

const char* mont_last_error(void) { return g_err; }

mx_status mont_ctx_init(mont_ctx** out, const uint64_t* moduli_host, uint32_t bits, uint32_t count, void* stream) {
  if (!out) return fail(MX_EINVAL, "mont_ctx_init: out is NULL");
  *out = nullptr;
  const mx::ClassOps* ops = mx::class_ops(bits);
  if (!ops) return fail(MX_EINVAL, "mont_ctx_init: unsupported size class %u", bits);
  const int limbs = ops->limbs;
  if (!moduli_host) return fail(MX_EINVAL, "mont_ctx_init: moduli_host is NULL");
  if (count == 0) return fail(MX_EINVAL, "mont_ctx_init: count is 0");
  const uint32_t W = words_for(bits);
  const uint32_t topbits = bits - 64 * (W - 1);
  for (uint32_t k = 0; k < count; ++k) {
    const uint64_t* m = moduli_host + (size_t)k * W;
    if ((m[0] & 1u) == 0) return fail(MX_EINVAL, "mont_ctx_init: modulus %u is even", k);
    bool big = false;
    for (uint32_t j = 1; j < W; ++j) big |= m[j] != 0;
    if (!big && m[0] < 3) return fail(MX_EINVAL, "mont_ctx_init: modulus %u is below 3", k);
    if (topbits < 64 && (m[W - 1] >> topbits) != 0)
      return fail(MX_EINVAL, "mont_ctx_init: modulus %u exceeds %u bits", k, bits);
  }
  mont_ctx* c = new (std::nothrow) mont_ctx;
  if (!c) return fail(MX_ENOMEM, "mont_ctx_init: host allocation failed");
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(MX_EDEVICE, "mont_ctx_init: no HIP device");
  }
  scratch_setup(c->device);  // this device's copy of the allocation-free entry point's scratch
  c->ops = ops;
  c->bits = bits;
  c->limbs = (uint32_t)limbs;
  c->count = count;
  const uint32_t stride = round_up(count, 64);
  const size_t arr = (size_t)limbs * stride * sizeof(uint32_t);
  c->bytes = 4 * arr;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMalloc(&c->mem, c->bytes);
  if (e != hipSuccess) {
    delete c;
    return dev_fail(e, "mont_ctx_init: context allocation");
  }
  uint8_t* base = (uint8_t*)c->mem;
  c->dev.n = (uint32_t*)(base);
  c->dev.np = (uint32_t*)(base + arr);
  c->dev.r2 = (uint32_t*)(base + 2 * arr);
  c->dev.r1 = (uint32_t*)(base + 3 * arr);
  c->dev.count = count;
  c->dev.stride = stride;
  uint64_t* dmods = nullptr;
  const size_t mbytes = (size_t)count * W * sizeof(uint64_t);
  e = hipMalloc(&dmods, mbytes);
  if (e == hipSuccess) e = hipMemcpyAsync(dmods, moduli_host, mbytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->mem, 0, c->bytes, st);
  if (e == hipSuccess) e = ops->ctx_init(dmods, c->dev, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (dmods) (void)hipFree(dmods);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ws_done, hipEventDisableTiming);
  if (e == hipSuccess) {
    // the library workspace: one launch of `count` instances at the class's default window, at most
    // kInitWsBytes (larger calls run in several launches, or call mont_ctx_reserve first)
    const uint32_t rows = ops->ws_rows(0, true, default_window(bits));
    const uint32_t fit = fit_instances(rows, count, kInitWsBytes);
    const size_t want = launch_bytes(rows, fit ? fit : 64);
    e = hipMalloc(&c->ws, want);
    if (e == hipSuccess) c->ws_bytes = want;
  }
  if (e != hipSuccess) {
    if (c->ws_done) (void)hipEventDestroy(c->ws_done);
    if (c->ws) (void)hipFree(c->ws);
    (void)hipFree(c->mem);
    delete c;
    return dev_fail(e, "mont_ctx_init");
  }
  *out = c;
  return MX_OK;
}

mx_status mont_ctx_reserve(mont_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(MX_EINVAL, "mont_ctx_reserve: ctx is NULL");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "mont_ctx_reserve: cannot select device");
  std::lock_guard<std::mutex> lk(ctx->ws_mu);
  if (ctx->ws_bytes >= bytes) return MX_OK;
  // queued work may still use the old buffer: wait for it (this context's work only)
  hipError_t e = hipEventSynchronize(ctx->ws_done);
  if (e != hipSuccess) return dev_fail(e, "mont_ctx_reserve");
  void* nw = nullptr;
  e = hipMalloc(&nw, bytes);
  if (e != hipSuccess) return dev_fail(e, "mont_ctx_reserve");
  if (ctx->ws) (void)hipFree(ctx->ws);
  ctx->ws = nw;
  ctx->ws_bytes = bytes;
  return MX_OK;
}

mx_status mont_ctx_query(const mont_ctx* ctx, uint32_t* bits, uint32_t* r_bits, uint32_t* limb_bits,
                         uint32_t* count, size_t* device_bytes) {
  if (!ctx) return fail(MX_EINVAL, "mont_ctx_query: ctx is NULL");
  if (bits) *bits = ctx->bits;
  if (r_bits) *r_bits = 28 * ctx->limbs;
  if (limb_bits) *limb_bits = 28;
  if (count) *count = ctx->count;
  if (device_bytes) *device_bytes = ctx->bytes + ctx->ws_bytes;
  return MX_OK;
}

mx_status mont_ctx_export(const mont_ctx* ctx, uint32_t idx, uint64_t* nprime_host, uint64_t* r2_host,
                          uint64_t* r1_host) {
  if (!ctx) return fail(MX_EINVAL, "mont_ctx_export: ctx is NULL");
  if (idx >= ctx->count) return fail(MX_EINVAL, "mont_ctx_export: index %u >= count %u", idx, ctx->count);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "mont_ctx_export: cannot select device");
  const uint32_t n = ctx->limbs;
  const uint32_t mw = words_for(28 * n);
  const uint32_t* srcs[3] = {ctx->dev.np, ctx->dev.r2, ctx->dev.r1};
  uint64_t* dsts[3] = {nprime_host, r2_host, r1_host};
  uint32_t limbs[512];
  for (int a = 0; a < 3; ++a) {
    if (!dsts[a]) continue;
    hipError_t e = hipMemcpy2D(limbs, sizeof(uint32_t), srcs[a] + idx, (size_t)ctx->dev.stride * sizeof(uint32_t),
                               sizeof(uint32_t), n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(e, "mont_ctx_export");
    memset(dsts[a], 0, mw * sizeof(uint64_t));
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t bit = 28 * i, wd = bit / 64, off = bit % 64;
      dsts[a][wd] |= (uint64_t)limbs[i] << off;
      if (off > 36 && wd + 1 < mw) dsts[a][wd + 1] |= (uint64_t)limbs[i] >> (64 - off);
    }
  }
  return MX_OK;
}

void mont_ctx_destroy(mont_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  if (ctx->ws_done) (void)hipEventDestroy(ctx->ws_done);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->mem) (void)hipFree(ctx->mem);
  delete ctx;
}

static mx_status mont_common(const char* name, const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* a,
                             const uint64_t* b, uint64_t* out, uint32_t n, uint32_t flags, void* stream, bool sqr) {
  if (!ctx) return fail(MX_EINVAL, "%s: ctx is NULL", name);
  if (n == 0) return MX_OK;
  if (!a || !out || (!sqr && !b)) return fail(MX_EINVAL, "%s: NULL operand pointer", name);
  if (flags & ~(uint32_t)(MX_REDC_PLAIN | MX_IMPL_BLOCK | MX_MUL_KARATSUBA | MX_REDC_CIOS | MX_REDC_KARATSUBA |
                          MX_CHECK_INPUTS))
    return fail(MX_EINVAL, "%s: unknown flags 0x%x", name, flags);
  const int impl = impl_of(ctx, flags);
  if (impl < 0) return fail(MX_EUNSUPPORTED, "%s: kernel family not built for the %u-bit class", name, ctx->bits);
  const int redc = redc_of(flags);
  if (mx_status rs = check_redc(name, ctx, impl, redc); rs != MX_OK) return rs;
  if (!ctx_idx && n > ctx->count) return fail(MX_EINVAL, "%s: n=%u exceeds context count %u", name, n, ctx->count);
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "%s: cannot select device", name);
  mont_ctx* mctx = const_cast<mont_ctx*>(ctx);
  const uint32_t mw = words_for(28 * ctx->limbs);
  const uint32_t rows = ctx->ops->ws_rows(impl, false, 0);
  hipStream_t st = (hipStream_t)stream;
  if (flags & MX_CHECK_INPUTS) {  // a, b < 2N, with 8 bytes of the context's workspace; waits for the stream
    WsTurn ct(mctx, st);
    if (ct.err != hipSuccess) return dev_fail(ct.err, name);
    mx_status cs = check_inputs(name, ctx, ctx_idx, a, mw, 2, n, mctx->ws, st, "a < 2N");
    if (cs == MX_OK && !sqr) cs = check_inputs(name, ctx, ctx_idx, b, mw, 2, n, mctx->ws, st, "b < 2N");
    (void)ct.done();
    if (cs != MX_OK) return cs;
  }
  if (rows == 0) {  // register-resident kernels: no workspace
    hipError_t e = ctx->ops->mont(impl, redc, sqr, ctx->dev, ctx_idx, a, b, out, n, nullptr, 0, 0,
                                  0u, st);
    return e == hipSuccess ? MX_OK : launch_fail(e, name);
  }
  WsTurn turn(mctx, st);
  if (turn.err != hipSuccess) return dev_fail(turn.err, name);
  const uint32_t chunk = fit_instances(rows, n, mctx->ws_bytes);
  if (chunk == 0)
    return fail(MX_ENOMEM, "%s: the context workspace (%zu bytes) holds no tile; reserve %zu bytes with "
                "mont_ctx_reserve", name, mctx->ws_bytes, launch_bytes(rows, 64));
  hipError_t e = hipSuccess;
  for (uint32_t off = 0; off < n && e == hipSuccess; off += chunk) {
    const uint32_t cnt = n - off < chunk ? n - off : chunk;
    e = ctx->ops->mont(impl, redc, sqr, ctx->dev, ctx_idx ? ctx_idx + off : nullptr, a + (size_t)off * mw,
                       b + (size_t)off * mw, out + (size_t)off * mw, cnt, (uint32_t*)mctx->ws,
                       round_up(cnt, 64), (uint32_t)launch_bytes(rows, cnt), ctx_idx ? 0u : off, st);
  }
  const hipError_t re = turn.done();
  if (e != hipSuccess) return launch_fail(e, name);
  return re == hipSuccess ? MX_OK : dev_fail(re, name);
}

mx_status mont_mul_batch(const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* a, const uint64_t* b,
                         uint64_t* out, uint32_t n, uint32_t flags, void* stream) {
  return mont_common("mont_mul_batch", ctx, ctx_idx, a, b, out, n, flags, stream, false);
}

mx_status mont_sqr_batch(const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* a, uint64_t* out, uint32_t n,
                         uint32_t flags, void* stream) {
  return mont_common("mont_sqr_batch", ctx, ctx_idx, a, a, out, n, flags, stream, true);
}

// Checks of an exponentiation call shared by the entry points; on MX_OK, *impl, *redc and *w hold
// the kernel family, the reduction and the window.
static mx_status modexp_args(const char* name, const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* base,
                             const uint64_t* exp, uint32_t exp_bits, uint32_t window, uint64_t* out, uint32_t n,
                             uint32_t flags, int* impl, int* redc, uint32_t* w) {
  if (!ctx) return fail(MX_EINVAL, "%s: ctx is NULL", name);
  if (n && (!base || !out || (exp_bits && !exp))) return fail(MX_EINVAL, "%s: NULL operand pointer", name);
  if (flags & ~(uint32_t)(MX_REDC_PLAIN | MX_IMPL_BLOCK | MX_MUL_KARATSUBA | MX_ONE_LANE | MX_REDC_CIOS |
                          MX_TWO_LANES | MX_REDC_KARATSUBA | MX_CHECK_INPUTS | MX_FOUR_LANES))
    return fail(MX_EINVAL, "%s: unknown flags 0x%x", name, flags);
  if (lane_flags_conflict(flags))
    return fail(MX_EINVAL, "%s: MX_ONE_LANE, MX_TWO_LANES and MX_FOUR_LANES exclude each other", name);
  *impl = impl_of(ctx, flags);
  if (*impl < 0) return fail(MX_EUNSUPPORTED, "%s: kernel family not built for the %u-bit class", name, ctx->bits);
  *redc = redc_of(flags);
  if (mx_status rs = check_redc(name, ctx, *impl, *redc); rs != MX_OK) return rs;
  if (window > 8) return fail(MX_EINVAL, "%s: window %u outside 1..8", name, window);
  if (!ctx_idx && n > ctx->count) return fail(MX_EINVAL, "%s: n=%u exceeds context count %u", name, n, ctx->count);
  *w = window ? window : default_window(ctx->bits);
  return MX_OK;
}

// Enqueues the exponentiation of n instances in as many launches as a workspace of ws_bytes
// needs (each launch under 2 GiB).  The caller owns the workspace for the stream's work.
static mx_status modexp_launches(const char* name, const mont_ctx* ctx, int impl, int redc, const uint32_t* ctx_idx,
                                 const uint64_t* base, const uint64_t* exp, uint32_t exp_bits, uint32_t w,
                                 uint64_t* out, uint32_t n, void* ws, size_t ws_bytes, bool caller_ws,
                                 hipStream_t st) {
  const uint32_t ewords = (exp_bits + 63) / 64;
  const uint32_t W = words_for(ctx->bits);
  const uint32_t rows = ctx->ops->ws_rows(impl, true, w);
  const uint32_t chunk = fit_instances(rows, n, ws_bytes);
  if (chunk == 0)
    return fail(caller_ws ? MX_EINVAL : MX_ENOMEM, "%s: a workspace of %zu bytes holds no 64-instance tile (%zu "
                "bytes at window %u)%s", name, ws_bytes, launch_bytes(rows, 64), w,
                caller_ws ? "" : ": reserve modexp_ws_bytes() with mont_ctx_reserve");
  for (uint32_t off = 0; off < n; off += chunk) {
    const uint32_t cnt = n - off < chunk ? n - off : chunk;
    hipError_t e = ctx->ops->modexp(impl, redc, ctx->dev, ctx_idx ? ctx_idx + off : nullptr, base + (size_t)off * W,
                                    exp_bits ? exp + (size_t)off * ewords : exp, exp_bits, ewords, w,
                                    out + (size_t)off * W, cnt, (uint32_t*)ws, round_up(cnt, 64),
                                    (uint32_t)launch_bytes(rows, cnt), ctx_idx ? 0u : off, st);
    if (e != hipSuccess) return launch_fail(e, name);
  }
  return MX_OK;
}

mx_status modexp_batch(const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* base, const uint64_t* exp,
                       uint32_t exp_bits, uint32_t window, uint64_t* out, uint32_t n, uint32_t flags, void* stream) {
  const char* name = "modexp_batch";
  int impl = 0, redc = 0;
  uint32_t w = 0;
  mx_status rs = modexp_args(name, ctx, ctx_idx, base, exp, exp_bits, window, out, n, flags, &impl, &redc, &w);
  if (rs != MX_OK || n == 0) return rs;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "%s: cannot select device", name);
  mont_ctx* c = const_cast<mont_ctx*>(ctx);
  WsTurn turn(c, (hipStream_t)stream);
  if (turn.err != hipSuccess) return dev_fail(turn.err, name);
  if (flags & MX_CHECK_INPUTS) {  // base < N, with 8 bytes of the workspace; waits for the stream
    rs = check_inputs(name, ctx, ctx_idx, base, words_for(ctx->bits), 1, n, c->ws, (hipStream_t)stream, "base < N");
    if (rs != MX_OK) {
      (void)turn.done();
      return rs;
    }
  }
  rs = modexp_launches(name, ctx, impl, redc, ctx_idx, base, exp, exp_bits, w, out, n, c->ws, c->ws_bytes, false,
                       (hipStream_t)stream);
  const hipError_t e = turn.done();
  if (rs == MX_OK && e != hipSuccess) return dev_fail(e, name);
  return rs;
}

mx_status modexp_batch_ws(const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* base, const uint64_t* exp,
                          uint32_t exp_bits, uint32_t window, uint64_t* out, uint32_t n, uint32_t flags, void* ws,
                          size_t ws_bytes, void* stream) {
  const char* name = "modexp_batch_ws";
  if (!ws) return fail(MX_EINVAL, "%s: workspace is NULL", name);
  int impl = 0, redc = 0;
  uint32_t w = 0;
  mx_status rs = modexp_args(name, ctx, ctx_idx, base, exp, exp_bits, window, out, n, flags, &impl, &redc, &w);
  if (rs != MX_OK || n == 0) return rs;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "%s: cannot select device", name);
  if (flags & MX_CHECK_INPUTS) {  // base < N, with 8 bytes of the caller's workspace; waits for the stream
    if (ws_bytes < 8) return fail(MX_EINVAL, "%s: workspace of %zu bytes", name, ws_bytes);
    rs = check_inputs(name, ctx, ctx_idx, base, words_for(ctx->bits), 1, n, ws, (hipStream_t)stream, "base < N");
    if (rs != MX_OK) return rs;
  }
  return modexp_launches(name, ctx, impl, redc, ctx_idx, base, exp, exp_bits, w, out, n, ws, ws_bytes, true,
                         (hipStream_t)stream);
}

mx_status modexp_batch_noalloc(const mont_ctx* ctx, const uint32_t* ctx_idx, const uint64_t* base,
                               const uint64_t* exp, uint32_t exp_bits, uint32_t window, uint64_t* out, uint32_t n,
                               uint32_t flags, void* stream) {
  const char* name = "modexp_batch_noalloc";
  int impl = 0, redc = 0;
  uint32_t w = 0;
  mx_status rs = modexp_args(name, ctx, ctx_idx, base, exp, exp_bits, window, out, n, flags, &impl, &redc, &w);
  if (rs != MX_OK || n == 0) return rs;
  const uint32_t rows = ctx->ops->ws_rows(impl, true, w);
  const size_t need = launch_bytes(rows, n);
  if (need > kScratchBytes)
    return fail(MX_EINVAL, "%s: %u instances at window %u need %zu bytes of scratch; the maximum is %zu bytes "
                "(%u instances): split the batch", name, n, w, need, kScratchBytes,
                fit_instances(rows, 0xFFFFFFFFu, kScratchBytes));
  hipError_t serr = hipSuccess;
  void* ptr = scratch_of(ctx->device, &serr);
  if (!ptr)
    return fail(MX_EDEVICE, "%s: no scratch address for device %d: %s", name, ctx->device, hipGetErrorString(serr));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(MX_EDEVICE, "%s: cannot select device", name);
  if (flags & MX_CHECK_INPUTS) {  // base < N, with 8 bytes of the scratch; waits for the stream
    rs = check_inputs(name, ctx, ctx_idx, base, words_for(ctx->bits), 1, n, ptr, (hipStream_t)stream, "base < N");
    if (rs != MX_OK) return rs;
  }
  // one launch (need <= kScratchBytes < 2 GiB); every row a kernel reads it has written first in the
  // same launch, so nothing in the scratch has to start at zero
  return modexp_launches(name, ctx, impl, redc, ctx_idx, base, exp, exp_bits, w, out, n, ptr, kScratchBytes, true,
                         (hipStream_t)stream);
}

}  // extern "C"

// Bytes of the two intermediates of a CRT batch (c mod p then m1, c mod q then m2), whole 256-byte units.
static size_t crt_inter_bytes(uint32_t bits, uint32_t n) {
  return ((size_t)n * 2 * words_for(bits) * sizeof(uint64_t) + 255) / 256 * 256;
}

// Workspace of the two exponentiations as one paired launch (0 where the class has no paired kernel).
static size_t crt_pair_bytes(const mont_ctx* cp, uint32_t n, uint32_t w, int redc) {
  if (!cp->ops->modexp_pair || redc == mx::kRedcCios) return 0;
  const size_t b = (size_t)cp->ops->ws_rows(0, true, w) * 64u * sizeof(uint32_t) * 2u * ((n + 63) / 64);
  return b <= mx::kMaxWsBytes ? b : 0;
}

static mx_status rsa_crt_common(const char* name, const mont_ctx* ctx_p, const mont_ctx* ctx_q, const uint32_t* key_idx,
                                const uint64_t* c, const uint64_t* dp, const uint64_t* dq, const uint64_t* qinv,
                                uint32_t window, uint64_t* out, uint32_t n, uint32_t flags, void* user_ws,
                                size_t user_ws_bytes, void* stream) {
  if (!ctx_p || !ctx_q) return fail(MX_EINVAL, "%s: ctx is NULL", name);
  if (ctx_p->bits != ctx_q->bits) return fail(MX_EINVAL, "%s: p and q contexts of different classes", name);
  if (ctx_p->device != ctx_q->device) return fail(MX_EINVAL, "%s: contexts on different devices", name);
  const uint32_t bits = ctx_p->bits;
  if (bits != 1024 && bits != 2048)
    return fail(MX_EUNSUPPORTED, "%s: %u-bit primes (1024 and 2048 are built)", name, bits);
  if (n == 0) return MX_OK;
  if (!c || !dp || !dq || !qinv || !out) return fail(MX_EINVAL, "%s: NULL operand pointer", name);
  if (flags & ~(uint32_t)(MX_REDC_PLAIN | MX_REDC_CIOS)) return fail(MX_EINVAL, "%s: unknown flags 0x%x", name, flags);
  // (MX_REDC_KARATSUBA is rejected here as an unknown flag: it has no exponentiation kernel)
  if (window > 8) return fail(MX_EINVAL, "%s: window %u outside 1..8", name, window);
  const uint32_t cnt_min = ctx_p->count < ctx_q->count ? ctx_p->count : ctx_q->count;
  if (!key_idx && n > cnt_min) return fail(MX_EINVAL, "%s: n=%u exceeds the key count %u", name, n, cnt_min);
  const int redc = redc_of(flags);
  if (redc < 0) return fail(MX_EINVAL, "%s: MX_REDC_PLAIN and MX_REDC_CIOS exclude each other", name);
  DeviceGuard g(ctx_p->device);
  if (!g.ok) return fail(MX_EDEVICE, "%s: cannot select device", name);
  mont_ctx* cp = const_cast<mont_ctx*>(ctx_p);
  mont_ctx* cq = const_cast<mont_ctx*>(ctx_q);
  hipStream_t st = (hipStream_t)stream;
  // workspace: the two intermediates, then the exponentiations' workspace
  std::unique_ptr<WsTurn> turn;
  uint8_t* ws = (uint8_t*)user_ws;
  size_t ws_bytes = user_ws_bytes;
  if (!ws) {
    turn.reset(new WsTurn(cp, st));
    if (turn->err != hipSuccess) return dev_fail(turn->err, name);
    ws = (uint8_t*)cp->ws;
    ws_bytes = cp->ws_bytes;
  }
  const uint32_t W = words_for(bits);
  const uint32_t w = window ? window : default_window(bits);
  const size_t inter = crt_inter_bytes(bits, n);
  const size_t one_tile = launch_bytes(cp->ops->ws_rows(0, true, w), 64);
  if (ws_bytes < inter + one_tile)
    return fail(user_ws ? MX_EINVAL : MX_ENOMEM, "%s: workspace of %zu bytes < %zu (intermediates and one tile)%s",
                name, ws_bytes, inter + one_tile, user_ws ? "" : ": reserve rsa_crt_ws_bytes() on ctx_p");
  uint64_t* xp = (uint64_t*)ws;           // c mod p, then m1
  uint64_t* xq = xp + (size_t)n * W;       // c mod q, then m2
  uint8_t* ews = ws + inter;
  const size_t ews_bytes = ws_bytes - inter;
  hipError_t e = bits == 1024 ? mx::crt_reduce_1024(cp->dev, cq->dev, key_idx, c, xp, xq, n, 0, st)
                              : mx::crt_reduce_2048(cp->dev, cq->dev, key_idx, c, xp, xq, n, 0, st);
  mx_status rs = e == hipSuccess ? MX_OK : dev_fail(e, name);
  // the two half-size exponentiations, in place (the outputs may alias the bases): one launch
  // over both halves where the class has it and the workspace holds it, else one after the other
  const size_t pair = crt_pair_bytes(cp, n, w, redc);
  if (rs == MX_OK && pair && pair <= ews_bytes) {
    e = cp->ops->modexp_pair(redc == mx::kRedcTrunc, cp->dev, cq->dev, key_idx, xp, dp, dq, bits, W, w, xp, n,
                             (uint32_t*)ews, (uint32_t)pair, st);
    if (e != hipSuccess) rs = launch_fail(e, name);
  } else if (rs == MX_OK) {
    const int impl = 0;
    rs = modexp_launches(name, cp, impl, redc, key_idx, xp, dp, bits, w, xp, n, ews, ews_bytes, true, st);
    if (rs == MX_OK)
      rs = modexp_launches(name, cq, impl, redc, key_idx, xq, dq, bits, w, xq, n, ews, ews_bytes, true, st);
  }
  if (rs == MX_OK) {
    e = bits == 1024 ? mx::crt_garner_1024(cp->dev, cq->dev, key_idx, xp, xq, qinv, out, n, 0, st)
                     : mx::crt_garner_2048(cp->dev, cq->dev, key_idx, xp, xq, qinv, out, n, 0, st);
    if (e != hipSuccess) rs = dev_fail(e, name);
  }
  if (turn) {
    e = turn->done();
    if (rs == MX_OK && e != hipSuccess) rs = dev_fail(e, name);
  }
  return rs;
}

extern "C" {

mx_status rsa_crt_batch(const mont_ctx* ctx_p, const mont_ctx* ctx_q, const uint32_t* key_idx, const uint64_t* c,
                        const uint64_t* dp, const uint64_t* dq, const uint64_t* qinv, uint32_t window, uint64_t* out,
                        uint32_t n, uint32_t flags, void* stream) {
  return rsa_crt_common("rsa_crt_batch", ctx_p, ctx_q, key_idx, c, dp, dq, qinv, window, out, n, flags, nullptr, 0,
                        stream);
}

mx_status rsa_crt_batch_ws(const mont_ctx* ctx_p, const mont_ctx* ctx_q, const uint32_t* key_idx, const uint64_t* c,
                           const uint64_t* dp, const uint64_t* dq, const uint64_t* qinv, uint32_t window,
                           uint64_t* out, uint32_t n, uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (!ws) return fail(MX_EINVAL, "rsa_crt_batch_ws: workspace is NULL");
  return rsa_crt_common("rsa_crt_batch_ws", ctx_p, ctx_q, key_idx, c, dp, dq, qinv, window, out, n, flags, ws,
                        ws_bytes, stream);
}

mx_status rsa_crt_ws_bytes(const mont_ctx* ctx_p, uint32_t n, uint32_t window, uint32_t flags, size_t* bytes) {
  if (!ctx_p || !bytes) return fail(MX_EINVAL, "rsa_crt_ws_bytes: NULL argument");
  if (ctx_p->bits != 1024 && ctx_p->bits != 2048)
    return fail(MX_EUNSUPPORTED, "rsa_crt_ws_bytes: %u-bit primes (1024 and 2048 are built)", ctx_p->bits);
  if (window > 8) return fail(MX_EINVAL, "rsa_crt_ws_bytes: window %u outside 1..8", window);
  const int redc = redc_of(flags);
  if (redc < 0 || (flags & ~(uint32_t)(MX_REDC_PLAIN | MX_REDC_CIOS)))
    return fail(MX_EINVAL, "rsa_crt_ws_bytes: bad flags 0x%x", flags);
  const uint32_t w = window ? window : default_window(ctx_p->bits);
  const size_t pair = crt_pair_bytes(ctx_p, n ? n : 1, w, redc);
  const uint32_t rows = ctx_p->ops->ws_rows(0, true, w);
  const size_t ex = pair ? pair : launch_bytes(rows, fit_instances(rows, n ? n : 1, mx::kMaxWsBytes));
  *bytes = crt_inter_bytes(ctx_p->bits, n) + ex;
  return MX_OK;
}

mx_status modexp_ws_bytes(const mont_ctx* ctx, uint32_t n, uint32_t window, uint32_t flags, size_t* bytes) {
  if (!ctx || !bytes) return fail(MX_EINVAL, "modexp_ws_bytes: NULL argument");
  const int impl = impl_of(ctx, flags);
  if (impl < 0) return fail(MX_EUNSUPPORTED, "modexp_ws_bytes: kernel family not built for this class");
  if (window > 8) return fail(MX_EINVAL, "modexp_ws_bytes: window %u outside 1..8", window);
  const uint32_t w = window ? window : default_window(ctx->bits);
  const uint32_t rows = ctx->ops->ws_rows(impl, true, w);
  const uint32_t chunk = fit_instances(rows, n ? n : 1, mx::kMaxWsBytes);
  *bytes = launch_bytes(rows, chunk ? chunk : 64);
  return MX_OK;
}

// Karatsuba levels of a raw product's flags (0, 1, 2), or -1 for flags that are not a method.
static int mul_levels(uint32_t flags) {
  if (flags == 0) return 0;
  if (flags == (uint32_t)MX_MUL_KARATSUBA) return 1;
  if (flags == (uint32_t)MX_MUL_KARATSUBA2) return 2;
  return -1;
}

mx_status mp_mul_ws_bytes(uint32_t bits, uint32_t n, uint32_t flags, size_t* bytes) {
  if (!bytes) return fail(MX_EINVAL, "mp_mul_ws_bytes: bytes is NULL");
  const int lv = mul_levels(flags);
  if (lv < 0) return fail(MX_EINVAL, "mp_mul_ws_bytes: flags 0x%x are not a product method", flags);
  const uint32_t rows = bits ? mx::mul_raw_rows(bits, lv) : 0u;
  if (rows == 0) return fail(MX_EUNSUPPORTED, "mp_mul_ws_bytes: %u-bit operands (1 .. 4256 are built)", bits);
  const uint32_t chunk = fit_instances(rows, n ? n : 1, mx::kMaxWsBytes);
  *bytes = launch_bytes(rows, chunk ? chunk : 64);
  return MX_OK;
}

mx_status mp_mul_batch(const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t bits, uint32_t n, uint32_t flags,
                       void* ws, size_t ws_bytes, void* stream) {
  const char* name = "mp_mul_batch";
  const int lv = mul_levels(flags);
  if (lv < 0) return fail(MX_EINVAL, "%s: flags 0x%x are not a product method", name, flags);
  const uint32_t rows = bits ? mx::mul_raw_rows(bits, lv) : 0u;
  if (rows == 0) return fail(MX_EUNSUPPORTED, "%s: %u-bit operands (1 .. 4256 are built)", name, bits);
  if (n == 0) return MX_OK;
  if (!a || !out || !ws) return fail(MX_EINVAL, "%s: NULL pointer", name);
  const uint32_t chunk = fit_instances(rows, n, ws_bytes);
  if (chunk == 0)
    return fail(MX_EINVAL, "%s: a workspace of %zu bytes holds no 64-instance tile (%zu bytes)", name, ws_bytes,
                launch_bytes(rows, 64));
  const uint32_t win = words_for(bits), wout = words_for(2 * bits);
  for (uint32_t off = 0; off < n; off += chunk) {
    const uint32_t cnt = n - off < chunk ? n - off : chunk;
    hipError_t e = mx::mul_raw(lv, a + (size_t)off * win, b ? b + (size_t)off * win : nullptr, out + (size_t)off * wout,
                               bits, win, wout, cnt, (uint32_t*)ws, (uint32_t)launch_bytes(rows, cnt),
                               (hipStream_t)stream);
    if (e != hipSuccess) return launch_fail(e, name);
  }
  return MX_OK;
}

mx_status mont_ws_bytes(const mont_ctx* ctx, uint32_t n, uint32_t flags, size_t* bytes) {
  if (!ctx || !bytes) return fail(MX_EINVAL, "mont_ws_bytes: NULL argument");
  const int impl = impl_of(ctx, flags);
  if (impl < 0) return fail(MX_EUNSUPPORTED, "mont_ws_bytes: kernel family not built for this class");
  const uint32_t rows = ctx->ops->ws_rows(impl, false, 0);
  const uint32_t chunk = fit_instances(rows, n ? n : 1, mx::kMaxWsBytes);
  *bytes = rows ? launch_bytes(rows, chunk ? chunk : 64) : 0;
  return MX_OK;
}

}  // extern "C"
