// Mixed-size exponentiation in one persistent launch, and the window /
// kernel-family autotuner.
//
// A plan holds several batches (one per size class, each with its own
// contexts).  Their instances are cut into tiles of 64 (one wavefront); the
// tiles become a job list ordered by decreasing cost (longest first).  One
// persistent grid of one wavefront per SIMD pulls jobs from a device counter
// until the list is exhausted, so the classes share the GPU without a launch
// per class and without idle tails between them.  Each persistent wave owns
// one workspace slot per batch (its window table and, for the block kernels,
// its working arrays), reused from tile to tile.
//
// A plan allocates everything at creation; launching it only enqueues a
// counter-reset kernel and the persistent kernel (no allocation, no memset),
// so a launch can be captured into a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/montexp.h"
#include "mx_block.hpp"
#include "mx_ctx.h"

namespace mx {

// kernel families reachable from the persistent kernel
enum Family : uint32_t {
  kF1024 = 0, kF1024B = 1, kF2048 = 2, kF2048B = 3, kF3072B = 4, kF4096B = 5, kF2048K = 6, kF4096K = 7, kNumFam = 8
};
constexpr int kMaxMixedBatches = 8;

struct MixedBatch {
  CtxDev ctx;
  const uint32_t* cidx;
  const uint64_t* base;
  const uint64_t* ex;
  uint64_t* out;
  uint32_t* ws;   // one region of rows x 64 words per persistent wave
  uint32_t count, ebits, ewords, w, family, rows;
  uint32_t lanes;  // lanes per instance: tiles of 64 / lanes instances
};

struct MixedArgs {
  MixedBatch b[kMaxMixedBatches];
  const uint32_t* jobs;  // batch index << 28 | tile index
  uint32_t* counter;
  uint32_t njobs;
};

__global__ void k_reset_counter(uint32_t* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

__global__ void __launch_bounds__(64) k_modexp_mixed(MixedArgs args) {
  __shared__ uint32_t s_ctx[2 * 74 * 64];  // N, N' staging of the largest register-resident class
  static_assert(2 * 74 * 64 >= 4 * 37 * 4 * 16, "a 4096-bit four-lane tile's Y, B and T rows fit s_ctx");
  const uint32_t lane = threadIdx.x & 63u;
  // the first tiles of all waves start together and are the costliest (the
  // largest class): spread their start phases as a 4096-bit, window-5 launch does
  stagger<148>(blockIdx.x, 5u);
  for (;;) {
    uint32_t j = 0;
    if (lane == 0) j = atomicAdd(args.counter, 1u);
    j = __builtin_amdgcn_readfirstlane(j);
    if (j >= args.njobs) break;  // every wave leaves once the list is exhausted
    const uint32_t job = args.jobs[j];
    const MixedBatch& mb = args.b[job >> 28];
    const uint32_t tile0 = (job & 0x0FFFFFFFu) * (64u / mb.lanes);
    const uint32_t tb = mb.rows * (256u / mb.lanes);            // this wave's region of the batch's workspace
    uint32_t* const tw = mb.ws + (size_t)blockIdx.x * (tb / 4u);
    switch (mb.family) {
      case kF1024:
        modexp_tile<37, 16, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, mb.out, mb.count,
                                  tw, tb, 0u, tile0, s_ctx);
        break;
      case kF1024B:
        modexp_tile_blk<37, 1, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 16u, mb.out,
                                     mb.count, tw, tb, 0u, tile0);
        break;
      case kF2048:
        modexp_tile<74, 32, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, mb.out, mb.count,
                                  tw, tb, 0u, tile0, s_ctx);
        break;
      case kF2048B:
        modexp_tile_blk<37, 2, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 32u, mb.out,
                                     mb.count, tw, tb, 0u, tile0);
        break;
      case kF3072B:
        if (mb.lanes == 4)  // the tile's arrays in the LDS that register-resident tiles stage N, N' in
          modexp_tile_blk<37, 3, true, false, 4, false, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords,
                                                              mb.w, 48u, mb.out, mb.count, tw, tb, 0u, tile0, s_ctx);
        else if (mb.lanes == 2)
          modexp_tile_blk<37, 3, true, false, 2>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 48u,
                                                 mb.out, mb.count, tw, tb, 0u, tile0);
        else
          modexp_tile_blk<37, 3, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 48u, mb.out,
                                       mb.count, tw, tb, 0u, tile0);
        break;
      case kF2048K:
        modexp_tile_blk<37, 2, true, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 32u, mb.out,
                                           mb.count, tw, tb, 0u, tile0);
        break;
      case kF4096K:
        modexp_tile_blk<37, 4, true, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 64u, mb.out,
                                           mb.count, tw, tb, 0u, tile0);
        break;
      default:  // 4096 bits, schoolbook
        if (mb.lanes == 4)
          modexp_tile_blk<37, 4, true, false, 4, false, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords,
                                                              mb.w, 64u, mb.out, mb.count, tw, tb, 0u, tile0, s_ctx);
        else if (mb.lanes == 2)
          modexp_tile_blk<37, 4, true, false, 2>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 64u,
                                                 mb.out, mb.count, tw, tb, 0u, tile0);
        else
          modexp_tile_blk<37, 4, true>(mb.ctx, mb.cidx, mb.base, mb.ex, mb.ebits, mb.ewords, mb.w, 64u, mb.out,
                                       mb.count, tw, tb, 0u, tile0);
        break;
    }
  }
}

// seeded fill for the autotuner's sample inputs: row r, word k of `words`
__global__ void k_fill(uint64_t* p, uint32_t rows, uint32_t words, uint32_t topbits, uint64_t seed) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  uint64_t x = seed ^ (0x9E3779B97F4A7C15ull * (r + 1));
  for (uint32_t k = 0; k < words; ++k) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    uint64_t v = x;
    if (k == words - 1 && topbits < 64) v &= (1ull << topbits) - 1ull;
    p[(size_t)r * words + k] = v;
  }
}

}  // namespace mx

namespace {

// Lanes per instance of a batch: MX_ONE_LANE, MX_TWO_LANES or MX_FOUR_LANES where the family has
// them (the block schoolbook kernels of 3072 and 4096 bits), else the default: two for 4096-bit
// schoolbook tiles (the longest, which otherwise bound the launch), one for the rest.  0 if the flags
// ask for what the family does not have.
uint32_t lanes_of(uint32_t fam, uint32_t flags) {
  const bool two_ok = fam == mx::kF3072B || fam == mx::kF4096B;
  if (flags & MX_FOUR_LANES) return two_ok ? 4u : 0u;
  if (flags & MX_TWO_LANES) return two_ok ? 2u : 0u;
  if (flags & MX_ONE_LANE) return 1u;
  return fam == mx::kF4096B ? 2u : 1u;
}

bool family_of(const mont_ctx* c, uint32_t flags, uint32_t* fam) {
  const bool blk = (flags & MX_IMPL_BLOCK) != 0, kara = (flags & MX_MUL_KARATSUBA) != 0;
  switch (c->bits) {
    case 1024:
      if (kara) return false;
      *fam = blk ? mx::kF1024B : mx::kF1024;
      return true;
    case 2048: *fam = kara ? mx::kF2048K : (blk ? mx::kF2048B : mx::kF2048); return true;
    case 3072:
      if (kara) return false;
      *fam = mx::kF3072B;
      return true;
    case 4096: *fam = kara ? mx::kF4096K : mx::kF4096B; return true;
    default: return false;
  }
}

}  // namespace

struct mx_mixed_plan {
  int device = 0;
  uint32_t nbatch = 0, njobs = 0, nslots = 0;
  mx::MixedArgs args{};
  uint32_t* d_jobs = nullptr;
  uint32_t* d_counter = nullptr;
  void* ws[mx::kMaxMixedBatches] = {};
  bool has_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

mx_status mx_mixed_plan_create(mx_mixed_plan** out, const mx_batch_desc* batches, uint32_t nbatch) {
  if (!out) return mx_fail(MX_EINVAL, "mx_mixed_plan_create: out is NULL");
  *out = nullptr;
  if (!batches || nbatch == 0 || nbatch > (uint32_t)mx::kMaxMixedBatches)
    return mx_fail(MX_EINVAL, "mx_mixed_plan_create: need 1..%d batches", mx::kMaxMixedBatches);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mx_fail(MX_EDEVICE, "mx_mixed_plan_create: no device");
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return mx_fail(MX_EDEVICE, "mx_mixed_plan_create: cannot query compute units");
  std::vector<uint32_t> fam(nbatch);
  uint64_t total_tiles = 0;
  for (uint32_t b = 0; b < nbatch; ++b) {
    const mx_batch_desc& d = batches[b];
    if (!d.ctx) return mx_fail(MX_EINVAL, "batch %u: ctx is NULL", b);
    if (d.ctx->device != dev) return mx_fail(MX_EINVAL, "batch %u: context lives on another device", b);
    if (d.flags & ~(uint32_t)(MX_IMPL_BLOCK | MX_MUL_KARATSUBA | MX_ONE_LANE | MX_TWO_LANES | MX_FOUR_LANES))
      return mx_fail(MX_EUNSUPPORTED, "batch %u: the mixed launch runs the truncated reduction only", b);
    const uint32_t lf = d.flags & (uint32_t)(MX_ONE_LANE | MX_TWO_LANES | MX_FOUR_LANES);
    if (lf & (lf - 1))
      return mx_fail(MX_EINVAL, "batch %u: MX_ONE_LANE, MX_TWO_LANES and MX_FOUR_LANES exclude each other", b);
    if (!family_of(d.ctx, d.flags, &fam[b]))
      return mx_fail(MX_EUNSUPPORTED, "batch %u: %u-bit class not in the mixed launch", b, d.ctx->bits);
    if (lanes_of(fam[b], d.flags) == 0)
      return mx_fail(MX_EUNSUPPORTED, "batch %u: two or four lanes per instance exist for the 3072- and "
                     "4096-bit schoolbook tiles only", b);
    if (d.n && (!d.base || !d.out || (d.exp_bits && !d.exp))) return mx_fail(MX_EINVAL, "batch %u: NULL pointer", b);
    if (!d.ctx_idx && d.n > d.ctx->count) return mx_fail(MX_EINVAL, "batch %u: n exceeds the context count", b);
    if (d.window > 8) return mx_fail(MX_EINVAL, "batch %u: window outside 1..8", b);
    const uint32_t per_tile = 64u / lanes_of(fam[b], d.flags);
    total_tiles += (d.n + per_tile - 1) / per_tile;
  }
  if (total_tiles >= (1u << 28)) return mx_fail(MX_EINVAL, "mx_mixed_plan_create: too many tiles");
  mx_mixed_plan* p = new (std::nothrow) mx_mixed_plan;
  if (!p) return mx_fail(MX_ENOMEM, "mx_mixed_plan_create: host allocation");
  p->device = dev;
  p->nbatch = nbatch;
  p->njobs = (uint32_t)total_tiles;
  p->nslots = (uint32_t)std::min<uint64_t>((uint64_t)cus * 4u, std::max<uint64_t>(total_tiles, 1));
  p->args.njobs = p->njobs;
  hipError_t e = hipSuccess;
  // jobs: every tile of every batch, the costliest first
  struct Tile {
    float cost;
    uint32_t code;
  };
  std::vector<Tile> tiles;
  tiles.reserve(total_tiles);
  for (uint32_t b = 0; b < nbatch && e == hipSuccess; ++b) {
    const mx_batch_desc& d = batches[b];
    const mont_ctx* c = d.ctx;
    // default window: 3 up to 2048 bits (table cache-resident), 5 above (6 needs > 2 GiB per slot set)
    const uint32_t w = d.window ? d.window : (c->bits <= 2048 ? 3u : 5u);
    const int impl = (d.flags & MX_MUL_KARATSUBA) ? 2 : ((d.flags & MX_IMPL_BLOCK) || c->bits > 2048 ? 1 : 0);
    const uint32_t rows = c->ops->ws_rows(impl, true, w);
    const size_t bytes = (size_t)rows * p->nslots * 64u * sizeof(uint32_t);
    if (bytes > mx::kMaxWsBytes) {
      mx_mixed_plan_destroy(p);  // frees the workspaces of the batches before this one
      return mx_fail(MX_EUNSUPPORTED, "batch %u: window %u needs %zu workspace bytes (> 2 GiB); use a smaller window",
                   b, w, bytes);
    }
    e = hipMalloc(&p->ws[b], bytes ? bytes : 4);
    mx::MixedBatch& mb = p->args.b[b];
    mb.ctx = c->dev;
    mb.cidx = d.ctx_idx;
    mb.base = d.base;
    mb.ex = d.exp;
    mb.out = d.out;
    mb.ws = (uint32_t*)p->ws[b];
    mb.count = d.n;
    mb.ebits = d.exp_bits;
    mb.ewords = (d.exp_bits + 63) / 64;
    mb.w = w;
    mb.family = fam[b];
    mb.rows = rows;
    // by default the longest tiles (4096-bit schoolbook) run two lanes per instance: their tile
    // takes about 0.8 of the one-lane time, so the launch is not bound by them
    mb.lanes = lanes_of(fam[b], d.flags);
    const uint32_t per_tile = 64u / mb.lanes;
    const float est = (float)c->limbs * c->limbs * (float)(d.exp_bits ? d.exp_bits : 1) * (mb.lanes == 2 ? 0.8f : 1.f);
    const float cost = d.tile_cost > 0.f ? d.tile_cost : est;
    for (uint32_t t = 0; t < (d.n + per_tile - 1) / per_tile; ++t) tiles.push_back({cost, (b << 28) | t});
  }
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& x, const Tile& y) { return x.cost > y.cost; });
  std::vector<uint32_t> jobs(tiles.size());
  for (size_t i = 0; i < tiles.size(); ++i) jobs[i] = tiles[i].code;
  if (e == hipSuccess && jobs.size() != p->njobs) e = hipErrorInvalidValue;  // the kernel reads njobs entries
  if (e == hipSuccess) e = hipMalloc(&p->d_jobs, std::max<size_t>(jobs.size(), 1) * sizeof(uint32_t));
  if (e == hipSuccess && !jobs.empty())
    e = hipMemcpy(p->d_jobs, jobs.data(), jobs.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_counter, sizeof(uint32_t));
  if (e != hipSuccess) {
    mx_mixed_plan_destroy(p);
    return mx_fail(e == hipErrorOutOfMemory ? MX_ENOMEM : MX_EDEVICE, "mx_mixed_plan_create: %s",
                 hipGetErrorString(e));
  }
  p->args.jobs = p->d_jobs;
  p->args.counter = p->d_counter;
  *out = p;
  return MX_OK;
}

static hipError_t enqueue(mx_mixed_plan* p, hipStream_t st) {
  hipLaunchKernelGGL(mx::k_reset_counter, dim3(1), dim3(64), 0, st, p->d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p->njobs == 0) return e;
  hipLaunchKernelGGL(mx::k_modexp_mixed, dim3(p->nslots), dim3(64), 0, st, p->args);
  return hipGetLastError();
}

mx_status mx_mixed_plan_launch(mx_mixed_plan* p, void* stream) {
  if (!p) return mx_fail(MX_EINVAL, "mx_mixed_plan_launch: plan is NULL");
  hipError_t e = enqueue(p, (hipStream_t)stream);
  if (e != hipSuccess) return mx_fail(MX_EDEVICE, "mx_mixed_plan_launch: %s", hipGetErrorString(e));
  return MX_OK;
}

mx_status mx_mixed_plan_launch_graph(mx_mixed_plan* p, void* stream) {
  if (!p) return mx_fail(MX_EINVAL, "mx_mixed_plan_launch_graph: plan is NULL");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (!p->has_graph) {
    // capture on a private stream so the caller's stream may be the legacy default stream
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = enqueue(p, cap);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cap, &g);
      if (e == hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
      if (e == hipSuccess) {
        p->graph = g;
        p->has_graph = true;
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
    }
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return mx_fail(MX_EDEVICE, "mx_mixed_plan_launch_graph: capture: %s", hipGetErrorString(e));
  }
  e = hipGraphLaunch(p->exec, st);
  if (e != hipSuccess) return mx_fail(MX_EDEVICE, "mx_mixed_plan_launch_graph: %s", hipGetErrorString(e));
  return MX_OK;
}

mx_status mx_mixed_plan_query(const mx_mixed_plan* p, uint32_t* njobs, uint32_t* nslots, uint32_t* windows) {
  if (!p) return mx_fail(MX_EINVAL, "mx_mixed_plan_query: plan is NULL");
  if (njobs) *njobs = p->njobs;
  if (nslots) *nslots = p->nslots;
  if (windows)
    for (uint32_t b = 0; b < p->nbatch; ++b) windows[b] = p->args.b[b].w;
  return MX_OK;
}

void mx_mixed_plan_destroy(mx_mixed_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  for (auto* w : p->ws)
    if (w) (void)hipFree(w);
  if (p->d_jobs) (void)hipFree(p->d_jobs);
  if (p->d_counter) (void)hipFree(p->d_counter);
  delete p;
}

mx_status mx_tune_modexp(const mont_ctx* ctx, uint32_t n, uint32_t exp_bits, const uint32_t* windows,
                         uint32_t nwin, uint32_t try_block, uint32_t reps, uint32_t* best_window,
                         uint32_t* best_flags, float* best_ms, void* stream) {
  if (!ctx || !windows || nwin == 0 || n == 0 || !best_window || !best_flags || !best_ms)
    return mx_fail(MX_EINVAL, "mx_tune_modexp: bad arguments");
  if (n > ctx->count) return mx_fail(MX_EINVAL, "mx_tune_modexp: n exceeds the context count");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t W = (ctx->bits + 63) / 64, ew = (exp_bits + 63) / 64;
  uint64_t *base = nullptr, *ex = nullptr, *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  const uint32_t fam_flags[3] = {0u, (uint32_t)MX_IMPL_BLOCK, (uint32_t)MX_MUL_KARATSUBA};
  for (uint32_t impl = 0; impl < 3; ++impl) {  // one workspace large enough for every candidate
    if ((impl == 1 && !ctx->ops->has_block) || (impl == 2 && !ctx->ops->has_kara) || (impl > 0 && !try_block))
      continue;
    for (uint32_t k = 0; k < nwin; ++k) {
      size_t b = 0;
      if (modexp_ws_bytes(ctx, n, windows[k], fam_flags[impl], &b) != MX_OK) return MX_EINVAL;
      ws_bytes = std::max(ws_bytes, b);
    }
  }
  hipError_t e = hipMalloc(&base, (size_t)n * W * 8);
  if (e == hipSuccess) e = hipMalloc(&ex, (size_t)n * std::max(ew, 1u) * 8);
  if (e == hipSuccess) e = hipMalloc(&out, (size_t)n * W * 8);
  if (e == hipSuccess) e = hipMalloc(&ws, ws_bytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    // bases below 2^(bits-1) <= N; exponents uniform
    const uint32_t topb = (ctx->bits - 1) - 64 * (W - 1);
    hipLaunchKernelGGL(mx::k_fill, dim3((n + 255) / 256), dim3(256), 0, st, base, n, W, topb, 0x1234567ull);
    if (ew) {
      const uint32_t tope = exp_bits - 64 * (ew - 1);
      hipLaunchKernelGGL(mx::k_fill, dim3((n + 255) / 256), dim3(256), 0, st, ex, n, ew, tope, 0x89abcdefull);
    }
    e = hipGetLastError();
  }
  mx_status rs = MX_OK;
  float best = 1e30f;
  for (uint32_t impl = 0; impl < 3 && e == hipSuccess; ++impl) {
    if (impl > 0 && !try_block) break;
    if (impl == 1 && !ctx->ops->has_block) continue;
    if (impl == 2 && !ctx->ops->has_kara) continue;
    for (uint32_t k = 0; k < nwin && e == hipSuccess; ++k) {
      const uint32_t flags = fam_flags[impl];
      rs = modexp_batch_ws(ctx, nullptr, base, ex, exp_bits, windows[k], out, n, flags, ws, ws_bytes,
                           stream);  // warm-up
      if (rs != MX_OK) break;
      float ms = 1e30f;
      for (uint32_t r = 0; r < std::max(reps, 1u) && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess)
          rs = modexp_batch_ws(ctx, nullptr, base, ex, exp_bits, windows[k], out, n, flags, ws, ws_bytes, stream);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess) ms = std::min(ms, t);
      }
      if (rs != MX_OK) break;
      if (ms < best) {
        best = ms;
        *best_window = windows[k];
        *best_flags = flags;
      }
    }
    if (rs != MX_OK) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (base) (void)hipFree(base);
  if (ex) (void)hipFree(ex);
  if (out) (void)hipFree(out);
  if (ws) (void)hipFree(ws);
  if (rs != MX_OK) return rs;  // modexp_batch_ws recorded the message
  if (e != hipSuccess) return mx_fail(MX_EDEVICE, "mx_tune_modexp: %s", hipGetErrorString(e));
  *best_ms = best * 64.f / (float)n;  // per 64-instance tile
  return MX_OK;
}

}  // extern "C"
