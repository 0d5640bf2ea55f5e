// Per-size-class instantiation of the kernels.  Built once per class with
// -DMX_CLASS_BITS=<bits>; each object exports mx::class_ops_<bits>().
// Classes up to 2048 bits use the register-resident kernels (mx_kernels.hpp);
// larger classes use the block-level schoolbook (mx_block.hpp).  The
// alternative-reduction kernels of a register-resident class (the
// word-interleaved multiplication of Algorithm 4, and the Karatsuba-truncated
// reduction) are built separately, with -DMX_CIOS_UNIT or -DMX_KREDC_UNIT as
// well, so that they compile in parallel with the rest of the class; those
// objects export the launchers cios_mont_<bits>, cios_modexp_<bits> and
// kredc_mont_<bits> (MX_CIOS_UNIT), and kredc_modexp_<bits> (MX_KREDC_UNIT).
#include "mx_block.hpp"
#if defined(MX_CIOS_UNIT) || defined(MX_KREDC_UNIT)
#include "mx_kredc.hpp"
#endif

#ifndef MX_CLASS_BITS
#error "MX_CLASS_BITS must be defined"
#endif

#define MX_CAT2(a, b) a##b
#define MX_CAT(a, b) MX_CAT2(a, b)

namespace mx {

#if MX_CLASS_BITS <= 2048
hipError_t MX_CAT(cios_mont_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                                             const uint64_t* b, uint64_t* out, uint32_t count, uint32_t coff,
                                             hipStream_t st);
hipError_t MX_CAT(cios_modexp_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base,
                                               const uint64_t* ex, uint32_t ebits, uint32_t ewords, uint32_t w,
                                               uint64_t* out, uint32_t count, uint32_t* ws, uint32_t ws_bytes,
                                               uint32_t coff, hipStream_t st);
hipError_t MX_CAT(kredc_mont_, MX_CLASS_BITS)(bool sqr, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                                              const uint64_t* b, uint64_t* out, uint32_t count, uint32_t coff,
                                              hipStream_t st);
hipError_t MX_CAT(kredc_modexp_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base,
                                                const uint64_t* ex, uint32_t ebits, uint32_t ewords, uint32_t w,
                                                uint64_t* out, uint32_t count, uint32_t* ws, uint32_t ws_bytes,
                                                uint32_t coff, hipStream_t st);
#endif

#ifdef MX_CIOS_UNIT
static_assert(MX_CLASS_BITS <= 2048, "the word-interleaved kernels exist for the register-resident classes");
constexpr int kCiosN = limbs_for(MX_CLASS_BITS);
hipError_t MX_CAT(kredc_mont_, MX_CLASS_BITS)(bool sqr, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                                              const uint64_t* b, uint64_t* out, uint32_t count, uint32_t coff,
                                              hipStream_t st) {
  constexpr int RW = words_for(28 * kCiosN);
  if (sqr)
    hipLaunchKernelGGL((k_mont_kredc<kCiosN, RW, true>), dim3((count + 63) / 64), dim3(64), 0, st, ctx, cidx, a, b,
                       out, count, coff);
  else
    hipLaunchKernelGGL((k_mont_kredc<kCiosN, RW, false>), dim3((count + 63) / 64), dim3(64), 0, st, ctx, cidx, a, b,
                       out, count, coff);
  return hipGetLastError();
}
hipError_t MX_CAT(cios_mont_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                                             const uint64_t* b, uint64_t* out, uint32_t count, uint32_t coff,
                                             hipStream_t st) {
  hipLaunchKernelGGL((k_mont_cios<kCiosN, words_for(28 * kCiosN)>), dim3((count + 63) / 64), dim3(64), 0, st, ctx,
                     cidx, a, b, out, count, coff);
  return hipGetLastError();
}
hipError_t MX_CAT(cios_modexp_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base,
                                               const uint64_t* ex, uint32_t ebits, uint32_t ewords, uint32_t w,
                                               uint64_t* out, uint32_t count, uint32_t* ws, uint32_t ws_bytes,
                                               uint32_t coff, hipStream_t st) {
  hipLaunchKernelGGL((k_modexp_cios<kCiosN, words_for(MX_CLASS_BITS)>), dim3((count + 63) / 64), dim3(64), 0, st,
                     ctx, cidx, base, ex, ebits, ewords, w, out, count, ws, ws_bytes, coff);
  return hipGetLastError();
}
}  // namespace mx
#elif defined(MX_KREDC_UNIT)
static_assert(MX_CLASS_BITS <= 2048, "the Karatsuba-truncated kernels exist for the register-resident classes");
constexpr int kKredcN = limbs_for(MX_CLASS_BITS);
hipError_t MX_CAT(kredc_modexp_, MX_CLASS_BITS)(const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base,
                                                const uint64_t* ex, uint32_t ebits, uint32_t ewords, uint32_t w,
                                                uint64_t* out, uint32_t count, uint32_t* ws, uint32_t ws_bytes,
                                                uint32_t coff, hipStream_t st) {
  hipLaunchKernelGGL((k_modexp_kredc<kKredcN, words_for(MX_CLASS_BITS)>), dim3((count + 63) / 64), dim3(64), 0, st,
                     ctx, cidx, base, ex, ebits, ewords, w, out, count, ws, ws_bytes, coff);
  return hipGetLastError();
}
}  // namespace mx
#else
namespace {

constexpr int kBits = MX_CLASS_BITS;
constexpr bool kBlock = kBits > 2048;                     // only the block kernels exist
constexpr int kH = 37;                                    // block limbs
constexpr int kK = (limbs_for(kBits) + kH - 1) / kH;      // blocks
constexpr int kN = kBlock ? kH * kK : limbs_for(kBits);   // limbs, R = 2^(28 kN)
constexpr bool kHasBlk = kN % kH == 0;                    // block kernels also built (same R)
constexpr bool kHasKara = kHasBlk && kK % 2 == 0;         // one-level Karatsuba needs an even block count
constexpr int kW = words_for(kBits);                      // canonical values (< N)
constexpr int kRW = words_for(28 * kN);                   // Montgomery-domain values (< 2N < R)

static_assert(!kHasBlk || (kK >= 1 && kK <= 4), "block kernels: redundant limbs need K <= 4");
// block exponentiations of at most this many instances run four (two) lanes
// per instance: 65536 lanes = one wavefront on each of MI355X's 1024 SIMDs
constexpr uint32_t kFourLaneMax = 32768;  // four lanes (arrays in LDS) beat one and two up to here
constexpr uint32_t kTwoLaneMax = 32768;

// k_modexp with a register budget for two wavefronts per SIMD: at 1024 bits the
// exponentiation fits 256 registers per lane with a few spills, and two
// wavefronts on a SIMD hide each other's issue stalls (measured 6-8 % faster
// than the 512-register build at 65536 and 131072 instances, same results).
template <int N, int BW, bool TRUNC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_modexp_2w(CtxDev ctx, const uint32_t* __restrict__ cidx, const uint64_t* __restrict__ base,
            const uint64_t* __restrict__ ex, uint32_t ebits, uint32_t ewords, uint32_t w, uint64_t* __restrict__ out,
            uint32_t count, uint32_t* __restrict__ ws, uint32_t ws_bytes, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * N * 64];
  const uint32_t tile0 = blockIdx.x * 64;
  const uint32_t tbytes = (1u << w) * (uint32_t)packed_words(N) * 256u;
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  stagger<N>(blockIdx.x, w);
  modexp_tile<N, BW, TRUNC>(ctx, cidx, base, ex, ebits, ewords, w, out, count, ws + (size_t)blockIdx.x * (tbytes / 4u),
                            tbytes, coff, tile0, s_ctx);
}
constexpr bool kTwoWaves = kBits == 1024;

// Two batches of `count` instances in one launch of k_modexp_2w's code (the two
// half-size exponentiations of a CRT-RSA operation): blocks below ceil(count/64)
// take batch 0 (context c0, exponents e0), the others batch 1 (c1, e1); bases
// and outputs are one array with batch 1 from instance `count` on.  With two
// wavefronts per SIMD, one launch over both halves fills both wavefront slots.
template <int N, int BW, bool TRUNC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_modexp_2w_pair(CtxDev c0, CtxDev c1, const uint32_t* __restrict__ cidx, const uint64_t* __restrict__ base,
                 const uint64_t* __restrict__ e0, const uint64_t* __restrict__ e1, uint32_t ebits, uint32_t ewords,
                 uint32_t w, uint64_t* __restrict__ out, uint32_t count, uint32_t* __restrict__ ws,
                 uint32_t ws_bytes) {
  __shared__ uint32_t s_ctx[2 * N * 64];
  const uint32_t nb = (count + 63) / 64;
  const bool second = blockIdx.x >= nb;
  const uint32_t tile0 = (blockIdx.x - (second ? nb : 0u)) * 64;
  const uint32_t tbytes = (1u << w) * (uint32_t)packed_words(N) * 256u;
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  const size_t off = second ? (size_t)count * BW : 0;
  stagger<N>(blockIdx.x, w);
  modexp_tile<N, BW, TRUNC>(second ? c1 : c0, cidx, base + off, second ? e1 : e0, ebits, ewords, w, out + off,
                            count, ws + (size_t)blockIdx.x * (tbytes / 4u), tbytes, 0u, tile0, s_ctx);
}

hipError_t ctx_fn(const uint64_t* mods, const CtxDev& ctx, hipStream_t st) {
  const uint32_t blocks = (ctx.count + 63) / 64;
  hipLaunchKernelGGL((k_ctx_init<kN, kW>), dim3(blocks), dim3(64), 0, st, mods, ctx);
  return hipGetLastError();
}

// per-lane workspace words: block classes keep Y, B, T, Q, S (and the table)
// in memory; register-resident classes need only the exponentiation table
uint32_t ws_rows_fn(int impl, bool modexp, uint32_t w) {
  // impl: 0 register-resident, 1 block, 2 block + Karatsuba, 3 block with one lane per instance,
  // 4 block with at most two lanes per instance
  if (kBlock || (kHasBlk && impl >= 1)) return modexp ? BlkLayout<kH, kK>::rows(w) : BlkLayout<kH, kK>::G;
  (void)impl;
  return modexp ? (1u << w) * (uint32_t)packed_words(kN) : 0u;  // densely packed table entries
}

hipError_t mont_fn(int impl, int redc, bool sqr, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                   const uint64_t* b, uint64_t* out, uint32_t count, uint32_t* ws, uint32_t tstride,
                   uint32_t ws_bytes, uint32_t coff, hipStream_t st) {
  const uint32_t blocks = (count + 63) / 64;
  const bool trunc = redc == kRedcTrunc;
  // every block's region must lie in ws: checked here, before anything is enqueued
  if ((uint64_t)ws_rows_fn(impl, false, 0) * 256u * blocks > ws_bytes) return hipErrorInvalidValue;
  if constexpr (kBlock) {  // block-word CIOS (Algorithm 4 with 37-limb words), one lane per instance
    if (redc == kRedcCios) {
      if (sqr)
        hipLaunchKernelGGL((k_mont_blk<kH, kK, false, true, false, false, true>), dim3(blocks), dim3(64), 0, st,
                           ctx, cidx, a, b, out, count, ws, ws_bytes, coff);
      else
        hipLaunchKernelGGL((k_mont_blk<kH, kK, false, false, false, false, true>), dim3(blocks), dim3(64), 0, st,
                           ctx, cidx, a, b, out, count, ws, ws_bytes, coff);
      return hipGetLastError();
    }
  }
  if constexpr (kHasKara) {
    // block kernels with the Karatsuba-truncated q N (one lane per instance); impl 2 also forms the
    // product by Karatsuba
    if (redc == kRedcKara && (kBlock || impl >= 1)) {
#define MX_L(KA, S)                                                                                                 \
  hipLaunchKernelGGL((k_mont_blk<kH, kK, true, S, KA, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, \
                     count, ws, ws_bytes, coff)
      if (impl == 2) {
        if (sqr) MX_L(true, true); else MX_L(true, false);
      } else {
        if (sqr) MX_L(false, true); else MX_L(false, false);
      }
#undef MX_L
      return hipGetLastError();
    }
    if (impl == 2) {
#define MX_L(T, S)                                                                                                \
  hipLaunchKernelGGL((k_mont_blk<kH, kK, T, S, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count, \
                     ws, ws_bytes, coff)
      if (trunc) {
        if (sqr) MX_L(true, true); else MX_L(true, false);
      } else {
        if (sqr) MX_L(false, true); else MX_L(false, false);
      }
#undef MX_L
      return hipGetLastError();
    }
  }
  if constexpr (kBlock || kHasBlk) {
    if (kBlock || impl == 1) {
#define MX_L(T, S)                                                                                              \
  hipLaunchKernelGGL((k_mont_blk<kH, kK, T, S>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count, ws, \
                     ws_bytes, coff)
      if (trunc) {
        if (sqr) MX_L(true, true); else MX_L(true, false);
      } else {
        if (sqr) MX_L(false, true); else MX_L(false, false);
      }
#undef MX_L
      return hipGetLastError();
    }
  }
  if constexpr (!kBlock) {
    (void)ws;
    (void)tstride;
    (void)ws_bytes;
#if MX_CLASS_BITS <= 2048
    // a square is the product with b = a (the caller passes a twice)
    if (redc == kRedcCios) return MX_CAT(cios_mont_, MX_CLASS_BITS)(ctx, cidx, a, b, out, count, coff, st);
    if (redc == kRedcKara) return MX_CAT(kredc_mont_, MX_CLASS_BITS)(sqr, ctx, cidx, a, b, out, count, coff, st);
#endif
#define MX_L(T, S) \
  hipLaunchKernelGGL((k_mont<kN, kRW, T, S>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count, coff)
    if (trunc) {
      if (sqr) MX_L(true, true); else MX_L(true, false);
    } else {
      if (sqr) MX_L(false, true); else MX_L(false, false);
    }
#undef MX_L
  }
  return hipGetLastError();
}

hipError_t modexp_fn(int impl, int redc, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base, const uint64_t* ex,
                     uint32_t ebits, uint32_t ewords, uint32_t w, uint64_t* out, uint32_t count, uint32_t* ws,
                     uint32_t tstride, uint32_t ws_bytes, uint32_t coff, hipStream_t st) {
  // each block works in its own tile region of ws (ws_rows x 64 words); tstride,
  // the launch width padded to 64, only sized ws
  (void)tstride;
  const uint32_t blocks = (count + 63) / 64;
  const bool trunc = redc == kRedcTrunc;
  // every block's region must lie in ws (with LP lanes per instance a block's region is 1/LP of a
  // 64-instance tile's): checked here, before anything is enqueued
  if ((uint64_t)ws_rows_fn(impl, true, w) * 256u * blocks > ws_bytes) return hipErrorInvalidValue;
  if constexpr (kBlock) {  // block-word CIOS, one lane per instance
    if (redc == kRedcCios) {
      hipLaunchKernelGGL((k_modexp_blk<kH, kK, false, false, 1, false, true>), dim3(blocks), dim3(64), 0, st, ctx,
                         cidx, base, ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      return hipGetLastError();
    }
  }
  if constexpr (kHasKara) {
    // block kernels with the Karatsuba-truncated q N: one lane per instance
    if (redc == kRedcKara && (kBlock || impl >= 1)) {
      if (impl == 2)
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, true, true, 1, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base,
                           ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      else
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, true, false, 1, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx,
                           base, ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      return hipGetLastError();
    }
    if (impl == 2) {
      if (trunc)
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, true, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex,
                           ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      else
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, false, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex,
                           ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      return hipGetLastError();
    }
  }
  if constexpr (kBlock || kHasBlk) {
    if (kBlock || impl == 1 || impl == 3 || impl == 4 || impl == 5) {
      // a batch of at most two wavefronts per SIMD at four lanes runs four lanes per
      // instance (lower latency, and faster than one or two lanes at these sizes)
      // unless one lane (impl 3) or at most two (impl 4) were asked for; four at any
      // size when asked for (impl 5); the workspace has room for any of them
      if ((count <= kFourLaneMax && impl != 3 && impl != 4) || impl == 5) {
        const uint32_t blocks4 = (count + 15) / 16;
        if (trunc)
          hipLaunchKernelGGL((k_modexp_blk<kH, kK, true, false, 4>), dim3(blocks4), dim3(64), 0, st, ctx, cidx, base,
                             ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
        else
          hipLaunchKernelGGL((k_modexp_blk<kH, kK, false, false, 4>), dim3(blocks4), dim3(64), 0, st, ctx, cidx,
                             base, ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
        return hipGetLastError();
      }
      if (count <= kTwoLaneMax && impl != 3) {
        const uint32_t blocks2 = (count + 31) / 32;
        if (trunc)
          hipLaunchKernelGGL((k_modexp_blk<kH, kK, true, false, 2>), dim3(blocks2), dim3(64), 0, st, ctx, cidx, base,
                             ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
        else
          hipLaunchKernelGGL((k_modexp_blk<kH, kK, false, false, 2>), dim3(blocks2), dim3(64), 0, st, ctx, cidx,
                             base, ex, ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
        return hipGetLastError();
      }
      if (trunc)
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits,
                           ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      else
        hipLaunchKernelGGL((k_modexp_blk<kH, kK, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex,
                           ebits, ewords, w, (uint32_t)kW, out, count, ws, ws_bytes, coff);
      return hipGetLastError();
    }
  }
  if constexpr (!kBlock) {
#if MX_CLASS_BITS <= 2048
    if (redc == kRedcCios)
      return MX_CAT(cios_modexp_, MX_CLASS_BITS)(ctx, cidx, base, ex, ebits, ewords, w, out, count, ws, ws_bytes, coff,
                                                 st);
    if (redc == kRedcKara)
      return MX_CAT(kredc_modexp_, MX_CLASS_BITS)(ctx, cidx, base, ex, ebits, ewords, w, out, count, ws, ws_bytes,
                                                  coff, st);
#endif
    if constexpr (kTwoWaves) {
      if (trunc)
        hipLaunchKernelGGL((k_modexp_2w<kN, kW, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits,
                           ewords, w, out, count, ws, ws_bytes, coff);
      else
        hipLaunchKernelGGL((k_modexp_2w<kN, kW, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits,
                           ewords, w, out, count, ws, ws_bytes, coff);
    } else if (trunc) {
      hipLaunchKernelGGL((k_modexp<kN, kW, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits, ewords,
                         w, out, count, ws, ws_bytes, coff);
    } else {
      hipLaunchKernelGGL((k_modexp<kN, kW, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits,
                         ewords, w, out, count, ws, ws_bytes, coff);
    }
  }
  return hipGetLastError();
}

// the word-interleaved kernels (Algorithm 4) exist for the register-resident classes
hipError_t modexp_pair_fn(bool trunc, const CtxDev& c0, const CtxDev& c1, const uint32_t* cidx,
                          const uint64_t* base, const uint64_t* e0, const uint64_t* e1, uint32_t ebits,
                          uint32_t ewords, uint32_t w, uint64_t* out, uint32_t count, uint32_t* ws, uint32_t ws_bytes,
                          hipStream_t st) {
  if constexpr (kTwoWaves) {
    const uint32_t blocks = 2 * ((count + 63) / 64);
    if ((uint64_t)ws_rows_fn(0, true, w) * 256u * blocks > ws_bytes) return hipErrorInvalidValue;
    if (trunc)
      hipLaunchKernelGGL((k_modexp_2w_pair<kN, kW, true>), dim3(blocks), dim3(64), 0, st, c0, c1, cidx, base, e0,
                         e1, ebits, ewords, w, out, count, ws, ws_bytes);
    else
      hipLaunchKernelGGL((k_modexp_2w_pair<kN, kW, false>), dim3(blocks), dim3(64), 0, st, c0, c1, cidx, base, e0,
                         e1, ebits, ewords, w, out, count, ws, ws_bytes);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

// has_cios: word-interleaved products in the register-resident classes, block-word CIOS above 2048 bits
const ClassOps kOps = {kBits, kN, kHasBlk || kBlock, kHasKara, true, ctx_fn, ws_rows_fn, mont_fn, modexp_fn,
                       kTwoWaves ? modexp_pair_fn : nullptr};

}  // namespace

const ClassOps* MX_CAT(class_ops_, MX_CLASS_BITS)() { return &kOps; }

}  // namespace mx
#endif  // MX_CIOS_UNIT / MX_KREDC_UNIT
