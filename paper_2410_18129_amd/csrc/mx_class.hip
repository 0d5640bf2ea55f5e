// Per-size-class instantiation of the kernels.  Built once per class with
// -DMX_CLASS_BITS=<bits>; each object exports mx::class_ops_<bits>().
#include "mx_kernels.hpp"

#ifndef MX_CLASS_BITS
#error "MX_CLASS_BITS must be defined"
#endif

namespace mx {
namespace {

constexpr int kBits = MX_CLASS_BITS;
constexpr int kN = limbs_for(kBits);
constexpr int kW = words_for(kBits);        // canonical values (< N)
constexpr int kRW = words_for(28 * kN);     // Montgomery-domain values (< 2N < R)

hipError_t ctx_fn(const uint64_t* mods, const CtxDev& ctx, hipStream_t st) {
  const uint32_t blocks = (ctx.count + 63) / 64;
  hipLaunchKernelGGL((k_ctx_init<kN, kW>), dim3(blocks), dim3(64), 0, st, mods, ctx);
  return hipGetLastError();
}

hipError_t mont_fn(bool trunc, bool sqr, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                   const uint64_t* b, uint64_t* out, uint32_t count, hipStream_t st) {
  const uint32_t blocks = (count + 63) / 64;
  if (trunc) {
    if (sqr)
      hipLaunchKernelGGL((k_mont<kN, kRW, true, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count);
    else
      hipLaunchKernelGGL((k_mont<kN, kRW, true, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count);
  } else {
    if (sqr)
      hipLaunchKernelGGL((k_mont<kN, kRW, false, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count);
    else
      hipLaunchKernelGGL((k_mont<kN, kRW, false, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, a, b, out, count);
  }
  return hipGetLastError();
}

hipError_t modexp_fn(bool trunc, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base, const uint64_t* ex,
                     uint32_t ebits, uint32_t ewords, uint32_t w, uint64_t* out, uint32_t count, uint32_t* table,
                     uint32_t tstride, uint32_t coff, hipStream_t st) {
  const uint32_t blocks = (count + 63) / 64;
  const size_t tbytes = ((size_t)1 << w) * kN * tstride * sizeof(uint32_t);
  if (tbytes > 0x7FFFFFFFull) return hipErrorInvalidValue;  // one buffer descriptor spans < 2 GiB
  if (trunc)
    hipLaunchKernelGGL((k_modexp<kN, kW, true>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits, ewords, w,
                       out, count, table, tstride, (uint32_t)tbytes, coff);
  else
    hipLaunchKernelGGL((k_modexp<kN, kW, false>), dim3(blocks), dim3(64), 0, st, ctx, cidx, base, ex, ebits, ewords,
                       w, out, count, table, tstride, (uint32_t)tbytes, coff);
  return hipGetLastError();
}

const ClassOps kOps = {kBits, kN, ctx_fn, mont_fn, modexp_fn};

}  // namespace

#define MX_CAT2(a, b) a##b
#define MX_CAT(a, b) MX_CAT2(a, b)
const ClassOps* MX_CAT(class_ops_, MX_CLASS_BITS)() { return &kOps; }

}  // namespace mx
