#pragma once
// Montgomery multiplication and exponentiation whose truncated high half of
// q N is formed by a one-level Karatsuba product (the Karatsuba paragraph of
// Section 5; low_half_q and kara_high_half in mx_core.hpp), for the
// register-resident classes.  Instantiated in the alternative-reduction units
// of mx_class.hip (MX_CIOS_UNIT, MX_KREDC_UNIT).
#include "mx_kernels.hpp"

namespace mx {

// out = REDC(a * b) (a square when the caller passes b = a: the product is
// then formed by sqr_sb) with the Karatsuba high half above.
template <int N, int RW, bool SQR>
__global__ void __launch_bounds__(64) k_mont_kredc(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                   const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                   uint64_t* __restrict__ out, uint32_t count, uint32_t coff) {
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  __shared__ uint32_t s_ctx[2 * N * 64];
  stage_ctx<N>(s_ctx, ctx.n + c, ctx.np + c, ctx.stride, threadIdx.x);
  uint32_t x[N];
  expand<N, RW>(a + (size_t)inst * RW, x);
  uint32_t t[2 * N];
  if constexpr (SQR) {
    sqr_sb<N, RotMad>(x, t);
  } else {
    uint32_t y[N];
    expand<N, RW>(b + (size_t)inst * RW, y);
    mul_sb<N, RotMad>(x, y, t);
  }
  const LdsU32* sm = (const LdsU32*)(s_ctx + threadIdx.x);  // ds_read, as in k_mont
  uint32_t q[N], r[N];
  low_half_q<N, RotMad>(t, [&](int i) { return sm[(N + i) * 64]; }, q);
  kara_high_half<N, RotMad>(t, q, [&](int j) { return sm[j * 64]; }, r);
  if (live) contract<N, RW>(r, out + (size_t)inst * RW);
}

// As k_modexp with every Montgomery product's truncated high half of q N formed by one-level Karatsuba
// (kara_high_half); same results.
template <int N, int BW>
__global__ void __launch_bounds__(64) k_modexp_kredc(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                     const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                                     uint32_t ebits, uint32_t ewords, uint32_t w,
                                                     uint64_t* __restrict__ out, uint32_t count,
                                                     uint32_t* __restrict__ ws, uint32_t ws_bytes, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * N * 64];
  const uint32_t tile0 = blockIdx.x * 64;
  const uint32_t tbytes = (1u << w) * (uint32_t)packed_words(N) * 256u;
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  stagger<N>(blockIdx.x, w);
  modexp_tile<N, BW, true, false, true>(ctx, cidx, base, ex, ebits, ewords, w, out, count,
                                        ws + (size_t)blockIdx.x * (tbytes / 4u), tbytes, coff, tile0, s_ctx);
}

}  // namespace mx
