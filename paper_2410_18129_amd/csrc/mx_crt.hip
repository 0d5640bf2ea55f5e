// RSA private-key operations by the Chinese remainder theorem: the
// application the paper's batched exponentiation serves (Section 1).  For a
// key (p, q, dp = d mod (p-1), dq = d mod (q-1), qinv = q^{-1} mod p) and a
// ciphertext c < p q:
//   m1 = (c mod p)^dp mod p,  m2 = (c mod q)^dq mod q,
//   h  = qinv (m1 - m2) mod p,  m = m2 + h q          (Garner's recombination)
// and m = c^d mod p q.  The two half-size exponentiations run on the class's
// exponentiation kernels; this unit holds the steps before and after them,
// one instance per lane.  Built per prime class (-DMX_CLASS_BITS = 1024 or
// 2048: RSA-2048 and RSA-4096); exports crt_reduce_<bits> and
// crt_garner_<bits>.  Both primes have exactly MX_CLASS_BITS bits.
#include "mx_kernels.hpp"

#ifndef MX_CLASS_BITS
#error "MX_CLASS_BITS must be defined"
#endif

#define MX_CAT2(a, b) a##b
#define MX_CAT(a, b) MX_CAT2(a, b)

namespace mx {
namespace {

constexpr int kN = limbs_for(MX_CLASS_BITS);  // limbs of a prime, R = 2^(28 kN)
constexpr int kW = words_for(MX_CLASS_BITS);  // words of a value mod p or q
static_assert(2 * kN * kLimbBits >= 2 * 64 * kW, "2 kN limbs hold a value of the modulus n = p q");

// The lane's context index for one of the two contexts of a key.
__device__ __forceinline__ uint32_t key_ctx(const uint32_t* kidx, uint32_t inst, uint32_t coff, uint32_t count) {
  const uint32_t k = kidx ? kidx[inst] : inst + coff;
  return k < count ? k : 0u;
}

// REDC with the prime whose N and N' sit in the lane's LDS column.
__device__ __forceinline__ void redc_lds(const uint32_t (&t)[2 * kN], const uint32_t* sm, uint32_t (&c)[kN]) {
  redc_blk<kN, true>(t, [&](int i) { return sm[i * 64]; }, [&](int i) { return sm[(kN + i) * 64]; }, c);
}

// x mod p for x < p R (p's context staged in LDS, r2 = R^2 mod p): two
// reductions, REDC(REDC(x) * R^2) = x R^{-1} R^2 R^{-1} = x (mod p), each
// below 2p (Section 4: T < p R gives REDC(T) < 2p), then one conditional
// subtraction: canonical.
__device__ __forceinline__ void mod_prime(const uint32_t (&x)[2 * kN], const uint32_t* sm, const uint32_t (&r2)[kN],
                                          uint32_t (&out)[kN]) {
  uint32_t t[2 * kN];
  redc_lds(x, sm, out);
  mul_sb<kN>(out, r2, t);
  redc_lds(t, sm, out);
  uint32_t m[kN];
  sfor<0, kN>([&](auto I) { m[decltype(I)::value] = sm[decltype(I)::value * 64]; });
  canon<kN>(out, m);
}

template <typename T>
__device__ __forceinline__ void load_limbs(const uint32_t* arr, size_t stride, uint32_t c, T (&x)[kN]) {
  sfor<0, kN>([&](auto I) { x[decltype(I)::value] = arr[(size_t)decltype(I)::value * stride + c]; });
}

// cp[i] = c[i] mod p, cq[i] = c[i] mod q (kW words each, canonical);
// c: 2 kW words per instance.
__global__ void __launch_bounds__(64) k_crt_reduce(CtxDev ctxp, CtxDev ctxq, const uint32_t* __restrict__ kidx,
                                                   const uint64_t* __restrict__ c, uint64_t* __restrict__ cp,
                                                   uint64_t* __restrict__ cq, uint32_t count, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * kN * 64];
  const uint32_t lane = threadIdx.x;
  const uint32_t gid = blockIdx.x * 64 + lane;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t x[2 * kN];
  expand<2 * kN, 2 * kW>(c + (size_t)inst * 2 * kW, x);
  const uint32_t* sm = s_ctx + lane;
#pragma unroll 1
  for (int side = 0; side < 2; ++side) {
    const CtxDev& ctx = side == 0 ? ctxp : ctxq;
    const uint32_t k = key_ctx(kidx, inst, coff, ctx.count);
    // the lane rewrites only its own LDS column: no barrier between the two primes
    stage_ctx<kN>(s_ctx, ctx.n + k, ctx.np + k, ctx.stride, lane);
    uint32_t r2[kN], y[kN];
    load_limbs(ctx.r2, ctx.stride, k, r2);
    mod_prime(x, sm, r2, y);
    if (live) contract<kN, kW>(y, (side == 0 ? cp : cq) + (size_t)inst * kW);
  }
}

// out[i] = m2 + h q with h = qinv (m1 - m2) mod p (2 kW words, < p q).
// m1 < p, m2 < q, qinv < p canonical (kW words each).
__global__ void __launch_bounds__(64) k_crt_garner(CtxDev ctxp, CtxDev ctxq, const uint32_t* __restrict__ kidx,
                                                   const uint64_t* __restrict__ m1, const uint64_t* __restrict__ m2,
                                                   const uint64_t* __restrict__ qinv, uint64_t* __restrict__ out,
                                                   uint32_t count, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * kN * 64];
  const uint32_t lane = threadIdx.x;
  const uint32_t gid = blockIdx.x * 64 + lane;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  const uint32_t kp = key_ctx(kidx, inst, coff, ctxp.count);
  const uint32_t kq = key_ctx(kidx, inst, coff, ctxq.count);
  stage_ctx<kN>(s_ctx, ctxp.n + kp, ctxp.np + kp, ctxp.stride, lane);
  const uint32_t* sm = s_ctx + lane;
  uint32_t r2[kN];
  load_limbs(ctxp.r2, ctxp.stride, kp, r2);

  uint32_t t[2 * kN];
  // qinv in Montgomery form: REDC(qinv R^2) = qinv R mod p (below 2p)
  uint32_t qi[kN];
  expand<kN, kW>(qinv + (size_t)inst * kW, qi);
  mul_sb<kN>(qi, r2, t);
  redc_lds(t, sm, qi);
  // m2 mod p (m2 < q < 2^bits < p R)
  uint32_t b[kN], d[kN];
  expand<kN, kW>(m2 + (size_t)inst * kW, b);
  sfor<0, kN>([&](auto I) {
    t[decltype(I)::value] = b[decltype(I)::value];
    t[kN + decltype(I)::value] = 0;
  });
  mod_prime(t, sm, r2, d);
  // d = m1 - (m2 mod p) mod p: subtract, then add p back under the borrow mask
  {
    uint32_t a[kN];
    expand<kN, kW>(m1 + (size_t)inst * kW, a);
    int64_t br = 0;
    sfor<0, kN>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const int64_t v = (int64_t)a[i] - (int64_t)d[i] + br;
      d[i] = (uint32_t)v & kLimbMask;
      br = v >> kLimbBits;  // 0 or -1
    });
    const uint32_t mask = br != 0 ? 0xFFFFFFFFu : 0u;
    uint32_t cy = 0;
    sfor<0, kN>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const uint32_t v = d[i] + (sm[i * 64] & mask) + cy;
      d[i] = v & kLimbMask;
      cy = v >> kLimbBits;
    });
  }
  // h = REDC(d * qinv R) = qinv (m1 - m2) mod p, canonical
  uint32_t h[kN];
  mul_sb<kN>(d, qi, t);
  redc_lds(t, sm, h);
  {
    uint32_t m[kN];
    sfor<0, kN>([&](auto I) { m[decltype(I)::value] = sm[decltype(I)::value * 64]; });
    canon<kN>(h, m);
  }
  // m = m2 + h q: h < p and m2 < q give m < p q, no reduction
  uint32_t qv[kN];
  load_limbs(ctxq.n, ctxq.stride, kq, qv);
  mul_sb<kN>(h, qv, t);
  uint32_t cy = 0;
  sfor<0, 2 * kN>([&](auto I) {
    constexpr int i = decltype(I)::value;
    uint32_t v = t[i] + cy;
    if constexpr (i < kN) v += b[i];
    t[i] = v & kLimbMask;
    cy = v >> kLimbBits;
  });
  if (live) contract<2 * kN, 2 * kW>(t, out + (size_t)inst * 2 * kW);
}

}  // namespace

hipError_t MX_CAT(crt_reduce_, MX_CLASS_BITS)(const CtxDev& ctxp, const CtxDev& ctxq, const uint32_t* kidx,
                                              const uint64_t* c, uint64_t* cp, uint64_t* cq, uint32_t count,
                                              uint32_t coff, hipStream_t st) {
  hipLaunchKernelGGL(k_crt_reduce, dim3((count + 63) / 64), dim3(64), 0, st, ctxp, ctxq, kidx, c, cp, cq, count,
                     coff);
  return hipGetLastError();
}

hipError_t MX_CAT(crt_garner_, MX_CLASS_BITS)(const CtxDev& ctxp, const CtxDev& ctxq, const uint32_t* kidx,
                                              const uint64_t* m1, const uint64_t* m2, const uint64_t* qinv,
                                              uint64_t* out, uint32_t count, uint32_t coff, hipStream_t st) {
  hipLaunchKernelGGL(k_crt_garner, dim3((count + 63) / 64), dim3(64), 0, st, ctxp, ctxq, kidx, m1, m2, qinv, out,
                     count, coff);
  return hipGetLastError();
}

}  // namespace mx
