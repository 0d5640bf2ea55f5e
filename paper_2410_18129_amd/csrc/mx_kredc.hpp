#pragma once
// Montgomery multiplication whose truncated high half of q N is formed by a
// one-level Karatsuba product (the Karatsuba paragraph of Section 5), for the
// register-resident classes.  Instantiated in the alternative-reduction unit
// of mx_class.hip (MX_CIOS_UNIT).
#include "mx_kernels.hpp"

namespace mx {

// q = T_lo N' mod R (Algorithm 6, step 1): the low half of T N', column by column.
template <int N, typename M, typename LoadNP>
__device__ __forceinline__ void low_half_q(const uint32_t (&t)[2 * N], LoadNP&& ldnp, uint32_t (&q)[N]) {
  constexpr int BK = kColBlock;
  uint64_t carry = 0;
  sfor<0, (N + BK - 1) / BK>([&](auto B) {
    constexpr int k0 = decltype(B)::value * BK;
    constexpr int bk = (N - k0) < BK ? (N - k0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
    colblock_ld<k0, bk, 0, N - 1, 0, N - 1, M>(t, ldnp, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      const uint64_t v = acc[d] + carry;
      q[k0 + d] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;
    });
    compiler_fence();
  });
}

// C = floor(T / R) + floor(q N / R) + c_add with the columns n-2 .. 2n-2 of
// q N formed by one-level Karatsuba: q = q0 + B q1, N = n0 + B n1 (halves of
// M = ceil(n/2) limbs, B = 2^(28 M)), D0 = q0 n0, D1 = (q0 + q1)(n0 + n1),
// D2 = q1 n1.  The half sums are taken limb by limb, without carries (29-bit
// limbs), so D1 - D0 - D2 = q0 n1 + q1 n0 holds column by column and
// column w of q N is
//   D0[w] + D1[w - M] - D0[w - M] - D2[w - M] + D2[w - 2M],
// the schoolbook column exactly; only the upper columns of D1 and D0 and the
// columns of D2 that reach w >= n-2 are formed, each once.  The positive and
// negative parts are summed separately (a multiply-add cannot subtract) and
// combined in wrapping 64-bit arithmetic, exact since the column itself is
// below 2^64; each part stays below 2^64 for M <= 37 (at most M products of
// 29-bit limbs plus M of 28-bit ones).  The carry into column
// n and the result follow as in redc_blk's truncated path (two-column ceil).
template <int N, typename M, typename LoadM>
__device__ __forceinline__ void kara_high_half(const uint32_t (&t)[2 * N], const uint32_t (&q)[N], LoadM&& ldm,
                                               uint32_t (&c)[N]) {
  constexpr int H = (N + 1) / 2;
  static_assert(H <= 37, "the positive column part holds up to H products of 29-bit limbs");
  constexpr int BK = kColBlock;
  uint32_t q0[H], q1[H], sq[H];
  sfor<0, H>([&](auto I) {
    constexpr int i = decltype(I)::value;
    q0[i] = q[i];
    q1[i] = (H + i < N) ? q[(H + i < N) ? H + i : 0] : 0u;
    sq[i] = q0[i] + q1[i];
  });
  const auto ldn0 = [&](int j) { return ldm(j); };
  const auto ldn1 = [&](int j) { return H + j < N ? ldm(H + j) : 0u; };
  const auto ldsn = [&](int j) { return ldn0(j) + ldn1(j); };
  constexpr int W0 = N - 2;
  constexpr int NCOL = 2 * N - 1 - W0;
  // D2's columns XB .. 2H-2 enter twice: negated at w = x + H, then added at
  // w = x + 2H; they are formed once, at the first use, and kept
  constexpr int XB = W0 - H;
  uint64_t d2u[2 * H - 1 - XB];
  uint64_t carry = 0, a2 = 0;
  sfor<0, (NCOL + BK - 1) / BK>([&](auto B) {
    constexpr int w0 = W0 + decltype(B)::value * BK;
    constexpr int bk = (2 * N - 1 - w0) < BK ? (2 * N - 1 - w0) : BK;
    uint64_t pos[bk], neg[bk], d2[bk];
    sfor<0, bk>([&](auto D) {
      pos[decltype(D)::value] = t[w0 + decltype(D)::value];
      neg[decltype(D)::value] = 0;
      d2[decltype(D)::value] = 0;
    });
    colblock_ld<w0, bk, 0, H - 1, 0, H - 1, M>(q0, ldn0, pos);      // D0[w]
    colblock_ld<w0 - H, bk, 0, H - 1, 0, H - 1, M>(sq, ldsn, pos);  // D1[w - H]
    colblock_ld<w0 - H, bk, 0, H - 1, 0, H - 1, M>(q0, ldn0, neg);  // D0[w - H]
    colblock_ld<w0 - H, bk, 0, H - 1, 0, H - 1, M>(q1, ldn1, d2);   // D2[w - H], kept
    // D2[w - 2H]: from the kept columns, or formed here below XB
    constexpr bool low = w0 - 2 * H < XB;
    uint64_t d2lo[bk];
    sfor<0, bk>([&](auto D) { d2lo[decltype(D)::value] = 0; });
    if constexpr (low) colblock_ld<w0 - 2 * H, bk, 0, H - 1, 0, H - 1, M>(q1, ldn1, d2lo);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      constexpr int w = w0 + d;
      constexpr int xn = w - H;      // column of D2 negated here, >= XB
      constexpr int xp = w - 2 * H;  // column of D2 added here
      if constexpr (xn <= 2 * H - 2) d2u[xn - XB] = d2[d];
      uint64_t plus = 0;
      if constexpr (xp >= XB && xp <= 2 * H - 2) plus = d2u[xp - XB];
      else if constexpr (xp >= 0 && xp <= 2 * H - 2) plus = d2lo[d];
      const uint64_t col = pos[d] + plus - neg[d] - d2[d];
      if constexpr (w == N - 2) {
        a2 = col;
      } else if constexpr (w == N - 1) {
        const uint64_t a1 = col + (a2 >> kLimbBits);
        carry = (a1 >> kLimbBits) + ((((uint32_t)a1 | (uint32_t)a2) & kLimbMask) != 0u ? 1u : 0u);
      } else {
        const uint64_t v = col + carry;
        c[w - N] = (uint32_t)v & kLimbMask;
        carry = v >> kLimbBits;
      }
    });
    compiler_fence();
  });
  c[N - 1] = (uint32_t)(carry + t[2 * N - 1]);
}

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
  // volatile reads keep each LDS read next to its use (as in k_mont)
  const volatile uint32_t* sm = s_ctx + threadIdx.x;
  uint32_t q[N], r[N];
  low_half_q<N, RotMad>(t, [&](int i) { return sm[(N + i) * 64]; }, q);
  kara_high_half<N, RotMad>(t, q, [&](int j) { return sm[j * 64]; }, r);
  if (live) contract<N, RW>(r, out + (size_t)inst * RW);
}

}  // namespace mx
