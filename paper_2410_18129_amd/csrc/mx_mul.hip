// Batched multiprecision products: the schoolbook product of Section 2
// (Algorithm 1; squares as Algorithm 2) and Karatsuba's product of Section 3 at
// one and two levels, on operands of up to 4256 bits, one instance per lane.
//
// A value of n = K H limbs of 28 bits is K blocks of H limbs, kept in the
// lane's rows of a workspace (limb-major: row r of the 64 lanes of a tile is
// 256 contiguous bytes).  The schoolbook product is block product scanning
// (scan_mul: the block pairs of each diagonal summed into 64-bit column sums
// held in registers, every column written once).  Karatsuba splits a number of
// M blocks into halves of M/2 blocks, beta = 2^(28 H M / 2):
//   D0 = A0 B0,  D2 = A1 B1,  D1 = (A0 + A1)(B0 + B1),
//   A B = D0 + (D1 - D0 - D2) beta + D2 beta^2,
// three half-size products instead of four; at two levels each of the three is
// itself split (nine quarter-size products instead of sixteen).  The half sums
// are taken modulo beta with their carry bit c, and D1 = SA SB + (cA SB + cB SA)
// beta + cA cB beta^2, the carry terms added under all-ones / all-zero masks so
// the instruction stream does not depend on the data.  The recombination runs
// in signed redundant 32-bit limbs (a few multiples of 2^28 at most), then one
// normalisation.  Below the last level the products are scan_mul's.
//
// The sizes are public: every branch, loop bound and address depends only on
// them, never on the operands.
#include <hip/hip_runtime.h>

#include "mx_block.hpp"

namespace mx {

// dst rows 0 .. 2 M H - 1 = the product (square when sqr) of the M-block numbers at rows ra and rb,
// normalised 28-bit limbs; row 2 M H = 0 (the product of two M H-limb values has 2 M H limbs).
template <int H, int M>
__device__ __forceinline__ void scan_mul(bool sqr, const LaneBuf& ws, uint32_t ra, uint32_t rb, uint32_t dst) {
  if (sqr) rb = ra;
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  uint32_t a[H], b[H];
  ld_rows<H>(ws, ra, a);
  ld_rows<H>(ws, rb, b);
  uint32_t c = 0, i = 0;
#pragma nounroll
  for (;;) {
    const uint32_t j = c - i;
    uint32_t nc = c, ni = i + 1;
    if (ni > (c < M ? c : M - 1) || (sqr && ni > c - ni)) {
      nc = c + 1;
      ni = nc >= M ? nc - M + 1 : 0u;
    }
    const bool more = nc < 2 * M - 1;
    uint32_t na[H], nb[H];
    if (more) {
      ld_rows<H>(ws, ra + ni * H, na);
      ld_rows<H>(ws, rb + (nc - ni) * H, nb);
    }
    compiler_fence();
    if (sqr && i == j) {
      uint32_t a2[H];
      sfor<0, H>([&](auto P) { a2[decltype(P)::value] = a[decltype(P)::value] << 1; });
      blk_cols<H, 0, 2 * H - 2, true>(cols, a, a2);
      sfor<0, H>([&](auto P) {
        constexpr int p = decltype(P)::value;
        cols[2 * p] += (uint64_t)a[p] * a[p];
      });
    } else {
      if (sqr) sfor<0, H>([&](auto P) { b[decltype(P)::value] <<= 1; });
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
    }
    if (nc != c) {  // diagonal c done: block c of the product is final
      uint32_t o[H];
      blk_emit<H>(cols, carry, o);
      st_rows<H>(ws, dst + c * H, o);
    }
    compiler_fence();
    if (!more) break;
    c = nc;
    i = ni;
    sfor<0, H>([&](auto P) {
      a[decltype(P)::value] = na[decltype(P)::value];
      b[decltype(P)::value] = nb[decltype(P)::value];
    });
  }
  uint32_t o[H];
  blk_emit<H>(cols, carry, o);
  st_rows<H>(ws, dst + (2 * M - 1) * H, o);
  ws.st(dst + 2 * M * H, (uint32_t)carry);
}

// Scratch rows kara_mul<H, M, L> needs from `sc` on.
template <int H, int M, int L>
struct KaraScratch {
  static constexpr uint32_t h = (M / 2) * H;
  static constexpr uint32_t own = (2 * h + 2) + 2 * (h + 1);  // D, SA, SB
  static constexpr uint32_t rows = own + (L > 1 ? KaraScratch<H, M / 2, L - 1>::rows : 0u);
};
template <int H, int M>
struct KaraScratch<H, M, 0> {
  static constexpr uint32_t rows = 0;
};

// dst rows 0 .. 2 M H + 1 = the product (square when sqr) of the M-block numbers at rows ra and rb,
// normalised 28-bit limbs (the top rows 0 for normalised operands), by L levels of Karatsuba above
// scan_mul.  M must be a multiple of 2^L; scratch rows from sc (KaraScratch<H, M, L>::rows).
template <int H, int M, int L>
__device__ void kara_mul(bool sqr, const LaneBuf& ws, uint32_t ra, uint32_t rb, uint32_t dst, uint32_t sc) {
  if constexpr (L == 0) {
    scan_mul<H, M>(sqr, ws, ra, rb, dst);
    ws.st(dst + 2 * M * H + 1, 0u);
  } else {
    static_assert(M % 2 == 0, "Karatsuba needs an even block count at every level");
    constexpr uint32_t h = (M / 2) * H, len = 2 * M * H + 2;
    const uint32_t D = sc, SA = sc + 2 * h + 2, SB = SA + h + 1, sub = SB + h + 1;
    if (sqr) rb = ra;
    zero_rows(ws, dst, len);
    // D0 = A0 B0 at beta^0 and -beta^1; D2 = A1 B1 at beta^2 and -beta^1
#pragma nounroll
    for (uint32_t half = 0; half < 2; ++half) {
      kara_mul<H, M / 2, L - 1>(sqr, ws, ra + half * h, rb + half * h, D, sub);
      acc_rows<H>(ws, dst + 2 * half * h, D, 2 * h, 1);
      acc_rows<H>(ws, dst + h, D, 2 * h, -1);
    }
    // D1 = (A0 + A1)(B0 + B1) at beta^1
    const uint32_t ca = half_sum<H>(ws, ra, h, SA);
    const uint32_t cb = sqr ? ca : half_sum<H>(ws, rb, h, SB);
    const uint32_t sb = sqr ? SA : SB;
    kara_mul<H, M / 2, L - 1>(sqr, ws, SA, sb, D, sub);
    const uint32_t ma = 0u - ca, mb = 0u - cb;  // all-ones when the carry bit is set
    uint32_t i = 0;
#pragma nounroll
    for (; i < h; i += H) {
      uint32_t d[H], x[H], y[H];
      ld_rows<H>(ws, D + h + i, d);
      ld_rows<H>(ws, SA + i, x);
      ld_rows<H>(ws, sb + i, y);
      sfor<0, H>([&](auto I) {
        constexpr int k = decltype(I)::value;
        d[k] += (y[k] & ma) + (x[k] & mb);
      });
      st_rows<H>(ws, D + h + i, d);
    }
    ws.st(D + 2 * h, ws.ld(D + 2 * h) + (ca & cb));
    norm_rows<H>(ws, D, 2 * h + 2);
    acc_rows<H>(ws, dst + h, D, 2 * h + 2, 1);
    norm_rows_signed<H>(ws, dst, len);
  }
}

// Rows of one lane: A (n), B (n), the product (2n + 2), then the Karatsuba scratch.
template <int H, int K, int L>
struct MulLayout {
  static constexpr uint32_t n = H * K;
  static constexpr uint32_t A = 0, B = n, T = 2 * n, SC = 4 * n + 2;
  static constexpr uint32_t rows = SC + KaraScratch<H, K, L>::rows;
};

// Loads `words` 64-bit words at src, keeping the low `bits` bits, into rows row .. row + n - 1.
template <int N>
__device__ __forceinline__ void load_limbs(const LaneBuf& ws, uint32_t row, const uint64_t* __restrict__ src,
                                           uint32_t words, uint32_t bits) {
#pragma nounroll
  for (uint32_t i = 0; i < (uint32_t)N; ++i) {
    const uint32_t bit = kLimbBits * i, wd = bit >> 6, off = bit & 63;
    uint64_t v = wd < words ? src[wd] >> off : 0ull;
    if (off > 64 - kLimbBits && wd + 1 < words) v |= src[wd + 1] << (64 - off);
    uint32_t limb = (uint32_t)v & kLimbMask;
    const uint32_t keep = bit >= bits ? 0u : (bits - bit >= kLimbBits ? kLimbMask : (1u << (bits - bit)) - 1u);
    ws.st(row + i, limb & keep);
  }
}

// out[i] = a[i] * b[i] (a[i]^2 when b is null), `wout` words; operands of `win` words, low `bits` bits.
template <int H, int K, int L>
__global__ void __launch_bounds__(64) k_mul_raw(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                uint64_t* __restrict__ out, uint32_t bits, uint32_t win, uint32_t wout,
                                                uint32_t count, uint32_t* __restrict__ ws_base, uint32_t ws_bytes) {
  using Lay = MulLayout<H, K, L>;
  constexpr uint32_t tbytes = Lay::rows * 256u;  // this block's region: rows x 64 lanes
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  const bool sqr = b == nullptr;
  const LaneBuf ws{make_buf(ws_base + (size_t)blockIdx.x * (tbytes / 4u), tbytes), (threadIdx.x & 63u) * 4u, 256u};
  load_limbs<Lay::n>(ws, Lay::A, a + (size_t)inst * win, win, bits);
  if (!sqr) load_limbs<Lay::n>(ws, Lay::B, b + (size_t)inst * win, win, bits);
  kara_mul<H, K, L>(sqr, ws, Lay::A, Lay::B, Lay::T, Lay::SC);
  if (live) contract_rows<H, 2 * K>(ws, Lay::T, out + (size_t)inst * wout, wout);
}

// Instantiations: (H, K) = (37, 4) holds 4144 bits, (38, 4) 4256 bits; L = 0, 1, 2 Karatsuba levels.
template <int H, int K>
uint32_t mul_rows(int levels) {
  return levels == 0 ? MulLayout<H, K, 0>::rows : levels == 1 ? MulLayout<H, K, 1>::rows : MulLayout<H, K, 2>::rows;
}

template <int H, int K>
hipError_t mul_launch(int levels, const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t bits, uint32_t win,
                      uint32_t wout, uint32_t count, uint32_t* ws, uint32_t ws_bytes, hipStream_t st) {
  const uint32_t blocks = (count + 63) / 64;
  if ((uint64_t)mul_rows<H, K>(levels) * 256u * blocks > ws_bytes) return hipErrorInvalidValue;
  if (levels == 0)
    hipLaunchKernelGGL((k_mul_raw<H, K, 0>), dim3(blocks), dim3(64), 0, st, a, b, out, bits, win, wout, count, ws,
                       ws_bytes);
  else if (levels == 1)
    hipLaunchKernelGGL((k_mul_raw<H, K, 1>), dim3(blocks), dim3(64), 0, st, a, b, out, bits, win, wout, count, ws,
                       ws_bytes);
  else
    hipLaunchKernelGGL((k_mul_raw<H, K, 2>), dim3(blocks), dim3(64), 0, st, a, b, out, bits, win, wout, count, ws,
                       ws_bytes);
  return hipGetLastError();
}

// Per-instance workspace rows of a product of `bits`-bit operands with `levels` Karatsuba levels (0 if
// no instantiation holds `bits`).
uint32_t mul_raw_rows(uint32_t bits, int levels) {
  if (bits <= 37u * 4u * kLimbBits) return mul_rows<37, 4>(levels);
  if (bits <= 38u * 4u * kLimbBits) return mul_rows<38, 4>(levels);
  return 0;
}

hipError_t mul_raw(int levels, const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t bits, uint32_t win,
                   uint32_t wout, uint32_t count, uint32_t* ws, uint32_t ws_bytes, hipStream_t st) {
  if (bits <= 37u * 4u * kLimbBits)
    return mul_launch<37, 4>(levels, a, b, out, bits, win, wout, count, ws, ws_bytes, st);
  return mul_launch<38, 4>(levels, a, b, out, bits, win, wout, count, ws, ws_bytes, st);
}

}  // namespace mx
