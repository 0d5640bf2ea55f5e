// Block-level kernels for the large size classes (3072 and 4096 bits; 1024 and 2048 bits as well, for
// comparison and for small batches).
//
// A number of n = K H limbs is K blocks of H = 37 limbs.  Every phase of the
// Montgomery product is a loop over block pairs (i, j), each pair handled by
// one of four fully unrolled H-limb routines (full product, square, low half,
// high part), so the code size does not grow with K.  The pair sets repeat,
// one level up, the triangles of the paper:
//   product   (Section 2): all pairs (squaring: i <= j, cross terms doubled)
//   q         (Algorithm 6 step 1): pairs i + j <= K - 1, the low half only
//             on the anti-diagonal i + j = K - 1
//   q N       truncated (Theorem 2): pairs i + j >= K - 2 -- full products
//             above the anti-diagonal, the columns >= H - 2 of the
//             anti-diagonal products, and the single top partial product of
//             the pairs i + j = K - 2 (global column n - 2); plain: all pairs.
// The pairs of one diagonal add into 64-bit column sums held in registers,
// and each block of columns is normalised once, when it is final (block
// product scanning, below).  The truncated result uses the same two-column
// ceil correction as redc(): with S the exact sum of the known columns
// n-2 .. 2n-1, C = floor(S / 2^56) + [S mod 2^56 != 0].  Also here: the
// block Karatsuba product (Section 3; redundant 32-bit limbs in the
// workspace), the Karatsuba-truncated q N (Section 5) and CIOS with block
// words (Algorithm 4).
//
// One lane per instance, or two or four (the residue split below; with four
// the arrays live in LDS).  Every loop bound, branch and address depends
// only on public values (sizes, step counter, window size, lane index).
#pragma once
#include "mx_kernels.hpp"

namespace mx {

// Workspace word offsets (in limb rows) of one lane's arrays.
template <int H, int K>
struct BlkLayout {
  static constexpr int n = H * K;
  static constexpr uint32_t Y = 0;            // current value (n)
  static constexpr uint32_t B = n;            // multiplier (n)
  static constexpr uint32_t T = 2 * n;        // product T (2n + 1)
  static constexpr uint32_t Q = 4 * n + 1;    // q (n)
  static constexpr uint32_t S = 5 * n + 1;    // T + q N columns (2n + 1)
  static constexpr uint32_t G = 7 * n + 2;    // window table (2^w n), modexp only
  static constexpr uint32_t rows(uint32_t w) { return G + (w ? (1u << w) * (uint32_t)n : 0u); }
};

// This lane's view of a limb-major array: row r at byte r * ls + vo.  ldx / stx: row + x for a
// per-lane x (the row itself the same in every lane).
struct LaneBuf {
  __amdgpu_buffer_rsrc_t r;
  uint32_t vo;
  uint32_t ls;
  __device__ __forceinline__ uint32_t ld(uint32_t row) const { return bload(r, vo, row * ls); }
  __device__ __forceinline__ void st(uint32_t row, uint32_t v) const { bstore(r, v, vo, row * ls); }
  __device__ __forceinline__ uint32_t ldx(uint32_t row, uint32_t x) const { return bload(r, vo + x * ls, row * ls); }
  __device__ __forceinline__ void stx(uint32_t row, uint32_t x, uint32_t v) const { bstore(r, v, vo + x * ls, row * ls); }
  // a read with cache policy P (kPolicyNT for the scan of tables the caches cannot hold, stream_tables):
  // L2 lines filled that way go first, so that N and N', read from the context arrays, stay
  template <int P>
  __device__ __forceinline__ uint32_t ldx_pol(uint32_t row, uint32_t x) const {
    return bload_pol<P>(r, vo + x * ls, row * ls);
  }
};

// The same view of an array in LDS: p is this lane's word of row 0, ls words between rows.
struct LdsBuf {
  uint32_t* p;
  uint32_t ls;
  __device__ __forceinline__ uint32_t ld(uint32_t row) const { return p[row * ls]; }
  __device__ __forceinline__ void st(uint32_t row, uint32_t v) const { p[row * ls] = v; }
  __device__ __forceinline__ uint32_t ldx(uint32_t row, uint32_t x) const { return p[(row + x) * ls]; }
  __device__ __forceinline__ void stx(uint32_t row, uint32_t x, uint32_t v) const { p[(row + x) * ls] = v; }
};

template <int M, typename Buf>
__device__ __forceinline__ void ld_rows(const Buf& b, uint32_t row, uint32_t (&x)[M]) {
  sfor<0, M>([&](auto I) { x[decltype(I)::value] = b.ld(row + decltype(I)::value); });
}
template <int M, typename Buf>
__device__ __forceinline__ void st_rows(const Buf& b, uint32_t row, const uint32_t (&x)[M]) {
  sfor<0, M>([&](auto I) { b.st(row + decltype(I)::value, x[decltype(I)::value]); });
}
// rows[row + i] += mult * p[i] (redundant limbs, no carries)
template <int M>
__device__ __forceinline__ void add_rows(const LaneBuf& b, uint32_t row, const uint32_t (&p)[M], uint32_t mult) {
  uint32_t x[M];
  ld_rows<M>(b, row, x);
  sfor<0, M>([&](auto I) { x[decltype(I)::value] += p[decltype(I)::value] * mult; });
  st_rows<M>(b, row, x);
}
__device__ __forceinline__ void zero_rows(const LaneBuf& b, uint32_t row, uint32_t len) {
#pragma nounroll
  for (uint32_t i = 0; i < len; ++i) b.st(row + i, 0u);
}
// Normalises len redundant limbs in place (chunks of C limbs held in
// registers) and returns the carry out of the top limb.  The next chunk is
// read before the current one is processed, so the reads' latency overlaps.
template <int C>
__device__ __forceinline__ uint64_t norm_rows(const LaneBuf& b, uint32_t row, uint32_t len, uint64_t carry = 0) {
  uint32_t i = 0;
  uint32_t x[C];
  if (len >= C) ld_rows<C>(b, row, x);
#pragma nounroll
  for (; i + C <= len; i += C) {
    uint32_t nx[C];
    const bool more = i + 2 * C <= len;
    if (more) ld_rows<C>(b, row + i + C, nx);
    compiler_fence();
    sfor<0, C>([&](auto I) {
      constexpr int k = decltype(I)::value;
      const uint64_t v = (uint64_t)x[k] + carry;
      x[k] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;
    });
    st_rows<C>(b, row + i, x);
    if (more) sfor<0, C>([&](auto I) { x[decltype(I)::value] = nx[decltype(I)::value]; });
  }
#pragma nounroll
  for (; i < len; ++i) {
    const uint64_t v = (uint64_t)b.ld(row + i) + carry;
    b.st(row + i, (uint32_t)v & kLimbMask);
    carry = v >> kLimbBits;
  }
  return carry;
}

// rows[dst + i] = rows[src + i] for i < len, C limbs per register batch, the
// next batch read before the current one is written.
template <int C, typename DB, typename SB>
__device__ __forceinline__ void copy_rows(const DB& d, uint32_t dst, const SB& sb, uint32_t src, uint32_t len) {
  uint32_t i = 0;
  uint32_t x[C];
  if (len >= C) ld_rows<C>(sb, src, x);
#pragma nounroll
  for (; i + C <= len; i += C) {
    uint32_t nx[C];
    const bool more = i + 2 * C <= len;
    if (more) ld_rows<C>(sb, src + i + C, nx);
    compiler_fence();
    st_rows<C>(d, dst + i, x);
    if (more) sfor<0, C>([&](auto I) { x[decltype(I)::value] = nx[decltype(I)::value]; });
  }
#pragma nounroll
  for (; i < len; ++i) d.st(dst + i, sb.ld(src + i));
}

// Karatsuba's half-size products: dst rows (dlen, zeroed here) += the product of the M-block numbers at rows
// a and b (b ignored when sqr), as redundant limbs.  Within a row the next
// operand block is loaded while the current block product runs, and the
// accumulator rows are read before it, so memory latency overlaps the
// multiply-accumulates.
template <int H>
__device__ __forceinline__ void blk_product(bool sqr, const LaneBuf& ws, uint32_t ra, uint32_t rb, uint32_t M,
                                            uint32_t dst, uint32_t dlen) {
  zero_rows(ws, dst, dlen);
#pragma nounroll
  for (uint32_t i = 0; i < M; ++i) {
    uint32_t a[H], b[H];
    ld_rows<H>(ws, ra + i * H, a);
    const uint32_t src = sqr ? ra : rb;
    const uint32_t j0 = sqr ? i : 0u;
    ld_rows<H>(ws, src + j0 * H, b);
#pragma nounroll
    for (uint32_t j = j0; j < M; ++j) {
      uint32_t acc[2 * H], bn[H];
      ld_rows<2 * H>(ws, dst + (i + j) * H, acc);
      if (j + 1 < M) ld_rows<H>(ws, src + (j + 1) * H, bn);
      compiler_fence();
      uint32_t t[2 * H];
      uint32_t mult = 1u;
      if (sqr && j == i) {
        sqr_sb<H>(a, t);
      } else {
        mul_sb<H>(a, b, t);
        mult = sqr ? 2u : 1u;
      }
      sfor<0, 2 * H>([&](auto I) { acc[decltype(I)::value] += t[decltype(I)::value] * mult; });
      st_rows<2 * H>(ws, dst + (i + j) * H, acc);
      compiler_fence();
      if (j + 1 < M) sfor<0, H>([&](auto I) { b[decltype(I)::value] = bn[decltype(I)::value]; });
    }
  }
}

// rows[dst + i] = rows[dst + i] + sign * rows[src + i] as signed 32-bit limbs, C at a time.
template <int C>
__device__ __forceinline__ void acc_rows(const LaneBuf& ws, uint32_t dst, uint32_t src, uint32_t len, int sign) {
  uint32_t i = 0;
#pragma nounroll
  for (; i + C <= len; i += C) {
    uint32_t x[C], y[C];
    ld_rows<C>(ws, dst + i, x);
    ld_rows<C>(ws, src + i, y);
    sfor<0, C>([&](auto I) {
      constexpr int k = decltype(I)::value;
      x[k] = (uint32_t)((int32_t)x[k] + sign * (int32_t)y[k]);
    });
    st_rows<C>(ws, dst + i, x);
  }
#pragma nounroll
  for (; i < len; ++i) ws.st(dst + i, (uint32_t)((int32_t)ws.ld(dst + i) + sign * (int32_t)ws.ld(src + i)));
}

// Normalises signed redundant limbs (the total is non-negative) to 28-bit limbs.
template <int C>
__device__ __forceinline__ void norm_rows_signed(const LaneBuf& b, uint32_t row, uint32_t len) {
  int64_t carry = 0;
  uint32_t i = 0;
#pragma nounroll
  for (; i + C <= len; i += C) {
    uint32_t x[C];
    ld_rows<C>(b, row + i, x);
    sfor<0, C>([&](auto I) {
      constexpr int k = decltype(I)::value;
      const int64_t v = (int64_t)(int32_t)x[k] + carry;
      x[k] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;  // arithmetic shift: floor division
    });
    st_rows<C>(b, row + i, x);
  }
#pragma nounroll
  for (; i < len; ++i) {
    const int64_t v = (int64_t)(int32_t)b.ld(row + i) + carry;
    b.st(row + i, (uint32_t)v & kLimbMask);
    carry = v >> kLimbBits;
  }
}

// s = x_lo + x_hi over h = M H limbs (rows), returns the carry bit (0 / 1).
template <int H>
__device__ __forceinline__ uint32_t half_sum(const LaneBuf& ws, uint32_t x, uint32_t h, uint32_t s) {
  uint32_t carry = 0;
#pragma nounroll
  for (uint32_t i = 0; i < h; i += H) {
    uint32_t p[H], q[H];
    ld_rows<H>(ws, x + i, p);
    ld_rows<H>(ws, x + h + i, q);
    sfor<0, H>([&](auto I) {
      constexpr int k = decltype(I)::value;
      const uint32_t v = p[k] + q[k] + carry;
      p[k] = v & kLimbMask;
      carry = v >> kLimbBits;
    });
    st_rows<H>(ws, s + i, p);
  }
  return carry;
}

// One-level Karatsuba (Section 3) at block granularity, K even, M = K/2 blocks
// per half, beta = 2^(28 M H):  D0 = A0 B0, D2 = A1 B1,
// D1 = (A0 + A1)(B0 + B1) = SA SB + cA SB beta + cB SA beta + cA cB beta^2 with
// SA = (A0 + A1) mod beta, cA its carry (and likewise SB, cB), and
// T = D0 + (D1 - D0 - D2) beta + D2 beta^2 in signed redundant limbs.
// Three half-size products instead of four (squaring: three half squarings).
// Rows: T gets the product; D (the S region) and SA, SB (the Q region) are scratch.
template <int H, int K>
__device__ __forceinline__ void kara_product(bool sqr, const LaneBuf& ws) {
  using Lay = BlkLayout<H, K>;
  constexpr uint32_t n = Lay::n, M = K / 2, h = M * H;
  constexpr uint32_t D = Lay::S, SA = Lay::Q, SB = Lay::Q + h;
  static_assert(K % 2 == 0, "Karatsuba needs an even block count");
  zero_rows(ws, Lay::T, 2 * n + 1);
  const uint32_t rb = sqr ? Lay::Y : Lay::B;
  // D0 and D2
  for (uint32_t half = 0; half < 2; ++half) {
    blk_product<H>(sqr, ws, Lay::Y + half * h, rb + half * h, M, D, 2 * h + 2);
    norm_rows<H>(ws, D, 2 * h);
    acc_rows<H>(ws, Lay::T + 2 * half * h, D, 2 * h, 1);
    acc_rows<H>(ws, Lay::T + h, D, 2 * h, -1);
  }
  // D1
  const uint32_t ca = half_sum<H>(ws, Lay::Y, h, SA);
  const uint32_t cb = sqr ? ca : half_sum<H>(ws, Lay::B, h, SB);
  blk_product<H>(sqr, ws, SA, sqr ? SA : SB, M, D, 2 * h + 2);
  const uint32_t ma = 0u - ca, mb = 0u - cb;  // all-ones when the carry bit is set
  uint32_t i = 0;
#pragma nounroll
  for (; i < h; i += H) {
    uint32_t d[H], x[H], y[H];
    ld_rows<H>(ws, D + h + i, d);
    ld_rows<H>(ws, SA + i, x);
    ld_rows<H>(ws, (sqr ? SA : SB) + i, y);
    sfor<0, H>([&](auto I) {
      constexpr int k = decltype(I)::value;
      d[k] += (y[k] & ma) + (x[k] & mb);
    });
    st_rows<H>(ws, D + h + i, d);
  }
  ws.st(D + 2 * h, ws.ld(D + 2 * h) + (ca & cb));
  norm_rows<H>(ws, D, 2 * h + 2);
  acc_rows<H>(ws, Lay::T + h, D, 2 * h + 2, 1);
  norm_rows_signed<H>(ws, Lay::T, 2 * n + 1);
}

// ---- block product scanning ---------------------------------------------
//
// The block products of one Montgomery operation are summed diagonal by
// diagonal (block pairs (i, j) with i + j = c) into 64-bit column sums held
// in registers, cols[L] for the global columns c H + L; when a diagonal is
// done, its low H columns are final: they are normalised and written once,
// and the high columns move down to start the next diagonal.  A column sum
// is a partial sum of one column of the full product, at most
// n (2^28 - 1)^2 < 2^64 for n <= 255 limbs, so it never overflows.  Each pair
// loads its two operand blocks one pair ahead (the reads overlap the previous
// pair's products); nothing is read back from the workspace.

// cols[L] += sum over a[i] b[j] with i + j = L, CLO <= L <= CHI (and i > j when UPPER), products
// issued by the policy M.
template <int H, int CLO, int CHI, bool UPPER, typename M = PlainMad, int NC>
__device__ __forceinline__ void blk_cols(uint64_t (&cols)[NC], const uint32_t (&a)[H], const uint32_t (&b)[H]) {
  constexpr int BK = kColBlock;
  sfor<0, (CHI - CLO + BK) / BK>([&](auto Bc) {
    constexpr int k0 = CLO + decltype(Bc)::value * BK;
    constexpr int bk = (CHI + 1 - k0) < BK ? (CHI + 1 - k0) : BK;
    colblock<k0, bk, 0, H - 1, 0, H - 1, UPPER, M>(a, b, *reinterpret_cast<uint64_t(*)[bk]>(&cols[k0]));
  });
}

// As blk_cols (no UPPER) with the multiply-add policy M.
template <int H, int CLO, int CHI, typename M, int NC>
__device__ __forceinline__ void blk_cols_m(uint64_t (&cols)[NC], const uint32_t (&a)[H], const uint32_t (&b)[H]) {
  constexpr int BK = kColBlock;
  sfor<0, (CHI - CLO + BK) / BK>([&](auto Bc) {
    constexpr int k0 = CLO + decltype(Bc)::value * BK;
    constexpr int bk = (CHI + 1 - k0) < BK ? (CHI + 1 - k0) : BK;
    colblock<k0, bk, 0, H - 1, 0, H - 1, false, M>(a, b, *reinterpret_cast<uint64_t(*)[bk]>(&cols[k0]));
  });
}

// Normalises cols[0 .. H-1] with the running carry into o, then moves the
// high columns down by H (the next diagonal's window).
template <int H>
__device__ __forceinline__ void blk_emit(uint64_t (&cols)[2 * H], uint64_t& carry, uint32_t (&o)[H]) {
  sfor<0, H>([&](auto D) {
    constexpr int d = decltype(D)::value;
    const uint64_t v = cols[d] + carry;
    o[d] = (uint32_t)v & kLimbMask;
    carry = v >> kLimbBits;
  });
  sfor<0, H>([&](auto D) {
    constexpr int d = decltype(D)::value;
    cols[d] = cols[d + H];
    cols[d + H] = 0;
  });
}

// Makes every word of x count as produced here (an empty asm per word): the reads that fill x are
// waited for at this point, and nothing computed from x is moved above it.
template <int I, int N>
__device__ __forceinline__ void pin_word(uint32_t (&x)[N]) {
  asm volatile("" : "+v"(x[I]));
}
template <int N>
__device__ __forceinline__ void pin_words(uint32_t (&x)[N]) {
  sfor<0, N>([&](auto I) { pin_word<decltype(I)::value>(x); });
}

// The block pairs of one phase, in order: pair p is multiplied while pair p + 1 is read, into the other
// of two register sets, so that nothing is copied between iterations.  next(c, s, nc, ns) gives the
// pair after (c, s) and whether there is one; load(c, s, x, y) reads a pair's blocks; body(c, s, nc,
// more, x, y) multiplies them (and emits when nc != c).  The current pair's words are pinned before
// the next pair's reads are issued: the compiler's wait for them (which it may not count exactly
// across the loop) then cannot also wait for the reads just issued.
template <int NA, int NB, typename Next, typename Load, typename Body>
__device__ __forceinline__ void run_pairs(uint32_t c, uint32_t s, Next&& next, Load&& load, Body&& body) {
  uint32_t a0[NA], b0[NB], a1[NA], b1[NB];
  load(c, s, a0, b0);
#pragma nounroll
  for (;;) {
    uint32_t nc, ns;
    pin_words(a0);
    pin_words(b0);
    bool more = next(c, s, nc, ns);
    if (more) load(nc, ns, a1, b1);
    compiler_fence();
    body(c, s, nc, more, a0, b0);
    compiler_fence();
    if (!more) break;
    c = nc;
    s = ns;
    pin_words(a1);
    pin_words(b1);
    more = next(c, s, nc, ns);
    if (more) load(nc, ns, a0, b0);
    compiler_fence();
    body(c, s, nc, more, a1, b1);
    compiler_fence();
    if (!more) break;
    c = nc;
    s = ns;
  }
}

// T = Y * B or Y^2 (Section 2 at block level; squares: pairs i <= j, the
// cross pairs with a doubled operand, the diagonal blocks as Algorithm 2).
// T rows: 2n normalised limbs and a zero top row.
template <int H, int K>
__device__ __forceinline__ void scan_product(bool sqr, const LaneBuf& ws) {
  using Lay = BlkLayout<H, K>;
  const uint32_t rb = sqr ? Lay::Y : Lay::B;
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  uint32_t a[H], b[H];
  ld_rows<H>(ws, Lay::Y, a);
  ld_rows<H>(ws, rb, b);
  uint32_t c = 0, i = 0;
#pragma nounroll
  for (;;) {
    const uint32_t j = c - i;
    uint32_t nc = c, ni = i + 1;
    if (ni > (c < K ? c : K - 1) || (sqr && ni > c - ni)) {
      nc = c + 1;
      ni = nc >= K ? nc - K + 1 : 0u;
    }
    const bool more = nc < 2 * K - 1;
    uint32_t na[H], nb[H];
    if (more) {
      ld_rows<H>(ws, Lay::Y + ni * H, na);
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
    if (nc != c) {  // diagonal c done: block c of T is final
      uint32_t o[H];
      blk_emit<H>(cols, carry, o);
      st_rows<H>(ws, Lay::T + c * H, o);
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
  st_rows<H>(ws, Lay::T + (2 * K - 1) * H, o);
  ws.st(Lay::T + 2 * Lay::n, (uint32_t)carry);
}

// q = T_lo * N' mod R (Algorithm 6 step 1): diagonals 0 .. K-1, the last one
// low halves only; q blocks to the Q rows.
template <int H, int K>
__device__ __forceinline__ void scan_q(const LaneBuf& ws, const LaneBuf& cnp) {
  using Lay = BlkLayout<H, K>;
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  uint32_t a[H], b[H];
  ld_rows<H>(ws, Lay::T, a);
  ld_rows<H>(cnp, 0, b);
  uint32_t c = 0, i = 0;
#pragma nounroll
  for (;;) {
    uint32_t nc = c, ni = i + 1;
    if (ni > c) {
      nc = c + 1;
      ni = 0;
    }
    const bool more = nc < K;
    uint32_t na[H], nb[H];
    if (more) {
      ld_rows<H>(ws, Lay::T + ni * H, na);
      ld_rows<H>(cnp, (nc - ni) * H, nb);
    }
    compiler_fence();
    if (c + 1 < K)
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
    else
      blk_cols<H, 0, H - 1, false>(cols, a, b);
    if (nc != c) {
      uint32_t o[H];
      blk_emit<H>(cols, carry, o);  // the carry out of block K-1 is dropped: mod R
      st_rows<H>(ws, Lay::Q + c * H, o);
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
}

// Y = (T + q N) / R (Algorithm 6 step 4 / Algorithm 3).  TRUNC (Theorem 2):
// diagonals from K-1, whose block pairs contribute only their columns
// >= H-2 (global columns >= n-2), plus the top partial product of each pair
// on diagonal K-2 (global column n-2); the exact sums a2, a1 of columns n-2
// and n-1 give the carry into column n with the ceil correction for the
// skipped columns.  PLAIN: every diagonal; the low columns vanish and pass on
// their carry.
template <int H, int K, bool TRUNC>
__device__ __forceinline__ void scan_qn(const LaneBuf& ws, const LaneBuf& cn) {
  using Lay = BlkLayout<H, K>;
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  constexpr uint32_t c0 = TRUNC ? K - 1 : 0;
  if constexpr (TRUNC && K >= 2) {
#pragma nounroll
    for (uint32_t i = 0; i + 2 <= K; ++i)
      cols[H - 2] += (uint64_t)ws.ld(Lay::Q + i * H + H - 1) * cn.ld((K - 2 - i) * H + H - 1);
  }
  uint32_t a[H], b[H];
  {
    const uint32_t i0 = c0 >= K ? c0 - K + 1 : 0u;
    ld_rows<H>(ws, Lay::Q + i0 * H, a);
    ld_rows<H>(cn, (c0 - i0) * H, b);
  }
  uint32_t c = c0, i = c0 >= K ? c0 - K + 1 : 0u;
#pragma nounroll
  for (;;) {
    uint32_t nc = c, ni = i + 1;
    if (ni > (c < K ? c : K - 1)) {
      nc = c + 1;
      ni = nc >= K ? nc - K + 1 : 0u;
    }
    const bool more = nc < 2 * K - 1;
    uint32_t na[H], nb[H];
    if (more) {
      ld_rows<H>(ws, Lay::Q + ni * H, na);
      ld_rows<H>(cn, (nc - ni) * H, nb);
    }
    compiler_fence();
    if (TRUNC && c == K - 1)
      blk_cols<H, H - 2, 2 * H - 2, false>(cols, a, b);
    else
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
    if (nc != c) {  // diagonal c done: add block c of T, then emit or fold the carry
      uint32_t tb[H];
      ld_rows<H>(ws, Lay::T + c * H, tb);
      sfor<0, H>([&](auto D) { cols[decltype(D)::value] += tb[decltype(D)::value]; });
      uint32_t o[H];
      if (TRUNC && c == K - 1) {
        const uint64_t a2 = cols[H - 2];
        const uint64_t a1 = cols[H - 1] + (a2 >> kLimbBits);
        carry = (a1 >> kLimbBits) + ((((uint32_t)a1 | (uint32_t)a2) & kLimbMask) != 0u ? 1u : 0u);
        sfor<0, H>([&](auto D) {
          constexpr int d = decltype(D)::value;
          cols[d] = cols[d + H];
          cols[d + H] = 0;
        });
      } else if (c < K) {  // PLAIN, low columns: they vanish mod 2^28
        blk_emit<H>(cols, carry, o);
      } else {
        blk_emit<H>(cols, carry, o);
        st_rows<H>(ws, Lay::Y + (c - K) * H, o);
      }
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
  // the top block: columns (2K-1) H .. 2n-1 and T's top limbs
  uint32_t tb[H];
  ld_rows<H>(ws, Lay::T + (2 * K - 1) * H, tb);
  sfor<0, H>([&](auto D) { cols[decltype(D)::value] += tb[decltype(D)::value]; });
  uint32_t o[H];
  blk_emit<H>(cols, carry, o);  // C < 2N < R: no carry remains
  st_rows<H>(ws, Lay::Y + (K - 1) * H, o);
}

// ---- truncated q N by one-level Karatsuba (Section 5, Karatsuba paragraph) ----
//
// Halves of M = K / 2 blocks: q = q0 + beta q1 and N = n0 + beta n1, beta = 2^(28 h), h = M H.  With
// the half sums taken limb by limb, without carries (sq = q0 + q1 and sn = n0 + n1, 29-bit limbs),
// column w of q N is
//   D0[w] + (D1 - D0 - D2)[w - h] + D2[w - 2h],   D0 = q0 n0, D1 = sq sn, D2 = q1 n1,
// which is the schoolbook column exactly, so scan_qn's two-column carry recovery applies unchanged.
// Columns are summed modulo 2^64: a partial sum of D1 may pass 2^64 (up to h products of 29-bit
// limbs), but every complete column of T + q N is below 2^64, so its sum modulo 2^64 is exact.
// D2 enters twice, at w - h (subtracted) and w - 2h: its 2h - 1 column sums are formed once, into
// the S rows (two 32-bit rows per column), and read back for both.  The middle term's block pairs
// add sq sn and subtract q0 n0 (signed multiply-adds with the modulus words negated).  Products:
// D2 whole (M^2 block products), the middle term's pairs on the anti-diagonal (high parts) and
// above, twice, and single top products for column n - 2 -- the schoolbook's truncated count at one
// level (Theorem 2; no saving, the identity is what two levels would build on).

// raw column sums of D2 = q1 n1 into rows dst (column x in rows dst + 2x, dst + 2x + 1: low, high)
template <int H, int M>
__device__ __forceinline__ void scan_d2_raw(const LaneBuf& ws, uint32_t q1, const LaneBuf& cn, uint32_t n1,
                                            uint32_t dst) {
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
#pragma nounroll
  for (uint32_t c = 0; c + 1 < 2 * M; ++c) {
    const uint32_t ilo = c >= M ? c - M + 1 : 0u, ihi = c < M ? c : M - 1;
#pragma nounroll
    for (uint32_t i = ilo; i <= ihi; ++i) {
      uint32_t a[H], b[H];
      ld_rows<H>(ws, q1 + i * H, a);
      ld_rows<H>(cn, n1 + (c - i) * H, b);
      compiler_fence();
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
      compiler_fence();
    }
    sfor<0, H>([&](auto D) {
      constexpr int d = decltype(D)::value;
      ws.st(dst + 2 * (c * H + d), (uint32_t)cols[d]);
      ws.st(dst + 2 * (c * H + d) + 1, (uint32_t)(cols[d] >> 32));
      cols[d] = cols[d + H];
      cols[d + H] = 0;
    });
  }
  sfor<0, H - 1>([&](auto D) {  // the last diagonal's high part: columns (2M - 1) H .. 2 M H - 2
    constexpr int d = decltype(D)::value;
    ws.st(dst + 2 * ((2 * M - 1) * H + d), (uint32_t)cols[d]);
    ws.st(dst + 2 * ((2 * M - 1) * H + d) + 1, (uint32_t)(cols[d] >> 32));
  });
}

template <int H, int K>
__device__ __forceinline__ void scan_qn_kara(const LaneBuf& ws, const LaneBuf& cn) {
  using Lay = BlkLayout<H, K>;
  static_assert(K % 2 == 0, "the Karatsuba halves need an even block count");
  constexpr uint32_t M = K / 2, h = M * H, n = Lay::n, ND2 = 2 * h - 1;
  static_assert(2 * ND2 <= 2 * Lay::n + 1, "D2's column sums fit the S rows");
  constexpr uint32_t D2 = Lay::S;
  scan_d2_raw<H, M>(ws, Lay::Q + h, cn, h, D2);
  auto d2 = [&](uint32_t x) -> uint64_t {  // column x of D2, 0 for x outside 0 .. 2h - 2
    const bool in = x <= ND2 - 1;
    const uint32_t r = D2 + 2 * (in ? x : 0u);
    const uint64_t v = (uint64_t)ws.ld(r) | ((uint64_t)ws.ld(r + 1) << 32);
    return in ? v : 0ull;
  };
  uint64_t cols[2 * H];
  sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
  // column n - 2 (local H - 2 of output diagonal K - 1): the middle term's top products on its local
  // diagonal M - 2, and D0's top product (D0[w] reaches no higher column)
#pragma nounroll
  for (uint32_t i = 0; i + 2 <= M; ++i) {
    const uint32_t j = M - 2 - i, ri = i * H + H - 1, rj = j * H + H - 1;
    const uint32_t a0 = ws.ld(Lay::Q + ri), a1 = ws.ld(Lay::Q + h + ri), b0 = cn.ld(rj), b1 = cn.ld(h + rj);
    cols[H - 2] += (uint64_t)(a0 + a1) * (b0 + b1) - (uint64_t)a0 * b0;
  }
  cols[H - 2] += (uint64_t)ws.ld(Lay::Q + h - 1) * cn.ld(h - 1);
  uint64_t carry = 0;
#pragma nounroll
  for (uint32_t b = K - 1; b + 1 < 2 * K; ++b) {
    // the middle term's block pairs (i, j), i + j = b - M, of the M-block products
    const uint32_t d = b - M, ilo = d >= M ? d - M + 1 : 0u, ihi = d < M ? d : M - 1;
#pragma nounroll
    for (uint32_t i = ilo; i <= ihi && i < M; ++i) {
      const uint32_t j = d - i;
      uint32_t q0[H], sq[H], n0[H], sn[H];
      ld_rows<H>(ws, Lay::Q + i * H, q0);
      ld_rows<H>(ws, Lay::Q + h + i * H, sq);
      ld_rows<H>(cn, j * H, n0);
      ld_rows<H>(cn, h + j * H, sn);
      compiler_fence();
      sfor<0, H>([&](auto P) {
        constexpr int p = decltype(P)::value;
        sq[p] += q0[p];
        sn[p] += n0[p];
        n0[p] = 0u - n0[p];
      });
      if (b == K - 1) {  // the anti-diagonal: only its columns >= H - 2 reach column n - 2
        blk_cols_m<H, H - 2, 2 * H - 2, PlainMad>(cols, sq, sn);
        blk_cols_m<H, H - 2, 2 * H - 2, SignedMad>(cols, q0, n0);
      } else {
        blk_cols_m<H, 0, 2 * H - 2, PlainMad>(cols, sq, sn);
        blk_cols_m<H, 0, 2 * H - 2, SignedMad>(cols, q0, n0);
      }
      compiler_fence();
    }
    // output block b is complete once T, -D2[w - h] and D2[w - 2h] are added (w = b H + k)
    uint32_t tb[H];
    ld_rows<H>(ws, Lay::T + b * H, tb);
    sfor<0, H>([&](auto D) {
      constexpr uint32_t k = decltype(D)::value;
      const uint32_t w = b * H + k;
      cols[k] += (uint64_t)tb[k] - d2(w - h) + d2(w - 2 * h);
    });
    if (b == K - 1) {
      const uint64_t a2 = cols[H - 2];
      const uint64_t a1 = cols[H - 1] + (a2 >> kLimbBits);
      carry = (a1 >> kLimbBits) + ((((uint32_t)a1 | (uint32_t)a2) & kLimbMask) != 0u ? 1u : 0u);
      sfor<0, H>([&](auto D) {
        constexpr int dd = decltype(D)::value;
        cols[dd] = cols[dd + H];
        cols[dd + H] = 0;
      });
    } else {
      uint32_t o[H];
      blk_emit<H>(cols, carry, o);
      st_rows<H>(ws, Lay::Y + (b - K) * H, o);
    }
    compiler_fence();
  }
  uint32_t tb[H];
  ld_rows<H>(ws, Lay::T + (2 * K - 1) * H, tb);
  sfor<0, H>([&](auto D) {
    constexpr uint32_t k = decltype(D)::value;
    const uint32_t w = (2 * K - 1) * H + k;
    cols[k] += (uint64_t)tb[k] + d2(w - 2 * h);
  });
  uint32_t o[H];
  blk_emit<H>(cols, carry, o);
  st_rows<H>(ws, Lay::Y + (K - 1) * H, o);
  (void)n;
}

// ---- several lanes per instance ----------------------------------------------
//
// For batches too small to give every SIMD a wavefront, LP = 2 or 4
// consecutive lanes hold the same instance and cut its latency.  The columns
// of every diagonal are split among them by residue: lane r of a group forms
// the local columns k = LP u + r (k = p + q over the limbs p of the first
// block and q of the second) in its register cols[u].  It reads the first
// operand block as is and the second shifted down by r, Br[m] = B[m + r] for
// -LP < m < H (zero where m + r falls outside the block), so that its column
// LP u + r is the sum over p of A[p] Br[LP u - p] with compile-time indices.
// Every lane thus does a 1/LP share (plus a few products by zero) of every
// block pair, and no partial sums are added across lanes.  When a diagonal's
// low H columns are final, every lane reads each of them from the lane that
// holds it (a DPP broadcast inside the group) and normalises the same limbs,
// and the high columns move to the lanes that hold them in the next diagonal
// (a DPP rotation by H mod LP, as H is not a multiple of LP).  Square blocks
// are formed as whole block products here.

// for each lane i of a quad: the lane of its group of LP that it reads, S fixed (bcast) or own + S (rot)
template <int LP, int S, bool ROT>
constexpr int quad_ctrl() {
  int ctrl = 0;
  for (int i = 0; i < 4; ++i) {
    const int g = i & ~(LP - 1);
    const int src = g | ((ROT ? i + S : S) & (LP - 1));
    ctrl |= src << (2 * i);
  }
  return ctrl;
}
template <int LP, int S, bool ROT>
__device__ __forceinline__ uint64_t grp_read64(uint64_t v) {
  constexpr int ctrl = quad_ctrl<LP, S, ROT>();
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, ctrl, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), ctrl, 0xF, 0xF, false);
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 p = {lo, hi};
  return __builtin_bit_cast(uint64_t, p);
}

template <int H, int LP>
struct Res {
  static constexpr int NB = H + LP - 1;           // Br[m], m = -(LP - 1) .. H - 1, at index m + LP - 1
  static constexpr int NU = (2 * H - 2) / LP + 1;  // registers for the local columns 0 .. 2H - 2
};

// The lane's boundary entries of Br: the 2 (LP - 1) indices m < 0 and m > H - LP, whose row m + r can
// fall outside the block.  Their reads take the clamped row qx and are cleared by keep after the read
// has landed (a mask at read time would make the wavefront wait for it).
template <int H, int LP>
struct ResLane {
  static constexpr int NE = LP > 1 ? 2 * (LP - 1) : 1;
  uint32_t qx[NE];
  uint32_t keep[NE];
  // entry e: m = e - (LP - 1) for e < LP - 1, else m = H - LP + 1 + (e - (LP - 1))
  static constexpr int m_of(int e) { return e < LP - 1 ? e - (LP - 1) : H - LP + 1 + (e - (LP - 1)); }
  __device__ __forceinline__ explicit ResLane(uint32_t r) {
    sfor<0, (LP > 1 ? NE : 0)>([&](auto E) {
      constexpr int e = decltype(E)::value;
      const int q = m_of(e) + (int)r;
      const bool in = q >= 0 && q <= H - 1;
      qx[e] = (uint32_t)(in ? q : 0);
      keep[e] = in ? 0xFFFFFFFFu : 0u;
    });
  }
};

// Br of the block at rows row0 .. row0 + H - 1 of b, for this lane's r, before res_mask
template <int H, int LP, typename Buf>
__device__ __forceinline__ void ld_shift(const Buf& b, uint32_t row0, uint32_t r, const ResLane<H, LP>& rl,
                                         uint32_t (&x)[Res<H, LP>::NB]) {
  sfor<0, Res<H, LP>::NB>([&](auto I) {
    constexpr int m = (int)decltype(I)::value - (LP - 1);
    if constexpr (m >= 0 && m + LP - 1 <= H - 1) {
      x[decltype(I)::value] = b.ldx(row0 + (uint32_t)m, r);  // m + r < H for every r
    } else {
      constexpr int e = m < 0 ? m + (LP - 1) : (LP - 1) + (m - (H - LP + 1));
      x[decltype(I)::value] = b.ldx(row0, rl.qx[e]);
    }
  });
}
template <int H, int LP>
__device__ __forceinline__ void res_mask(const ResLane<H, LP>& rl, uint32_t (&x)[Res<H, LP>::NB]) {
  sfor<0, (LP > 1 ? ResLane<H, LP>::NE : 0)>([&](auto E) {
    constexpr int e = decltype(E)::value;
    constexpr int m = ResLane<H, LP>::m_of(e);
    x[m + LP - 1] &= rl.keep[e];
  });
}


// cols[u] += sum over p of a[p] Br[LP u - p] for the registers ULO .. UHI, eight at a time (the
// products of one a[p] into eight accumulators, carry-outs rotated: RotMad)
template <int H, int LP, int ULO, int UHI, int NU>
__device__ __forceinline__ void res_cols(uint64_t (&cols)[NU], const uint32_t (&a)[H],
                                         const uint32_t (&bs)[Res<H, LP>::NB]) {
  constexpr int BK = kColBlock;
  sfor<0, (UHI - ULO + BK) / BK>([&](auto Bc) {
    constexpr int u0 = ULO + decltype(Bc)::value * BK;
    constexpr int bk = (UHI + 1 - u0) < BK ? (UHI + 1 - u0) : BK;
    sfor<0, H>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr auto ok = [](int u) { return LP * u - p >= -(LP - 1) && LP * u - p <= H - 1; };
      constexpr auto ix = [](int u) { return LP * u - p + LP - 1; };
      if constexpr (bk == 8 && ok(u0) && ok(u0 + 7)) {  // ok is an interval in u: its ends decide
        RotMad::mad8(*reinterpret_cast<uint64_t(*)[8]>(&cols[u0]), bs[ix(u0)], bs[ix(u0 + 1)], bs[ix(u0 + 2)],
                     bs[ix(u0 + 3)], bs[ix(u0 + 4)], bs[ix(u0 + 5)], bs[ix(u0 + 6)], bs[ix(u0 + 7)], a[p]);
      } else {
        sfor<0, bk>([&](auto D) {
          constexpr int d = decltype(D)::value;
          if constexpr (ok(u0 + d)) RotMad::template mac<d>(cols[u0 + d], bs[ix(u0 + d)], a[p]);
        });
      }
    });
  });
}

// The diagonal's low H columns, normalised with the running carry into o (every lane of the group alike).
template <int H, int LP, int NU>
__device__ __forceinline__ void res_emit(const uint64_t (&cols)[NU], uint64_t& carry, uint32_t (&o)[H]) {
  sfor<0, H>([&](auto D) {
    constexpr int k = decltype(D)::value;
    const uint64_t v = grp_read64<LP, k % LP, false>(cols[k / LP]) + carry;
    o[k] = (uint32_t)v & kLimbMask;
    carry = v >> kLimbBits;
  });
}

// The high columns H .. 2H - 2 become the next diagonal's columns 0 .. H - 2: lane r' takes column
// LP u' + r' + H from lane s = (r' + H) mod LP, register u' + (r' + H) / LP; every other register is
// cleared.  The wrap ((r' + H) / LP = q0 + 1) happens exactly when s < H mod LP, so each source lane
// picks the register it hands over and one rotation moves it.
template <int H, int LP, int NU>
__device__ __forceinline__ void res_roll(uint64_t (&cols)[NU], uint32_t r) {
  constexpr int h0 = H % LP, q0 = H / LP;
  constexpr int NUP = (H - 2) / LP + 1;  // registers of the columns 0 .. H - 2
  static_assert(NUP + q0 <= NU, "rolled registers");
  const bool wraps = r < (uint32_t)h0;  // as a source lane
  uint64_t nx[NUP];
  sfor<0, NUP>([&](auto U) {
    constexpr int u = decltype(U)::value;
    uint64_t x;
    if constexpr (u + q0 + 1 < NU)
      x = wraps ? cols[u + q0 + 1] : cols[u + q0];
    else
      x = wraps ? 0ull : cols[u + q0];
    nx[u] = grp_read64<LP, h0, true>(x);
  });
  sfor<0, NU>([&](auto U) {
    constexpr int u = decltype(U)::value;
    if constexpr (u < NUP)
      cols[u] = nx[u];
    else
      cols[u] = 0;
  });
}

// Pairs (i, c - i) of diagonal c, i >= ilo: their count, for the product
// (squares: i <= c - i), the q triangle (c < K) and q N.
template <int K>
__device__ __forceinline__ uint32_t diag_ilo(uint32_t c) { return c >= K ? c - K + 1 : 0u; }
template <int K>
__device__ __forceinline__ uint32_t diag_pairs(uint32_t c, bool sqr) {
  const uint32_t ilo = diag_ilo<K>(c), ihi = c < K ? c : K - 1;
  const uint32_t top = sqr && c / 2 < ihi ? c / 2 : ihi;
  return top - ilo + 1;
}

// With several lanes per instance, q takes the multiplier's rows (B is not read after the product), so
// that Y, B and T (4n rows) are all a Montgomery operation needs of the lane's arrays.
template <int H, int K>
__device__ __forceinline__ constexpr uint32_t kQrows() { return BlkLayout<H, K>::B; }


template <int H, int K, int LP, typename WB>
__device__ __forceinline__ void scang_product(bool sqr, const WB& ws) {
  using Lay = BlkLayout<H, K>;
  constexpr int NB = Res<H, LP>::NB, NU = Res<H, LP>::NU;
  const uint32_t rb = sqr ? Lay::Y : Lay::B;
  const uint32_t r = threadIdx.x % LP;
  const ResLane<H, LP> rl(r);
  uint64_t cols[NU];
  sfor<0, NU>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  // pair s of diagonal c: (i, c - i), i = diag_ilo(c) + s
  auto next = [&](uint32_t c, uint32_t s, uint32_t& nc, uint32_t& ns) {
    nc = c;
    ns = s + 1;
    if (ns >= diag_pairs<K>(c, sqr)) {
      nc = c + 1;
      ns = 0;
    }
    return nc < 2 * K - 1;
  };
  auto load = [&](uint32_t c, uint32_t s, uint32_t (&x)[H], uint32_t (&y)[NB]) {
    const uint32_t i = diag_ilo<K>(c) + s, j = c - i;
    ld_rows<H>(ws, Lay::Y + i * H, x);
    ld_shift<H, LP>(ws, rb + j * H, r, rl, y);
  };
  auto body = [&](uint32_t c, uint32_t s, uint32_t nc, bool more, uint32_t (&a)[H], uint32_t (&b)[NB]) {
    const uint32_t i = diag_ilo<K>(c) + s;
    const uint32_t sh = sqr && 2 * i < c ? 1u : 0u;  // cross pairs of a square count twice
    res_mask<H, LP>(rl, b);
    sfor<0, H>([&](auto P) { a[decltype(P)::value] <<= sh; });
    res_cols<H, LP, 0, NU - 1>(cols, a, b);
    if (nc != c) {  // diagonal c done: block c of T is final
      uint32_t o[H];
      res_emit<H, LP>(cols, carry, o);
      st_rows<H>(ws, Lay::T + c * H, o);
      if (more) res_roll<H, LP>(cols, r);
    }
    (void)more;
  };
  run_pairs<H, NB>(0u, 0u, next, load, body);
  // the top block: the last diagonal's high columns
  res_roll<H, LP>(cols, r);
  uint32_t o[H];
  res_emit<H, LP>(cols, carry, o);  // no carry remains: T < 2^(28 2n); T's top row is not kept here
  st_rows<H>(ws, Lay::T + (2 * K - 1) * H, o);
}

template <int H, int K, int LP, typename WB>
__device__ __forceinline__ void scang_q(const WB& ws, const LaneBuf& cnp) {
  using Lay = BlkLayout<H, K>;
  constexpr int NB = Res<H, LP>::NB, NU = Res<H, LP>::NU;
  const uint32_t r = threadIdx.x % LP;
  const ResLane<H, LP> rl(r);
  uint64_t cols[NU];
  sfor<0, NU>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  // pair i of diagonal c < K: (i, c - i)
  auto next = [&](uint32_t c, uint32_t i, uint32_t& nc, uint32_t& ni) {
    nc = c;
    ni = i + 1;
    if (ni > c) {
      nc = c + 1;
      ni = 0;
    }
    return nc < K;
  };
  auto load = [&](uint32_t c, uint32_t i, uint32_t (&x)[H], uint32_t (&y)[NB]) {
    // N' block as the unshifted operand: its reads are the same row in every lane of a group (one line
    // per read), while the shifted reads, four rows per group, go to the lane's arrays
    ld_rows<H>(cnp, (c - i) * H, x);
    ld_shift<H, LP>(ws, Lay::T + i * H, r, rl, y);
  };
  auto body = [&](uint32_t c, uint32_t i, uint32_t nc, bool more, uint32_t (&a)[H], uint32_t (&b)[NB]) {
    res_mask<H, LP>(rl, b);
    if (c + 1 < K)
      res_cols<H, LP, 0, NU - 1>(cols, a, b);
    else  // the anti-diagonal: its low H columns (a few more in some lanes, never read)
      res_cols<H, LP, 0, (H - 1) / LP>(cols, a, b);
    if (nc != c) {
      uint32_t o[H];
      res_emit<H, LP>(cols, carry, o);  // the carry out of block K-1 is dropped: mod R
      st_rows<H>(ws, kQrows<H, K>() + c * H, o);
      if (more) res_roll<H, LP>(cols, r);
    }
    (void)i;
  };
  run_pairs<H, NB>(0u, 0u, next, load, body);
}

// cols += block c of T, each lane its own columns k = LP u + r < H
template <int H, int LP, int NU, typename WB>
__device__ __forceinline__ void res_add_rows(uint64_t (&cols)[NU], const WB& ws, uint32_t row0, uint32_t r) {
  sfor<0, (H - 1) / LP + 1>([&](auto U) {
    constexpr int u = decltype(U)::value;
    if constexpr (LP * u + LP - 1 <= H - 1) {
      cols[u] += ws.ldx(row0 + (uint32_t)(LP * u), r);
    } else {  // the lanes past the block read its row LP u (inside it) and add nothing
      const bool in = (uint32_t)(LP * u) + r <= (uint32_t)(H - 1);
      const uint32_t t = ws.ldx(row0 + (uint32_t)(LP * u), in ? r : 0u);
      cols[u] += in ? t : 0u;
    }
  });
}

template <int H, int K, bool TRUNC, int LP, typename WB>
__device__ __forceinline__ void scang_qn(const WB& ws, const LaneBuf& cn) {
  using Lay = BlkLayout<H, K>;
  constexpr int NB = Res<H, LP>::NB, NU = Res<H, LP>::NU;
  const uint32_t r = threadIdx.x % LP;
  const ResLane<H, LP> rl(r);
  uint64_t cols[NU];
  sfor<0, NU>([&](auto L) { cols[decltype(L)::value] = 0; });
  uint64_t carry = 0;
  constexpr uint32_t c0 = TRUNC ? K - 1 : 0;
  static_assert(H - 1 - LP >= 0, "blocks of at least LP + 1 limbs");
  if constexpr (TRUNC && K >= 2) {
    // the top products of diagonal K-2 (global column n-2 = local column H-2 of diagonal K-1), in the
    // lane that holds that column
    const uint32_t own = r == (uint32_t)((H - 2) % LP) ? 0xFFFFFFFFu : 0u;
#pragma nounroll
    for (uint32_t i = 0; i + 2 <= K; ++i)
      cols[(H - 2) / LP] += (uint64_t)(ws.ld(kQrows<H, K>() + i * H + H - 1) & own) * cn.ld((K - 2 - i) * H + H - 1);
  }
  // pair i of diagonal c: (i, c - i), diag_ilo(c) <= i <= min(c, K - 1)
  auto next = [&](uint32_t c, uint32_t i, uint32_t& nc, uint32_t& ni) {
    nc = c;
    ni = i + 1;
    if (ni > (c < K ? c : K - 1)) {
      nc = c + 1;
      ni = diag_ilo<K>(nc);
    }
    return nc < 2 * K - 1;
  };
  auto load = [&](uint32_t c, uint32_t i, uint32_t (&x)[H], uint32_t (&y)[NB]) {
    ld_rows<H>(cn, (c - i) * H, x);  // the modulus block unshifted, as N' in scang_q
    ld_shift<H, LP>(ws, kQrows<H, K>() + i * H, r, rl, y);
  };
  auto body = [&](uint32_t c, uint32_t i, uint32_t nc, bool more, uint32_t (&a)[H], uint32_t (&b)[NB]) {
    res_mask<H, LP>(rl, b);
    if (TRUNC && c == K - 1)  // columns >= H-2 (a few lower ones in some lanes, never read)
      res_cols<H, LP, (H - 1 - LP) / LP, NU - 1>(cols, a, b);
    else
      res_cols<H, LP, 0, NU - 1>(cols, a, b);
    if (nc != c) {  // diagonal c done: add block c of T, then emit or fold the carry
      res_add_rows<H, LP>(cols, ws, Lay::T + c * H, r);
      if (TRUNC && c == K - 1) {
        const uint64_t a2 = grp_read64<LP, (H - 2) % LP, false>(cols[(H - 2) / LP]);
        const uint64_t a1 = grp_read64<LP, (H - 1) % LP, false>(cols[(H - 1) / LP]) + (a2 >> kLimbBits);
        carry = (a1 >> kLimbBits) + ((((uint32_t)a1 | (uint32_t)a2) & kLimbMask) != 0u ? 1u : 0u);
      } else {
        uint32_t o[H];
        res_emit<H, LP>(cols, carry, o);
        if (c >= K) st_rows<H>(ws, Lay::Y + (c - K) * H, o);  // PLAIN, c < K: the low columns vanish mod 2^28
      }
      res_roll<H, LP>(cols, r);
    }
    (void)i;
    (void)more;
  };
  run_pairs<H, NB>(c0, diag_ilo<K>(c0), next, load, body);
  // the top block: columns (2K-1) H .. 2n-1 and T's top limbs
  res_add_rows<H, LP>(cols, ws, Lay::T + (2 * K - 1) * H, r);
  uint32_t o[H];
  res_emit<H, LP>(cols, carry, o);  // C < 2N < R: no carry remains
  st_rows<H>(ws, Lay::Y + (K - 1) * H, o);
}

// ---- word-interleaved Montgomery multiplication at block level (Section 4, Algorithm 4) ----
//
// CIOS with 37-limb blocks as its words, W = 2^(28 H): for each block a_i of the first operand,
// T = Z + a_i B, q_i = (T mod W) N'_0 mod W with N'_0 = N' mod W = -N^{-1} mod W, and
// Z = (T + q_i N) / W, the low block of T + q_i N vanishing.  The q_i are the blocks of the unique
// q = -A B N^{-1} mod R, so after K steps Z = (A B + q N) / R: the other reductions' integer.  Each
// step runs over the output blocks c with one 64-bit column window (blk_cols, 2H columns): block c
// collects Z_c and the low halves of a_i B_c and q_i N_c, the high halves of a_i B_{c-1} and
// q_i N_{c-1}; block 0's low half gives q_i first.  A column collects at most 4 H products below 2^56
// plus a limb and a carry, within 64 bits.  Products per operation: 2 K^2 block products and K
// half-block products for the q_i -- the same for a square (no symmetry to use).  Z (n + 1 limbs,
// below 3N < R, so its top limb stays 0) lives in the S rows; the last step writes the result over
// Y, whose blocks it has read by then.  One lane per instance.
template <int H, int K>
__device__ __forceinline__ void scan_cios(bool sqr, const LaneBuf& ws, const LaneBuf& cn, const LaneBuf& cnp) {
  using Lay = BlkLayout<H, K>;
  constexpr uint32_t n = Lay::n, Z = Lay::S;
  const uint32_t rb = sqr ? Lay::Y : Lay::B;
  zero_rows(ws, Z, n + 1);
#pragma nounroll
  for (uint32_t i = 0; i < K; ++i) {
    const uint32_t dst = i + 1 == K ? Lay::Y : Z;
    uint32_t a[H], q[H];
    ld_rows<H>(ws, Lay::Y + i * H, a);
    uint64_t cols[2 * H];
    sfor<0, 2 * H>([&](auto L) { cols[decltype(L)::value] = 0; });
    uint64_t carry = 0;
    {  // block 0: T's low block, q_i, and the vanishing low block of T + q_i N
      uint32_t b[H], z[H];
      ld_rows<H>(ws, rb, b);
      ld_rows<H>(ws, Z, z);
      compiler_fence();
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
      sfor<0, H>([&](auto D) { cols[decltype(D)::value] += z[decltype(D)::value]; });
      uint32_t t0[H];  // T mod W
      uint64_t c = 0;
      sfor<0, H>([&](auto D) {
        constexpr int d = decltype(D)::value;
        const uint64_t v = cols[d] + c;
        t0[d] = (uint32_t)v & kLimbMask;
        c = v >> kLimbBits;
      });
      uint32_t np0[H];
      ld_rows<H>(cnp, 0, np0);
      compiler_fence();
      uint64_t qc[H];
      sfor<0, H>([&](auto D) { qc[decltype(D)::value] = 0; });
      blk_cols<H, 0, H - 1, false>(qc, t0, np0);  // q_i = t0 N'_0 mod W: the low half only
      c = 0;
      sfor<0, H>([&](auto D) {
        constexpr int d = decltype(D)::value;
        const uint64_t v = qc[d] + c;
        q[d] = (uint32_t)v & kLimbMask;
        c = v >> kLimbBits;
      });
      uint32_t m[H];
      ld_rows<H>(cn, 0, m);
      compiler_fence();
      blk_cols<H, 0, 2 * H - 2, false>(cols, q, m);
      sfor<0, H>([&](auto D) {  // limbs 0 (T + q_i N = 0 mod W): only the carry goes on
        constexpr int d = decltype(D)::value;
        carry = (cols[d] + carry) >> kLimbBits;
        cols[d] = cols[d + H];
        cols[d + H] = 0;
      });
    }
    uint32_t b[H], m[H], z[H];
    if (K > 1) {
      ld_rows<H>(ws, rb + H, b);
      ld_rows<H>(cn, H, m);
      ld_rows<H>(ws, Z + H, z);
    }
#pragma nounroll
    for (uint32_t c = 1; c < K; ++c) {
      uint32_t nb[H], nm[H], nz[H];
      const bool more = c + 1 < K;
      if (more) {
        ld_rows<H>(ws, rb + (c + 1) * H, nb);
        ld_rows<H>(cn, (c + 1) * H, nm);
        ld_rows<H>(ws, Z + (c + 1) * H, nz);
      }
      compiler_fence();
      blk_cols<H, 0, 2 * H - 2, false>(cols, a, b);
      blk_cols<H, 0, 2 * H - 2, false>(cols, q, m);
      sfor<0, H>([&](auto D) { cols[decltype(D)::value] += z[decltype(D)::value]; });
      uint32_t o[H];
      blk_emit<H>(cols, carry, o);
      st_rows<H>(ws, dst + (c - 1) * H, o);  // Z_{c-1}, read at c - 1, or Y's block c - 1, read by now
      compiler_fence();
      if (more) {
        sfor<0, H>([&](auto P) {
          constexpr int p = decltype(P)::value;
          b[p] = nb[p];
          m[p] = nm[p];
          z[p] = nz[p];
        });
      }
    }
    // the top block: the high halves of a_i B_{K-1} and q_i N_{K-1}, Z's top limb
    cols[0] += ws.ld(Z + n);
    uint32_t o[H];
    blk_emit<H>(cols, carry, o);
    st_rows<H>(ws, dst + (K - 1) * H, o);
    if (i + 1 < K) ws.st(Z + n, (uint32_t)carry);  // 0 (Z < 3N < R); the result has n limbs
    compiler_fence();
  }
}

// One Montgomery product on the workspace: Y <- REDC(Y * B) or REDC(Y^2).
// n = K H; context blocks come from the limb-major context arrays.  LP lanes
// per instance (1, or 2 or 4 for the schoolbook product).
// KREDC: the truncated q N by one-level Karatsuba (scan_qn_kara; one lane per instance, K even).
// BCIOS: block-word CIOS (scan_cios; one lane per instance).
template <int H, int K, bool TRUNC, bool KARA = false, int LP = 1, bool KREDC = false, bool BCIOS = false,
          typename WB>
__device__ __forceinline__ void mont_blk(bool sqr, const WB& ws, const LaneBuf& cn, const LaneBuf& cnp) {
  static_assert(LP == 1 || ((LP == 2 || LP == 4) && !KARA), "several lanes per instance: schoolbook products only");
  static_assert(!KREDC || (LP == 1 && TRUNC && K % 2 == 0), "Karatsuba-truncated q N: one lane, even block count");
  static_assert(!BCIOS || (LP == 1 && !KARA && !KREDC), "block-word CIOS: one lane, its own products");
  if constexpr (BCIOS) {
    scan_cios<H, K>(sqr, ws, cn, cnp);
  } else if constexpr (LP > 1) {
    scang_product<H, K, LP>(sqr, ws);
    scang_q<H, K, LP>(ws, cnp);
    scang_qn<H, K, TRUNC, LP>(ws, cn);
  } else {
    // ---- product T = Y * B (or Y^2): Section 2 at block level, or Section 3 --
    if constexpr (KARA)
      kara_product<H, K>(sqr, ws);
    else
      scan_product<H, K>(sqr, ws);
    // ---- q = T_lo * N' mod R: pairs i + j <= K - 1 (Algorithm 6 step 1) ------
    scan_q<H, K>(ws, cnp);
    // ---- C = (T + q N) / R, truncated (Theorem 2) or whole (Algorithm 3) -----
    if constexpr (KREDC)
      scan_qn_kara<H, K>(ws, cn);
    else
      scan_qn<H, K, TRUNC>(ws, cn);
  }
}

// Loads the RW-word little-endian value at src into rows row .. row+n-1 (28-bit limbs).
template <int H, int K, typename Buf>
__device__ __forceinline__ void expand_rows(const Buf& ws, uint32_t row, const uint64_t* __restrict__ src,
                                            uint32_t words) {
  constexpr uint32_t n = H * K;
#pragma nounroll
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t bit = kLimbBits * i, wd = bit >> 6, off = bit & 63;
    uint64_t v = wd < words ? src[wd] >> off : 0ull;
    if (off > 64 - kLimbBits && wd + 1 < words) v |= src[wd + 1] << (64 - off);
    ws.st(row + i, (uint32_t)v & kLimbMask);
  }
}

template <int H, int K, typename Buf>
__device__ __forceinline__ void contract_rows(const Buf& ws, uint32_t row, uint64_t* __restrict__ dst,
                                              uint32_t words) {
  constexpr uint32_t n = H * K;
#pragma nounroll
  for (uint32_t j = 0; j < words; ++j) {
    uint64_t v = 0;
    const uint32_t i0 = (64 * j) / kLimbBits;
#pragma nounroll
    for (uint32_t i = i0; i < n && i <= i0 + 3; ++i) {
      const int lo = (int)(kLimbBits * i) - (int)(64 * j);
      const uint64_t x = ws.ld(row + i);
      if (lo >= 0 && lo < 64) v |= x << lo;
      if (lo < 0 && lo > -kLimbBits) v |= x >> (-lo);
    }
    dst[j] = v;
  }
}

// ---- batched modmul / modsqr, block version ---------------------------------
template <int H, int K, bool TRUNC, bool SQR, bool KARA = false, bool KREDC = false, bool BCIOS = false>
__global__ void __launch_bounds__(64) k_mont_blk(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                 const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                 uint64_t* __restrict__ out, uint32_t count, uint32_t* ws_base,
                                                 uint32_t ws_bytes, uint32_t coff) {
  using Lay = BlkLayout<H, K>;
  constexpr uint32_t n = Lay::n;
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  constexpr uint32_t tbytes = Lay::G * 256u;  // this block's region: G rows x 64 lanes
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  const uint32_t rw = (kLimbBits * n + 63) / 64;
  const LaneBuf ws{make_buf(ws_base + (size_t)blockIdx.x * (tbytes / 4u), tbytes), (threadIdx.x & 63u) * 4u, 256u};
  const uint32_t cbytes = n * ctx.stride * 4u;
  const LaneBuf cn{make_buf(ctx.n, cbytes), c * 4u, ctx.stride * 4u};
  const LaneBuf cnp{make_buf(ctx.np, cbytes), c * 4u, ctx.stride * 4u};
  expand_rows<H, K>(ws, Lay::Y, a + (size_t)inst * rw, rw);
  if (!SQR) expand_rows<H, K>(ws, Lay::B, b + (size_t)inst * rw, rw);
  mont_blk<H, K, TRUNC, KARA, 1, KREDC, BCIOS>(SQR, ws, cn, cnp);
  if (live) contract_rows<H, K>(ws, Lay::Y, out + (size_t)inst * rw, rw);
}

// ---- modexp, block version (same schedule as k_modexp) ----------------------
// A tile is 64 / LP instances (LP lanes per instance).  tws: this
// wavefront's own workspace region (BlkLayout rows(w) rows of 64 / LP
// instances, 256 / LP bytes per row), contiguous in memory.  hot: where the
// Montgomery operations keep Y, B (q) and T -- the same region (LDSHOT
// false) or 4n rows of LDS for the tile (LDSHOT, several lanes per instance,
// s_hot 4n (64 / LP) words); the window table stays in the region.
// With LDSHOT the lanes of a group split the table scan and the table's
// copies by residue (limb LP t + r in lane r): each lane reads back from the
// table only the limbs it wrote there, and the rows it writes to the LDS
// arrays are read by the whole group after a compiler fence (LDS operations of
// one wavefront are performed in order).  In the workspace path every lane
// copies and scans every limb, so no lane reads what another lane wrote.

// dst rows [dr, dr + n) = src rows [sr, sr + n), lane r of each group of LP copying the limbs LP t + r
template <int LP, int NL, typename DB, typename SB>
__device__ __forceinline__ void copy_rows_split(const DB& d, uint32_t dr, const SB& sb, uint32_t sr, uint32_t r) {
  if constexpr (LP == 1) {
    copy_rows<37>(d, dr, sb, sr, NL);
  } else {
    constexpr int NT = (NL + LP - 1) / LP;
    uint32_t x[NT];
    sfor<0, NT>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (LP * t + LP <= NL) {
        x[t] = sb.ldx(sr + (uint32_t)(LP * t), r);
      } else {  // the last t of some lanes is past the array
        const bool in = LP * t + (int)r < NL;
        x[t] = sb.ldx(sr + (uint32_t)(LP * t), in ? r : 0u);
      }
    });
    sfor<0, NT>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (LP * t + LP <= NL)
        d.stx(dr + (uint32_t)(LP * t), r, x[t]);
      else if (LP * t + (int)r < NL)
        d.stx(dr + (uint32_t)(LP * t), r, x[t]);
    });
  }
}

template <int H, int K, bool TRUNC, bool KARA = false, int LP = 1, bool KREDC = false, bool LDSHOT = false,
          bool BCIOS = false>
__device__ __forceinline__ void modexp_tile_blk(const CtxDev& ctx, const uint32_t* __restrict__ cidx,
                                                const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                                uint32_t ebits, uint32_t ewords, uint32_t w, uint32_t bw,
                                                uint64_t* __restrict__ out, uint32_t count, uint32_t* tws,
                                                uint32_t tws_bytes, uint32_t coff, uint32_t tile0,
                                                uint32_t* s_hot = nullptr) {
  static_assert(!LDSHOT || LP > 1, "LDS-resident arrays: several lanes per instance");
  using Lay = BlkLayout<H, K>;
  constexpr uint32_t n = Lay::n;
  const uint32_t slot = (threadIdx.x & 63u) / LP;  // this lane's instance within the tile
  const uint32_t gid = tile0 + slot;
  const bool live = gid < count;
  const bool writer = live && (threadIdx.x % LP) == 0u;  // the lanes of an instance hold equal results
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  const LaneBuf ws{make_buf(tws, tws_bytes), slot * 4u, 256u / LP};
  const uint32_t r = threadIdx.x % LP;
  constexpr int SP = LDSHOT ? LP : 1;  // lanes that split the table's scan and copies
  const uint32_t rs = LDSHOT ? r : 0u;
  using HotBuf = typename std::conditional<LDSHOT, LdsBuf, LaneBuf>::type;
  HotBuf hot;
  if constexpr (LDSHOT)
    hot = LdsBuf{s_hot + slot, 64u / LP};
  else
    hot = ws;
  const uint32_t cbytes = n * ctx.stride * 4u;
  const LaneBuf cn{make_buf(ctx.n, cbytes), c * 4u, ctx.stride * 4u};
  const LaneBuf cnp{make_buf(ctx.np, cbytes), c * 4u, ctx.stride * 4u};
  const LaneBuf cr1{make_buf(ctx.r1, cbytes), c * 4u, ctx.stride * 4u};
  const LaneBuf cr2{make_buf(ctx.r2, cbytes), c * 4u, ctx.stride * 4u};
  const uint64_t* e64 = ex + (size_t)inst * ewords;

  const uint32_t nent = 1u << w;
  const bool stream = stream_tables(count, nent, (uint32_t)n * 4u);
  const uint32_t nwin = ebits ? (ebits + w - 1) / w : 1u;
  // G[0] = R mod N
  copy_rows_split<SP, n>(ws, Lay::G, cr1, 0, rs);
  expand_rows<H, K>(hot, Lay::Y, base + (size_t)inst * bw, bw);

  const uint32_t n_tab = nent - 1;
  const uint32_t n_main = (nwin - 1) * (w + 1);
  const uint32_t total = n_tab + 1 + n_main + 1;
#pragma nounroll
  for (uint32_t s = 0; s < total; ++s) {
    int kind;
    int store_e = -1;
    uint32_t win = 0;
    if (s < n_tab) {
      kind = s == 0 ? kMulR2 : kMulG1;
      store_e = (int)s + 1;
    } else if (s == n_tab) {
      kind = kLoadSel;
      win = nwin - 1;
    } else if (s < n_tab + 1 + n_main) {
      const uint32_t step = s - n_tab - 1;
      win = nwin - 2 - step / (w + 1);
      kind = (step % (w + 1)) < w ? kSqr : kMulSel;
    } else {
      kind = kMulOne;
    }
    if (kind == kMulSel || kind == kLoadSel) {
      const uint32_t p = win * w;
      const uint32_t width = ebits > p ? (ebits - p < w ? ebits - p : w) : 0u;
      const uint32_t lo = p >> 6, sh = p & 63;
      uint64_t v = (width > 0 && lo < ewords) ? e64[lo] >> sh : 0ull;
      if (width > 0 && sh + width > 64 && lo + 1 < ewords) v |= e64[lo + 1] << (64 - sh);
      const uint32_t bits = (uint32_t)v & ((1u << width) - 1u);
      const uint32_t dst = kind == kLoadSel ? Lay::Y : Lay::B;
      // full masked scan of the table, H limbs at a time, SE entries per
      // iteration (SE H reads in flight; the registers of the Montgomery
      // operation are free here).  With fewer than SE entries (w < 3) the
      // missing ones re-read entry 0 under a zero mask.  Lane rs of a group
      // of SP scans the limbs SP t + rs (t in chunks of H).
      constexpr uint32_t SE = 8;
      constexpr uint32_t NT = (n + SP - 1) / SP;        // limbs per lane
      constexpr uint32_t CH = NT < H ? NT : H;          // limbs per lane and chunk
      constexpr bool kFull = n % SP == 0 && NT % CH == 0;  // every (chunk, i, lane) names a limb
#pragma nounroll
      for (uint32_t t0 = 0; t0 < NT; t0 += CH) {
        uint32_t acc[CH];
        sfor<0, CH>([&](auto I) { acc[decltype(I)::value] = 0; });
        // the reads' cache policy (a uniform choice from the launch's size) selects one of two loop copies
        auto scan = [&](auto pol) {
          constexpr int P = decltype(pol)::value;
#pragma nounroll
          for (uint32_t e = 0; e < nent; e += SE) {
            uint32_t g[SE][CH];
            uint32_t mask[SE];
            sfor<0, SE>([&](auto U) {
              constexpr uint32_t u = decltype(U)::value;
              const bool in = e + u < nent;
              mask[u] = in && e + u == bits ? 0xFFFFFFFFu : 0u;
              const uint32_t er = Lay::G + (in ? e + u : 0u) * n;
              sfor<0, CH>([&](auto I) {
                constexpr uint32_t i = decltype(I)::value;
                const uint32_t l = SP * (t0 + i) + rs;  // this lane's limb
                if constexpr (kFull) {
                  g[u][i] = ws.template ldx_pol<P>(er, l);
                } else {  // past n: row n - 1 under a zero mask
                  const bool li = l < n;
                  g[u][i] = ws.template ldx_pol<P>(er, li ? l : n - 1u) & (li ? 0xFFFFFFFFu : 0u);
                }
              });
            });
            sfor<0, CH>([&](auto I) {
              constexpr int i = decltype(I)::value;
              uint32_t v = acc[i];
              sfor<0, SE>([&](auto U) { v |= g[decltype(U)::value][i] & mask[decltype(U)::value]; });
              acc[i] = v;
            });
          }
        };
        if (stream)
          scan(std::integral_constant<int, kPolicyNT>{});
        else
          scan(std::integral_constant<int, 0>{});
        sfor<0, CH>([&](auto I) {
          constexpr uint32_t i = decltype(I)::value;
          const uint32_t l = SP * (t0 + i) + rs;
          if constexpr (kFull)
            hot.stx(dst, l, acc[i]);
          else if (l < n)
            hot.stx(dst, l, acc[i]);
        });
      }
      compiler_fence();
      if (kind == kLoadSel) continue;
    } else if (kind == kMulR2) {
      copy_rows_split<SP, n>(hot, Lay::B, cr2, 0, rs);
    } else if (kind == kMulG1) {
      copy_rows_split<SP, n>(hot, Lay::B, ws, Lay::G + n, rs);
    } else if (kind == kMulOne) {
#pragma nounroll
      for (uint32_t i = 0; i < n; ++i) hot.st(Lay::B + i, i == 0 ? 1u : 0u);
    }
    compiler_fence();
    mont_blk<H, K, TRUNC, KARA, LP, KREDC, BCIOS>(kind == kSqr, hot, cn, cnp);
    compiler_fence();
    if (store_e >= 0) copy_rows_split<SP, n>(ws, Lay::G + (uint32_t)store_e * n, hot, Lay::Y, rs);
  }
  // canonical result: subtract N once if Y >= N, in constant time: B = Y - N, then every limb of B
  // becomes Y's or stays B's under an all-ones / all-zero mask, so the rows read and written, and
  // the row the result is taken from, do not depend on the value
  int64_t br = 0;
#pragma nounroll
  for (uint32_t i = 0; i < n; ++i) {
    const int64_t v = (int64_t)hot.ld(Lay::Y + i) - (int64_t)cn.ld(i) + br;
    hot.st(Lay::B + i, (uint32_t)v & kLimbMask);
    br = v >> kLimbBits;
  }
  const uint32_t keep_y = (uint32_t)br;  // br is -1 (Y < N: keep Y) or 0 (keep Y - N)
#pragma nounroll
  for (uint32_t i = 0; i < n; ++i)
    hot.st(Lay::B + i, (hot.ld(Lay::Y + i) & keep_y) | (hot.ld(Lay::B + i) & ~keep_y));
  if (writer) contract_rows<H, K>(hot, Lay::B, out + (size_t)inst * bw, bw);
}

template <int H, int K, bool TRUNC, bool KARA = false, int LP = 1, bool KREDC = false, bool BCIOS = false>
__global__ void __launch_bounds__(64) k_modexp_blk(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                   const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                                   uint32_t ebits, uint32_t ewords, uint32_t w, uint32_t bw,
                                                   uint64_t* __restrict__ out, uint32_t count, uint32_t* ws_base,
                                                   uint32_t ws_bytes, uint32_t coff) {
  const uint32_t tile0 = blockIdx.x * (64u / LP);
  const uint32_t tbytes = BlkLayout<H, K>::rows(w) * (256u / LP);  // this block's region
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  stagger<H * K>(blockIdx.x, w);
  constexpr bool kLds = LP == 4;  // 4n rows of 16 words: 37.9 KB at 4096 bits, four wavefronts per CU
  __shared__ uint32_t s_hot[kLds ? 4 * H * K * (64 / LP) : 1];
  modexp_tile_blk<H, K, TRUNC, KARA, LP, KREDC, kLds, BCIOS>(ctx, cidx, base, ex, ebits, ewords, w, bw, out, count,
                                                      ws_base + (size_t)blockIdx.x * (tbytes / 4u), tbytes, coff,
                                                      tile0, s_hot);
}

}  // namespace mx
