// Device arithmetic for batched Montgomery multiplication on gfx950.
//
// One instance per lane: the word-slicing of Section 2 (Table 1), where every
// SIMD lane carries one independent instance, mapped onto 64-lane wavefronts.
// Numbers are little-endian arrays of 28-bit limbs held in 32-bit registers.
// A 28x28-bit partial product is one v_mad_u64_u32 accumulated into a 64-bit
// column sum; a column of up to 255 such products cannot overflow, so the
// products run without carry instructions and carries are resolved once per
// column (the role of the final carry pass of Algorithm 1).
//
// R = 2^(28 n) with n = ceil((bits + 2) / 28), so R >= 4N and results stay
// in [0, 2N) without a final subtraction (Section 4, Algorithms 3 and 5).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace mx {

constexpr int kLimbBits = 28;
constexpr uint32_t kLimbMask = (1u << kLimbBits) - 1u;

// Limb count of a size class: smallest n with 28 n >= bits + 2 (R >= 4N).
constexpr int limbs_for(int bits) { return (bits + 2 + kLimbBits - 1) / kLimbBits; }
// 64-bit words holding a value of `bits` bits.
constexpr int words_for(int bits) { return (bits + 63) / 64; }

// ---- compile-time loops ---------------------------------------------------
template <int B, typename F, int... I>
__device__ __forceinline__ void sfor_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, B + I>{}), ...);
}
// Calls f(integral_constant<int, i>) for i = B .. E-1 (nothing when E <= B).
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (E > B) sfor_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

// ---- partial products ----------------------------------------------------
//
// One 28x28-bit partial product into a 64-bit column sum is one
// v_mad_u64_u32 (acc + a * b).  The column routines below take the way the
// products are issued as a policy M: M::mad8 is eight products sharing one
// multiplier (eight independent accumulators), M::mac<S> a single product.
//
// PlainMad leaves the instructions to the compiler.  v_mad_u64_u32 also
// writes a carry-out SGPR pair that nothing reads, and the compiler gives
// every such instruction the same pair; issued back to back by one
// wavefront, instructions writing the same pair wait on each other (about 9
// SIMD cycles apart on gfx950 with one wavefront per SIMD, against about 5.8
// when the carry-outs rotate over 8 pairs).  RotMad issues the products from
// inline assembly with their carry-outs in s[40:41] .. s[54:55] in turn
// (declared clobbered, never read).  Which is faster depends on the kernel
// (it removes the compiler's freedom to schedule the products), so each
// kernel picks the one measured faster.
struct PlainMad {
  template <int S>
  __device__ __forceinline__ static void mac(uint64_t& acc, uint32_t a, uint32_t b) {
    acc += (uint64_t)a * (uint64_t)b;
  }
  __device__ __forceinline__ static void mad8(uint64_t (&acc)[8], uint32_t x0, uint32_t x1, uint32_t x2,
                                              uint32_t x3, uint32_t x4, uint32_t x5, uint32_t x6, uint32_t x7,
                                              uint32_t v) {
    acc[0] += (uint64_t)x0 * v;
    acc[1] += (uint64_t)x1 * v;
    acc[2] += (uint64_t)x2 * v;
    acc[3] += (uint64_t)x3 * v;
    acc[4] += (uint64_t)x4 * v;
    acc[5] += (uint64_t)x5 * v;
    acc[6] += (uint64_t)x6 * v;
    acc[7] += (uint64_t)x7 * v;
  }
};

// As PlainMad with both words read as signed 32-bit values (v_mad_i64_i32): with one of them negated
// (0 - x), each step subtracts the product in wrapping 64-bit arithmetic.
struct SignedMad {
  template <int S>
  __device__ __forceinline__ static void mac(uint64_t& acc, uint32_t a, uint32_t b) {
    acc += (uint64_t)((int64_t)(int32_t)a * (int64_t)(int32_t)b);
  }
  __device__ __forceinline__ static void mad8(uint64_t (&acc)[8], uint32_t x0, uint32_t x1, uint32_t x2,
                                              uint32_t x3, uint32_t x4, uint32_t x5, uint32_t x6, uint32_t x7,
                                              uint32_t v) {
    const int64_t sv = (int32_t)v;
    acc[0] += (uint64_t)((int32_t)x0 * sv);
    acc[1] += (uint64_t)((int32_t)x1 * sv);
    acc[2] += (uint64_t)((int32_t)x2 * sv);
    acc[3] += (uint64_t)((int32_t)x3 * sv);
    acc[4] += (uint64_t)((int32_t)x4 * sv);
    acc[5] += (uint64_t)((int32_t)x5 * sv);
    acc[6] += (uint64_t)((int32_t)x6 * sv);
    acc[7] += (uint64_t)((int32_t)x7 * sv);
  }
};

#define MX_MAD_SDST(P, LO, HI)                                                                     \
  if constexpr ((S & 7) == P)                                                                      \
    asm("v_mad_u64_u32 %0, s[" #LO ":" #HI "], %1, %2, %0" : "+v"(acc) : "v"(a), "v"(b)           \
        : "s" #LO, "s" #HI);
struct RotMad {
  template <int S>
  __device__ __forceinline__ static void mac(uint64_t& acc, uint32_t a, uint32_t b) {
    MX_MAD_SDST(0, 40, 41)
    MX_MAD_SDST(1, 42, 43)
    MX_MAD_SDST(2, 44, 45)
    MX_MAD_SDST(3, 46, 47)
    MX_MAD_SDST(4, 48, 49)
    MX_MAD_SDST(5, 50, 51)
    MX_MAD_SDST(6, 52, 53)
    MX_MAD_SDST(7, 54, 55)
  }
  __device__ __forceinline__ static void mad8(uint64_t (&acc)[8], uint32_t x0, uint32_t x1, uint32_t x2,
                                              uint32_t x3, uint32_t x4, uint32_t x5, uint32_t x6, uint32_t x7,
                                              uint32_t v) {
    asm("v_mad_u64_u32 %0, s[40:41], %8, %16, %0\n\t"
        "v_mad_u64_u32 %1, s[42:43], %9, %16, %1\n\t"
        "v_mad_u64_u32 %2, s[44:45], %10, %16, %2\n\t"
        "v_mad_u64_u32 %3, s[46:47], %11, %16, %3\n\t"
        "v_mad_u64_u32 %4, s[48:49], %12, %16, %4\n\t"
        "v_mad_u64_u32 %5, s[50:51], %13, %16, %5\n\t"
        "v_mad_u64_u32 %6, s[52:53], %14, %16, %6\n\t"
        "v_mad_u64_u32 %7, s[54:55], %15, %16, %7"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]),
          "+v"(acc[7])
        : "v"(x0), "v"(x1), "v"(x2), "v"(x3), "v"(x4), "v"(x5), "v"(x6), "v"(x7), "v"(v)
        : "s40", "s41", "s42", "s43", "s44", "s45", "s46", "s47", "s48", "s49", "s50", "s51", "s52", "s53", "s54",
          "s55");
  }
};
#undef MX_MAD_SDST

// ---- column blocks ---------------------------------------------------------
//
// Every product below is formed BK = 8 columns at a time: for the columns
// K0 .. K0+BK-1 and each limb index j of the second operand,
// acc[d] += a[K0 + d - j] * b[j], so one word of the second operand feeds up
// to eight products (one mad8 where all eight lie inside the bounds).  b is
// in registers or, for the modulus and N', in LDS.  The accumulators of one
// block are then normalised into limbs; a compiler barrier between blocks
// keeps the loaded words short-lived instead of letting them pile up in
// registers.
constexpr int kColBlock = 8;

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// The products of one word v = (second operand)[j] with the first operand for
// the columns K0 .. K0+BK-1: acc[d] += a[K0 + d - j] * v wherever
// ILO <= K0 + d - j <= IHI and, when UPPER, K0 + d - j > j (each off-diagonal
// pair of a square once).
template <int K0, int BK, int ILO, int IHI, bool UPPER, int J, typename M, int NA>
__device__ __forceinline__ void colstep(const uint32_t (&a)[NA], uint32_t v, uint64_t (&acc)[BK]) {
  constexpr auto ok = [](int d) {
    const int i = K0 + d - J;
    return i >= ILO && i <= IHI && (!UPPER || i > J);
  };
  constexpr bool full = BK == 8 && ok(0) && ok(1) && ok(2) && ok(3) && ok(4) && ok(5) && ok(6) && ok(7);
  if constexpr (full) {  // BK == 8: acc is the eight accumulators
    static_assert(K0 - J >= 0 && K0 + 7 - J < NA, "column index");
    M::mad8(*reinterpret_cast<uint64_t(*)[8]>(&acc[0]), a[K0 - J], a[K0 + 1 - J], a[K0 + 2 - J], a[K0 + 3 - J],
         a[K0 + 4 - J], a[K0 + 5 - J], a[K0 + 6 - J], a[K0 + 7 - J], v);
  } else {
    sfor<0, BK>([&](auto D) {
      constexpr int d = decltype(D)::value;
      if constexpr (ok(d)) M::template mac<d>(acc[d], a[K0 + d - J], v);
    });
  }
}

// acc[d] += sum over i of a[i] * b[K0 + d - i] for the columns K0 .. K0+BK-1,
// restricted to ILO <= i <= IHI (and i > K0 + d - i when UPPER); b in registers.
template <int K0, int BK, int ILO, int IHI, int JLO, int JHI, bool UPPER, typename M, int NA, int NB>
__device__ __forceinline__ void colblock(const uint32_t (&a)[NA], const uint32_t (&b)[NB], uint64_t (&acc)[BK]) {
  constexpr int jmin = (K0 - IHI) > JLO ? (K0 - IHI) : JLO;
  constexpr int jmax = (K0 + BK - 1 - ILO) < JHI ? (K0 + BK - 1 - ILO) : JHI;
  sfor<jmin, jmax + 1>([&](auto J) {
    constexpr int j = decltype(J)::value;
    colstep<K0, BK, ILO, IHI, UPPER, j, M>(a, b[j], acc);
  });
}

// As colblock, with the words of the second operand read from memory (LDS)
// by ld(j).  They are read in groups of kPrefetch words, one group ahead of
// the products that use them, so that the latency of a group's reads is
// covered by the previous group's products (one wavefront per SIMD has no
// other wavefront to switch to).
constexpr int kPrefetch = 16;

template <int K0, int BK, int ILO, int IHI, int JLO, int JHI, typename M, int NA, typename Ld>
__device__ __forceinline__ void colblock_ld(const uint32_t (&a)[NA], Ld&& ld, uint64_t (&acc)[BK]) {
  constexpr int jmin = (K0 - IHI) > JLO ? (K0 - IHI) : JLO;
  constexpr int jmax = (K0 + BK - 1 - ILO) < JHI ? (K0 + BK - 1 - ILO) : JHI;
  constexpr int G = kPrefetch;
  constexpr int NG = jmax >= jmin ? (jmax - jmin + G) / G : 0;
  uint32_t buf[2][G];
  sfor<0, (NG > 0 ? G : 0)>([&](auto U) {
    constexpr int j = jmin + decltype(U)::value;
    if constexpr (j <= jmax) buf[0][decltype(U)::value] = ld(j);
  });
  sfor<0, NG>([&](auto GG) {
    constexpr int g = decltype(GG)::value;
    if constexpr (g + 1 < NG) {
      sfor<0, G>([&](auto U) {
        constexpr int j = jmin + (g + 1) * G + decltype(U)::value;
        if constexpr (j <= jmax) buf[(g + 1) & 1][decltype(U)::value] = ld(j);
      });
    }
    compiler_fence();  // the next group's reads are issued before this group's products
    sfor<0, G>([&](auto U) {
      constexpr int j = jmin + g * G + decltype(U)::value;
      if constexpr (j <= jmax) colstep<K0, BK, ILO, IHI, false, j, M>(a, buf[g & 1][decltype(U)::value], acc);
    });
  });
}

// ---- products (Section 2 / Algorithms 1 and 2) ----------------------------

// t = a * b, 2N normalised limbs.
template <int N, typename M = PlainMad>
__device__ __forceinline__ void mul_sb(const uint32_t (&a)[N], const uint32_t (&b)[N], uint32_t (&t)[2 * N]) {
  constexpr int BK = kColBlock;
  uint64_t carry = 0;
  sfor<0, (2 * N - 1 + BK - 1) / BK>([&](auto B) {
    constexpr int k0 = decltype(B)::value * BK;
    constexpr int bk = (2 * N - 1 - k0) < BK ? (2 * N - 1 - k0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
    colblock<k0, bk, 0, N - 1, 0, N - 1, false, M>(a, b, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      const uint64_t v = acc[d] + carry;
      t[k0 + d] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;
    });
    compiler_fence();
  });
  t[2 * N - 1] = (uint32_t)carry;
}

// t = a^2: off-diagonal products once, doubled, plus the diagonal (Algorithm 2).
template <int N, typename M = PlainMad>
__device__ __forceinline__ void sqr_sb(const uint32_t (&a)[N], uint32_t (&t)[2 * N]) {
  constexpr int BK = kColBlock;
  uint64_t carry = 0;
  sfor<0, (2 * N - 1 + BK - 1) / BK>([&](auto B) {
    constexpr int k0 = decltype(B)::value * BK;
    constexpr int bk = (2 * N - 1 - k0) < BK ? (2 * N - 1 - k0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
    colblock<k0, bk, 0, N - 1, 0, N - 1, true, M>(a, a, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      constexpr int k = k0 + d;
      uint64_t v = acc[d] << 1;
      if constexpr ((k & 1) == 0) M::template mac<d>(v, a[k / 2], a[k / 2]);
      v += carry;
      t[k] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;
    });
    compiler_fence();
  });
  t[2 * N - 1] = (uint32_t)carry;
}

// ---- Montgomery reduction (Section 5) --------------------------------------
//
// q = (T mod R) * N' mod R                         (Algorithm 6, step 1)
// TRUNC: only the partial products q_i N_j with i + j >= n - 2 are formed
//   (Theorem 2).  With P_w = sum_{i+j=w} q_i N_j:
//     a2 = T[n-2] + P_{n-2},  a1 = T[n-1] + P_{n-1} + (a2 >> 28)
//     k  = (a1 >> 28) + [(a1 | a2) mod 2^28 != 0]
//   k is the exact carry into limb n: the skipped columns only add a carry
//   smaller than 2^56 below column n-2, and limbs 0..n-1 of T + qN vanish
//   (Theorem 1, equation (3)), so k = ceil((a1 2^28 + a2 mod 2^28) / 2^56).
//   The indicator is the analogue of c_add (equation (1)).
// PLAIN: every partial product of q N is formed (Algorithm 3, B_fma); the
//   carry out of the low n limbs is floor(L/R) + [T mod R != 0] with L the
//   low columns of q N (Theorem 1's form with the whole q N).
// C = floor(T / R) + sum_{w >= n} P_w 2^{28 (w - n)} + k   (Algorithm 6, step 4)
//
// The modulus limbs m[j] and N' limbs np[j] come from LDS (lane-private
// columns, [limb][lane]: consecutive lanes hit consecutive banks) through
// ldm / ldnp; each word read feeds up to eight products.
template <int N, bool TRUNC, typename M = PlainMad, typename LoadM, typename LoadNP>
__device__ __forceinline__ void redc_blk(const uint32_t (&t)[2 * N], LoadM&& ldm, LoadNP&& ldnp, uint32_t (&c)[N]) {
  static_assert(N >= 3, "size class too small");
  constexpr int BK = kColBlock;
  uint32_t q[N];
  // q = T_lo * N' mod R: columns 0 .. N-1, column k = sum_{i<=k} t[i] np[k-i].
  uint64_t carry = 0, lcarry = 0;
  uint32_t nz = 0;  // PLAIN: T_lo != 0
  if constexpr (!TRUNC) sfor<0, N>([&](auto I) { nz |= t[decltype(I)::value]; });
  (void)nz;
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
  // PLAIN: every product of q N, the low ones (columns below n, their sum L) after q.  The low n limbs
  // of T + q N vanish, so the carry into limb n is (T_lo + L) / R = floor(L / R) + [T_lo != 0]
  // (T_lo + (L mod R) is 0 or R, and 0 only when T_lo = 0, hence q = 0 and L = 0): Theorem 1's
  // floor(T/R) + floor(qN/R) + c_add with the whole q N.  Normalising L's columns gives floor(L / R),
  // and T_lo is dead once q is formed.
  if constexpr (!TRUNC) {
    sfor<0, (N + BK - 1) / BK>([&](auto B) {
      constexpr int k0 = decltype(B)::value * BK;
      constexpr int bk = (N - k0) < BK ? (N - k0) : BK;
      uint64_t acc[bk];
      sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
      colblock_ld<k0, bk, 0, N - 1, 0, N - 1, M>(q, ldm, acc);
      sfor<0, bk>([&](auto D) { lcarry = (acc[decltype(D)::value] + lcarry) >> kLimbBits; });
      compiler_fence();
    });
    lcarry += nz != 0u ? 1u : 0u;
  }
  // q * N: columns from n-2 (truncated, Theorem 2) or n (plain, the low
  // columns are done) to 2n-2
  constexpr int W0 = TRUNC ? N - 2 : N;
  constexpr int NCOL = 2 * N - 1 - W0;
  carry = TRUNC ? 0 : lcarry;
  uint64_t a2 = 0;
  sfor<0, (NCOL + BK - 1) / BK>([&](auto B) {
    constexpr int w0 = W0 + decltype(B)::value * BK;
    constexpr int bk = (2 * N - 1 - w0) < BK ? (2 * N - 1 - w0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = t[w0 + decltype(D)::value]; });
    colblock_ld<w0, bk, 0, N - 1, 0, N - 1, M>(q, ldm, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      constexpr int w = w0 + d;
      if constexpr (TRUNC && w == N - 2) {
        a2 = acc[d];
      } else if constexpr (TRUNC && w == N - 1) {
        const uint64_t a1 = acc[d] + (a2 >> kLimbBits);
        carry = (a1 >> kLimbBits) + ((((uint32_t)a1 | (uint32_t)a2) & kLimbMask) != 0u ? 1u : 0u);
      } else {
        const uint64_t v = acc[d] + carry;
        c[w - N] = (uint32_t)v & kLimbMask;
        carry = v >> kLimbBits;
      }
    });
    compiler_fence();
  });
  c[N - 1] = (uint32_t)(carry + t[2 * N - 1]);
}

// ---- word-interleaved Montgomery multiplication (Section 4, Algorithm 4) --
//
// CIOS: for each limb a_i of the first operand, Y += a_i B, then
// q_i = (Y mod 2^28) N'_0 mod 2^28 and Y = (Y + q_i N) / 2^28, with
// N'_0 = -N^{-1} mod 2^28.  Y lives in 64-bit column sums y[w] indexed by
// absolute weight, so the division by 2^28 is a renaming: only column i,
// divisible by 2^28 once q_i N is added, hands its carry to column i+1.  The
// q_i are the limbs of q = -AB N^{-1} mod R, so c = (AB + qN) / R exactly,
// the same integer as the separated reduction.  Column w collects at most
// 2n products below 2^56 plus a carry below 2^37, within 64 bits for
// n <= 127.  2n^2 + n multiplications, for a square too: the interleaving
// leaves no room for the symmetry of Algorithm 2.
//
// The outer steps run in groups of P: q_i needs only the products of q_i' N
// (i' < i) that land in column i, so inside a group each q_i' adds its
// products with N_0 .. N_{P-1} at once, and one sweep over N_P .. N_{n-1}
// then adds the rest for the whole group, reading each modulus limb once per
// group instead of once per step.  Every product is formed once; the result
// does not depend on P.
//
// a_i and the modulus limbs come through the loaders lda / ldm (LDS: the
// column sums, b and the group's q take the registers); b is in registers.
// c may alias b: it is written after the last read.
constexpr int kCiosGroup = 4;

template <int N, int P, typename LoadA, typename LoadM>
__device__ __forceinline__ void cios_mul(LoadA&& lda, const uint32_t (&b)[N], LoadM&& ldm, uint32_t n0,
                                         uint32_t (&c)[N]) {
  static_assert(N >= 2 && N <= 127, "64-bit column sums hold at most 254 products plus a carry");
  uint64_t y[2 * N];
  sfor<0, 2 * N>([&](auto W) { y[decltype(W)::value] = 0; });
  sfor<0, (N + P - 1) / P>([&](auto G) {
    constexpr int i0 = decltype(G)::value * P;
    constexpr int pg = (N - i0) < P ? (N - i0) : P;
    uint32_t q[pg], mlo[pg];
    sfor<0, pg>([&](auto J) { mlo[decltype(J)::value] = ldm(decltype(J)::value); });
    sfor<0, pg>([&](auto Q) {
      constexpr int p = decltype(Q)::value;
      constexpr int i = i0 + p;
      const uint32_t ai = lda(i);
      sfor<0, N>([&](auto J) {
        constexpr int j = decltype(J)::value;
        y[i + j] += (uint64_t)ai * b[j];
      });
      q[p] = ((uint32_t)y[i] * n0) & kLimbMask;
      sfor<0, pg>([&](auto J) {
        constexpr int j = decltype(J)::value;
        y[i + j] += (uint64_t)q[p] * mlo[j];
      });
      y[i + 1] += y[i] >> kLimbBits;
    });
    sfor<pg, N>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const uint32_t mj = ldm(j);
      sfor<0, pg>([&](auto Q) {
        constexpr int p = decltype(Q)::value;
        y[i0 + p + j] += (uint64_t)q[p] * mj;
      });
    });
  });
  uint64_t carry = 0;
  sfor<0, N>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const uint64_t v = y[N + k] + carry;
    c[k] = (uint32_t)v & kLimbMask;
    carry = v >> kLimbBits;
  });
}

// ---- block routines for the block-level schoolbook (large size classes) ---

// r = a * b mod 2^(28 H): the low half of the product (Algorithm 6 step 1 on a block).
template <int H>
__device__ __forceinline__ void lo_sb(const uint32_t (&a)[H], const uint32_t (&b)[H], uint32_t (&r)[H]) {
  constexpr int BK = kColBlock;
  uint64_t carry = 0;
  sfor<0, (H + BK - 1) / BK>([&](auto B) {
    constexpr int k0 = decltype(B)::value * BK;
    constexpr int bk = (H - k0) < BK ? (H - k0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
    colblock<k0, bk, 0, H - 1, 0, H - 1, false, PlainMad>(a, b, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      const uint64_t v = acc[d] + carry;
      r[k0 + d] = (uint32_t)v & kLimbMask;
      carry = v >> kLimbBits;
    });
    compiler_fence();
  });
}

// v = sum over the partial products a_i b_j with i + j >= H - 2 of
// a_i b_j 2^(28 (i + j - H + 2)), normalised to H + 2 limbs: the partial
// products of Theorem 2 that a block contributes at or above column n - 2.
template <int H>
__device__ __forceinline__ void hi_sb(const uint32_t (&a)[H], const uint32_t (&b)[H], uint32_t (&v)[H + 2]) {
  constexpr int BK = kColBlock;
  constexpr int W0 = H - 2, NCOL = 2 * H - 1 - W0;
  uint64_t carry = 0;
  sfor<0, (NCOL + BK - 1) / BK>([&](auto B) {
    constexpr int w0 = W0 + decltype(B)::value * BK;
    constexpr int bk = (2 * H - 1 - w0) < BK ? (2 * H - 1 - w0) : BK;
    uint64_t acc[bk];
    sfor<0, bk>([&](auto D) { acc[decltype(D)::value] = 0; });
    colblock<w0, bk, 0, H - 1, 0, H - 1, false, PlainMad>(a, b, acc);
    sfor<0, bk>([&](auto D) {
      constexpr int d = decltype(D)::value;
      const uint64_t x = acc[d] + carry;
      v[w0 + d - W0] = (uint32_t)x & kLimbMask;
      carry = x >> kLimbBits;
    });
    compiler_fence();
  });
  v[H + 1] = (uint32_t)carry;
}

// ---- layout: 64-bit words <-> 28-bit limbs (expand / contract, Section 6) -

// x = the low 28 N bits of the W-word little-endian value at src.
template <int N, int W>
__device__ __forceinline__ void expand(const uint64_t* __restrict__ src, uint32_t (&x)[N]) {
  uint64_t w[W];
  sfor<0, W>([&](auto J) { w[decltype(J)::value] = src[decltype(J)::value]; });
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int bit = kLimbBits * i, wd = bit / 64, off = bit % 64;
    uint64_t v = 0;
    if constexpr (wd < W) v = w[wd] >> off;
    if constexpr (off > 64 - kLimbBits && wd + 1 < W) v |= w[wd + 1] << (64 - off);
    x[i] = (uint32_t)v & kLimbMask;
  });
}

// dst = the W-word value of the limbs x (bits beyond 64 W are dropped).
template <int N, int W>
__device__ __forceinline__ void contract(const uint32_t (&x)[N], uint64_t* __restrict__ dst) {
  sfor<0, W>([&](auto J) {
    constexpr int j = decltype(J)::value;
    uint64_t v = 0;
    sfor<0, N>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int lo = kLimbBits * i - 64 * j;  // bit position of limb i inside word j
      if constexpr (lo > -kLimbBits && lo < 64) {
        if constexpr (lo >= 0)
          v |= (uint64_t)x[i] << lo;
        else
          v |= (uint64_t)x[i] >> (-lo);
      }
    });
    dst[j] = v;
  });
}

// ---- dense packing of 28-bit limbs into 32-bit words (window table) --------

// Words holding N 28-bit limbs.
constexpr int packed_words(int n) { return (kLimbBits * n + 31) / 32; }

// w = the N limbs of x as a dense little-endian bit string of packed_words(N) words.
template <int N>
__device__ __forceinline__ void pack(const uint32_t (&x)[N], uint32_t (&w)[packed_words(N)]) {
  sfor<0, packed_words(N)>([&](auto J) {
    constexpr int j = decltype(J)::value;
    uint32_t v = 0;
    sfor<0, N>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int lo = kLimbBits * i - 32 * j;  // bit position of limb i inside word j
      if constexpr (lo > -kLimbBits && lo < 32) {
        if constexpr (lo >= 0)
          v |= x[i] << lo;
        else
          v |= x[i] >> (-lo);
      }
    });
    w[j] = v;
  });
}

// x = the N 28-bit limbs of the dense bit string w.
template <int N>
__device__ __forceinline__ void unpack(const uint32_t (&w)[packed_words(N)], uint32_t (&x)[N]) {
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int bit = kLimbBits * i, wd = bit / 32, off = bit % 32;
    uint32_t v = w[wd] >> off;
    if constexpr (off > 32 - kLimbBits && wd + 1 < packed_words(N)) v |= w[wd + 1] << (32 - off);
    x[i] = v & kLimbMask;
  });
}

// c = x - m if x >= m else x (constant time; x <= m on entry gives [0, m)).
template <int N>
__device__ __forceinline__ void canon(uint32_t (&x)[N], const uint32_t (&m)[N]) {
  uint32_t d[N];
  int64_t br = 0;
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    int64_t v = (int64_t)x[i] - (int64_t)m[i] + br;
    d[i] = (uint32_t)v & kLimbMask;
    br = v >> kLimbBits;  // 0 or -1
  });
  const uint32_t keep = (uint32_t)(br != 0 ? 0xFFFFFFFFu : 0u);  // borrow => x < m => keep x
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    x[i] = (x[i] & keep) | (d[i] & ~keep);
  });
}

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

}  // namespace mx
