#pragma once
// Batched Montgomery kernels (templates; instantiated per size class in mx_class.hip) for gfx950: context set-up, modmul / modsqr and
// constant-time fixed-window modular exponentiation (Algorithm 7).
// One instance per lane; see mx_core.hpp for the arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mx_core.hpp"
#include "mx_internal.h"

namespace mx {

// Raw buffer descriptor over `bytes` bytes at p (gfx9 word 3: 32-bit untyped
// dwords).  Buffer accesses take a per-lane byte offset plus a uniform scalar
// offset (no per-load address arithmetic) and are bounds-checked by the
// hardware: an out-of-range load returns 0, an out-of-range store is dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_buf(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint32_t bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 0);
}
// Cache policy of the constant-time table scan's reads.  Every window streams the whole table of every
// instance; when the launch's tables exceed the 256 MB last-level cache no cache level can keep them, and the
// scan reads them with the non-temporal policy (bit NT of the buffer instruction's cache-policy field), which
// leaves the caches to the rest of the kernel's traffic.  Tables that fit are read with the default policy.
constexpr int kPolicyNT = 2;
constexpr uint64_t kCacheBytes = 256ull << 20;
__device__ __forceinline__ bool stream_tables(uint32_t count, uint32_t nent, uint32_t entry_bytes) {
  return (uint64_t)count * nent * entry_bytes > kCacheBytes;
}
template <int P>
__device__ __forceinline__ uint32_t bload_pol(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, P);
}

// Copies this lane's N and N' limbs into its LDS column ([limb][lane]).  Each
// lane reads back only its own column, so no barrier is needed.  The reads of
// each array are all issued before the first LDS write, so their latencies
// overlap.
template <int N>
__device__ __forceinline__ void stage_ctx(uint32_t* s_ctx, const uint32_t* cn, const uint32_t* cnp, size_t cs,
                                          uint32_t lane) {
  uint32_t v[N];
  sfor<0, N>([&](auto I) { v[decltype(I)::value] = cn[(size_t)decltype(I)::value * cs]; });
  sfor<0, N>([&](auto I) { s_ctx[decltype(I)::value * 64 + lane] = v[decltype(I)::value]; });
  sfor<0, N>([&](auto I) { v[decltype(I)::value] = cnp[(size_t)decltype(I)::value * cs]; });
  sfor<0, N>([&](auto I) { s_ctx[(N + decltype(I)::value) * 64 + lane] = v[decltype(I)::value]; });
}

// ---- context: N, N' = -N^{-1} mod R, R mod N, R^2 mod N (Section 4) -------
//
// N' digit by digit: q_i = acc_0 * (-N_0^{-1}) mod 2^28 with acc += q_i N and a
// one-limb shift per digit (the q of the Montgomery reduction of 1, taken
// limb-serially; acc keeps only the limbs still below R).  R mod N and
// R^2 mod N start from 2^(t-1) <= N (t = bit length of N) and double with a
// conditional subtraction until 2^(28 n) and 2^(56 n).
template <int N, int W>
__global__ void __launch_bounds__(64) k_ctx_init(const uint64_t* __restrict__ mods, CtxDev ctx) {
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  if (gid >= ctx.count) return;
  uint32_t m[N];
  expand<N, W>(mods + (size_t)gid * W, m);
  const size_t cs = ctx.stride;
#pragma unroll 1
  for (int i = 0; i < N; ++i) ctx.n[(size_t)i * cs + gid] = m[i];

  // -N_0^{-1} mod 2^28 by Newton's iteration on 32-bit words (3 -> 96 bits)
  uint32_t inv = m[0];
  for (int it = 0; it < 5; ++it) inv *= 2u - m[0] * inv;
  const uint32_t n0p = (0u - inv) & kLimbMask;
  {
    uint32_t acc[N];  // acc[j] is limb i + j of 1 + (q_0 .. q_{i-1}) N
    sfor<0, N>([&](auto J) { acc[decltype(J)::value] = decltype(J)::value == 0 ? 1u : 0u; });
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
      const uint32_t qi = (uint32_t)(((uint64_t)acc[0] * n0p) & kLimbMask);
      ctx.np[(size_t)i * cs + gid] = qi;
      uint64_t carry = 0;
      sfor<0, N>([&](auto J) {
        constexpr int j = decltype(J)::value;
        const uint64_t v = (uint64_t)acc[j] + (uint64_t)qi * m[j] + carry;
        acc[j] = (uint32_t)v & kLimbMask;
        carry = v >> kLimbBits;
      });
      sfor<0, N - 1>([&](auto J) { acc[decltype(J)::value] = acc[decltype(J)::value + 1]; });
      acc[N - 1] = 0;
    }
  }
  uint32_t t = 0;  // bit length of N
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if (m[i]) t = kLimbBits * i + (32u - __clz(m[i]));
  });
  uint32_t r[N];
  sfor<0, N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    r[i] = (uint32_t)i == (t - 1) / kLimbBits ? 1u << ((t - 1) % kLimbBits) : 0u;
  });
  const uint32_t total = 2u * kLimbBits * N - (t - 1);
#pragma unroll 1
  for (uint32_t s = 0; s < total; ++s) {
    // r = 2 r (r < N <= R/4 so no limb overflows), then subtract N if r >= N
    uint32_t top = 0;
    sfor<0, N>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const uint32_t v = (r[i] << 1) | top;
      top = r[i] >> (kLimbBits - 1);
      r[i] = v & kLimbMask;
    });
    canon<N>(r, m);
    if (s + t == (uint32_t)(kLimbBits * N)) {  // r = 2^(t - 1 + s + 1) = R mod N
#pragma unroll 1
      for (int i = 0; i < N; ++i) ctx.r1[(size_t)i * cs + gid] = r[i];
    }
  }
#pragma unroll 1
  for (int i = 0; i < N; ++i) ctx.r2[(size_t)i * cs + gid] = r[i];
}

// ---- batched modmul / modsqr ---------------------------------------------
// A word in LDS named by its address space (3), so that reads of it are ds_read.
typedef __attribute__((address_space(3))) uint32_t LdsU32;

// out = REDC(a * b) (or REDC(a^2)) for each instance, values of RW words.
template <int N, int RW, bool TRUNC, bool SQR>
__global__ void __launch_bounds__(64) k_mont(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                             const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                             uint64_t* __restrict__ out, uint32_t count, uint32_t coff) {
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  const uint32_t* cn = ctx.n + c;
  const uint32_t* cnp = ctx.np + c;
  const size_t cs = ctx.stride;

  __shared__ uint32_t s_ctx[2 * N * 64];
  stage_ctx<N>(s_ctx, cn, cnp, cs, threadIdx.x);

  uint32_t x[N];
  expand<N, RW>(a + (size_t)inst * RW, x);
  uint32_t t[2 * N];
  // one product and one reduction per launch: the rotated carry-outs measure faster here
  if constexpr (SQR) {
    sqr_sb<N, RotMad>(x, t);
  } else {
    uint32_t y[N];
    expand<N, RW>(b + (size_t)inst * RW, y);
    mul_sb<N, RotMad>(x, y, t);
  }
  uint32_t r[N];
  // N and N' are read through a pointer in the LDS address space: through a
  // generic pointer the reads are flat loads (the vector memory path, 64-bit
  // addresses that spilled), and volatile reads would wait for each read
  const LdsU32* sm = (const LdsU32*)(s_ctx + threadIdx.x);
  redc_blk<N, TRUNC, RotMad>(t, [&](int i) { return sm[i * 64]; }, [&](int i) { return sm[(N + i) * 64]; }, r);
  if (live) contract<N, RW>(r, out + (size_t)inst * RW);
}

// out = REDC(a * b) by the word-interleaved multiplication of Algorithm 4
// (cios_mul); a square is the product with b = a (the method has no squaring
// of its own).  LDS column of the lane: rows 0 .. N-1 the modulus, rows
// N .. 2N-1 the first operand; N'_0 is limb 0 of N'.
template <int N, int RW>
__global__ void __launch_bounds__(64) k_mont_cios(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                  const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                  uint64_t* __restrict__ out, uint32_t count, uint32_t coff) {
  const uint32_t gid = blockIdx.x * 64 + threadIdx.x;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  const size_t cs = ctx.stride;
  const uint32_t lane = threadIdx.x;

  __shared__ uint32_t s_ctx[2 * N * 64];
  uint32_t x[N], r[N];
  sfor<0, N>([&](auto I) { x[decltype(I)::value] = ctx.n[(size_t)decltype(I)::value * cs + c]; });
  sfor<0, N>([&](auto I) { s_ctx[decltype(I)::value * 64 + lane] = x[decltype(I)::value]; });
  const uint32_t n0 = ctx.np[c];
  expand<N, RW>(a + (size_t)inst * RW, x);
  sfor<0, N>([&](auto I) { s_ctx[(N + decltype(I)::value) * 64 + lane] = x[decltype(I)::value]; });
  // plain reads: the compiler reads each word once and keeps what does not
  // fit the 256 VGPRs in AGPRs (volatile reads, one per use, spill to scratch)
  const uint32_t* sm = s_ctx + lane;
  expand<N, RW>(b + (size_t)inst * RW, x);
  cios_mul<N, kCiosGroup>([&](int i) { return sm[(N + i) * 64]; }, x, [&](int j) { return sm[j * 64]; }, n0, r);
  if (live) contract<N, RW>(r, out + (size_t)inst * RW);
}

// ---- constant-time fixed-window exponentiation (Algorithm 7) --------------
//
// Per lane: A~ = REDC(base * R^2); table G[0] = R mod N, G[1] = A~,
// G[i] = REDC(G[i-1] A~); Y = G[top window]; for each further window:
// w squarings, a full masked scan of the table, one multiplication;
// finally REDC(Y) and one conditional subtraction.  Every branch depends
// only on public values (step counter, window size, exponent length); the
// table addresses depend only on the entry counter.
//
// The whole schedule runs through one loop so that the squaring code, the
// multiplication code and the reduction each exist once in the binary.
enum StepKind : int { kSqr = 0, kMulR2 = 1, kMulG1 = 2, kMulSel = 3, kMulOne = 4, kLoadSel = 5 };

// Start-phase stagger.  Every wavefront runs the same schedule at the same
// speed, so without it the table scans of all wavefronts (the one phase that
// streams memory) coincide, and the four wavefronts of a compute unit compete
// for its load path at the same moments while it idles during the squarings.
// Wavefronts start at 16 phases spread over one window period, about
// 12 (w + 1) N^2 cycles ((w + 1) Montgomery operations of about 2 N^2
// products at about 6 cycles each): the SIMD a wavefront runs on (read from
// the HW_ID register) picks a quarter of the period, so the four wavefronts of
// a compute unit scan at different times, and the block index a sixteenth
// within it.  s_sleep(127) waits 127 x 64 cycles.
__device__ __forceinline__ uint32_t simd_id() {
  // s_getreg_b32 HW_REG_HW_ID (id 4), bits [5:4]: the SIMD of this wavefront
  return (uint32_t)__builtin_amdgcn_s_getreg(4 | (4 << 6) | ((2 - 1) << 11));
}

template <int N>
__device__ __forceinline__ void stagger(uint32_t block, uint32_t w) {
  const uint32_t phase = simd_id() * 4u + ((block >> 3) & 3u);
  const uint32_t naps = phase * ((w + 1u) * 12u * (uint32_t)(N * N) / 16u / (127u * 64u));
  for (uint32_t i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(127);
}

// Modular exponentiation of one tile of 64 instances (one wavefront).
// tile0: first instance of the tile; lane l handles instance tile0 + l (the
// lanes past `count` recompute the last instance and store nothing).
// table: this wavefront's own workspace region of tbytes >= 2^w NW 256 bytes,
// word-major over its 64 lanes (entry e, word j of lane l at byte
// (e NW + j) 256 + 4 l, NW = packed_words(N): the entry's limbs packed
// densely), so that every read of the table scan is a whole 256-byte row and
// a wavefront's table is one contiguous range of memory.
// s_ctx: 2 N 64 words of LDS for the lane's N and N'.
// CIOS: every Montgomery product is the word-interleaved one of Algorithm 4
// (cios_mul); s_ctx then holds the modulus (rows 0 .. N-1) and a copy of Y,
// the first operand of every product (rows N .. 2N-1), and TRUNC is unused.
// KREDC: the truncated high half of every product's q N is formed by one-level
// Karatsuba (kara_high_half) instead of redc_blk's schoolbook columns.
template <int N, int BW, bool TRUNC, bool CIOS = false, bool KREDC = false>
__device__ __forceinline__ void modexp_tile(const CtxDev& ctx, const uint32_t* __restrict__ cidx,
                                            const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                            uint32_t ebits, uint32_t ewords, uint32_t w,
                                            uint64_t* __restrict__ out, uint32_t count, uint32_t* __restrict__ table,
                                            uint32_t tbytes, uint32_t coff, uint32_t tile0, uint32_t* s_ctx) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t gid = tile0 + lane;
  const bool live = gid < count;
  const uint32_t inst = live ? gid : count - 1;
  uint32_t c = cidx ? cidx[inst] : inst + coff;
  c = c < ctx.count ? c : 0u;
  const uint32_t* cn = ctx.n + c;
  const uint32_t* cnp = ctx.np + c;
  const size_t cs = ctx.stride;
  const __amdgpu_buffer_rsrc_t tr = make_buf(table, tbytes);
  const uint32_t tvo = lane * 4u;
  const uint32_t tls = 256u;  // bytes between consecutive words of an entry
  // entries are stored densely packed: NW 32-bit words of 28-bit limbs
  constexpr int NW = packed_words(N);
  const uint32_t ent_bytes = (uint32_t)NW * tls;
  const uint64_t* e64 = ex + (size_t)inst * ewords;

  const uint32_t nent = 1u << w;
  const bool stream = stream_tables(count, nent, (uint32_t)packed_words(N) * 4u);
  const uint32_t nwin = ebits ? (ebits + w - 1) / w : 1u;

  uint32_t n0 = 0;
  if constexpr (CIOS) {
    uint32_t v[N];
    sfor<0, N>([&](auto I) { v[decltype(I)::value] = cn[(size_t)decltype(I)::value * cs]; });
    sfor<0, N>([&](auto I) { s_ctx[decltype(I)::value * 64 + lane] = v[decltype(I)::value]; });
    n0 = cnp[0];
  } else {
    stage_ctx<N>(s_ctx, cn, cnp, cs, lane);
  }
  const uint32_t* sm = s_ctx + lane;

  uint32_t y[N];
  {  // G[0] = R mod N
    sfor<0, N>([&](auto I) { y[decltype(I)::value] = ctx.r1[(size_t)decltype(I)::value * cs + c]; });
    uint32_t pw[NW];
    pack<N>(y, pw);
    sfor<0, NW>([&](auto J) { bstore(tr, pw[decltype(J)::value], tvo, (uint32_t)decltype(J)::value * tls); });
  }
  expand<N, BW>(base + (size_t)inst * BW, y);

  const uint32_t n_tab = nent - 1;              // REDC(base R^2), then nent - 2 table products
  const uint32_t n_main = (nwin - 1) * (w + 1);  // per window: w squarings + 1 product
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
      const uint32_t r = s - n_tab - 1;
      win = nwin - 2 - r / (w + 1);
      kind = (r % (w + 1)) < w ? kSqr : kMulSel;
    } else {
      kind = kMulOne;
    }

    if constexpr (CIOS) {
      // Y, the first operand of this step's product, goes to the lane's LDS
      // column before the table scan, so it takes no registers meanwhile
      if (kind != kLoadSel) sfor<0, N>([&](auto I) { s_ctx[(N + decltype(I)::value) * 64 + lane] = y[decltype(I)::value]; });
    }
    uint32_t bsrc[N];
    if (kind == kMulSel || kind == kLoadSel) {
      // window bits [win w, win w + w) of the exponent, clipped to ebits
      const uint32_t p = win * w;
      const uint32_t width = ebits > p ? (ebits - p < w ? ebits - p : w) : 0u;
      const uint32_t lo = p >> 6, sh = p & 63;
      uint64_t v = (width > 0 && lo < ewords) ? e64[lo] >> sh : 0ull;
      if (width > 0 && sh + width > 64 && lo + 1 < ewords) v |= e64[lo + 1] << (64 - sh);
      const uint32_t bits = (uint32_t)v & ((1u << width) - 1u);
      // full masked scan: every entry is read, the selected one survives
      uint32_t selw[NW];
      sfor<0, NW>([&](auto I) { selw[decltype(I)::value] = 0; });
      // two entries per iteration keep 2 NW loads in flight (nent >= 2); the policy (a uniform choice from
      // the launch's size) selects one of two copies of the loop
      auto scan = [&](auto pol) {
        constexpr int P = decltype(pol)::value;
#pragma nounroll
        for (uint32_t e = 0; e < nent; e += 2) {
          const uint32_t mask0 = e == bits ? 0xFFFFFFFFu : 0u;
          const uint32_t mask1 = e + 1 == bits ? 0xFFFFFFFFu : 0u;
          const uint32_t s0 = e * ent_bytes;
          uint32_t v0[NW], v1[NW];
          sfor<0, NW>([&](auto I) {
            constexpr int i = decltype(I)::value;
            v0[i] = bload_pol<P>(tr, tvo, s0 + (uint32_t)i * tls);
            v1[i] = bload_pol<P>(tr, tvo, s0 + ent_bytes + (uint32_t)i * tls);
          });
          sfor<0, NW>([&](auto I) {
            constexpr int i = decltype(I)::value;
            selw[i] |= (v0[i] & mask0) | (v1[i] & mask1);
          });
        }
      };
      if (stream)
        scan(std::integral_constant<int, kPolicyNT>{});
      else
        scan(std::integral_constant<int, 0>{});
      unpack<N>(selw, bsrc);
      if (kind == kLoadSel) {
        sfor<0, N>([&](auto I) { y[decltype(I)::value] = bsrc[decltype(I)::value]; });
        continue;
      }
    } else if (kind == kMulR2 || kind == kMulG1) {
      if (kind == kMulR2) {
        const uint32_t* src = ctx.r2 + c;
        sfor<0, N>([&](auto I) {
          constexpr int i = decltype(I)::value;
          bsrc[i] = src[(size_t)i * cs];
        });
      } else {
        uint32_t pw[NW];
        sfor<0, NW>([&](auto I) { pw[decltype(I)::value] = bload(tr, tvo, ent_bytes + (uint32_t)decltype(I)::value * tls); });
        unpack<N>(pw, bsrc);
      }
    } else if (kind == kMulOne) {
      sfor<0, N>([&](auto I) { bsrc[decltype(I)::value] = decltype(I)::value == 0 ? 1u : 0u; });
    }

    if constexpr (CIOS) {
      // one copy of the multiplication code: a squaring multiplies Y by itself
      if (kind == kSqr) sfor<0, N>([&](auto I) { bsrc[decltype(I)::value] = y[decltype(I)::value]; });
      cios_mul<N, kCiosGroup>([&](int i) { return sm[(N + i) * 64]; }, bsrc, [&](int j) { return sm[j * 64]; }, n0,
                              y);
    } else {
      uint32_t t[2 * N];
      if (kind == kSqr)
        sqr_sb<N>(y, t);
      else
        mul_sb<N>(y, bsrc, t);
      if constexpr (KREDC) {  // truncated high half of q N by one-level Karatsuba (same value)
        uint32_t q[N];
        low_half_q<N, PlainMad>(t, [&](int i) { return sm[(N + i) * 64]; }, q);
        kara_high_half<N, PlainMad>(t, q, [&](int j) { return sm[j * 64]; }, y);
      } else {
        redc_blk<N, TRUNC>(t, [&](int i) { return sm[i * 64]; }, [&](int i) { return sm[(N + i) * 64]; }, y);
      }
    }
    if (store_e >= 0) {
      const uint32_t s0 = (uint32_t)store_e * ent_bytes;
      uint32_t pw[NW];
      pack<N>(y, pw);
      sfor<0, NW>([&](auto I) { bstore(tr, pw[decltype(I)::value], tvo, s0 + (uint32_t)decltype(I)::value * tls); });
    }
  }
  uint32_t m[N];
  sfor<0, N>([&](auto I) { m[decltype(I)::value] = sm[decltype(I)::value * 64]; });
  canon<N>(y, m);
  if (live) contract<N, BW>(y, out + (size_t)inst * BW);
}

// ws: ceil(count / 64) tile regions of 2^w packed_words(N) 256 bytes each, one per block.
template <int N, int BW, bool TRUNC>
__global__ void __launch_bounds__(64) k_modexp(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                               const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                               uint32_t ebits, uint32_t ewords, uint32_t w,
                                               uint64_t* __restrict__ out, uint32_t count, uint32_t* __restrict__ ws,
                                               uint32_t ws_bytes, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * N * 64];
  const uint32_t tile0 = blockIdx.x * 64;
  const uint32_t tbytes = (1u << w) * (uint32_t)packed_words(N) * 256u;
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  stagger<N>(blockIdx.x, w);
  modexp_tile<N, BW, TRUNC>(ctx, cidx, base, ex, ebits, ewords, w, out, count, ws + (size_t)blockIdx.x * (tbytes / 4u),
                            tbytes, coff, tile0, s_ctx);
}

// As k_modexp with the word-interleaved multiplication (Algorithm 4).
template <int N, int BW>
__global__ void __launch_bounds__(64) k_modexp_cios(CtxDev ctx, const uint32_t* __restrict__ cidx,
                                                    const uint64_t* __restrict__ base, const uint64_t* __restrict__ ex,
                                                    uint32_t ebits, uint32_t ewords, uint32_t w,
                                                    uint64_t* __restrict__ out, uint32_t count,
                                                    uint32_t* __restrict__ ws, uint32_t ws_bytes, uint32_t coff) {
  __shared__ uint32_t s_ctx[2 * N * 64];
  const uint32_t tile0 = blockIdx.x * 64;
  const uint32_t tbytes = (1u << w) * (uint32_t)packed_words(N) * 256u;
  if ((uint64_t)(blockIdx.x + 1) * tbytes > ws_bytes) return;  // unreachable: the launcher checked ws
  stagger<N>(blockIdx.x, w);
  modexp_tile<N, BW, false, true>(ctx, cidx, base, ex, ebits, ewords, w, out, count,
                                  ws + (size_t)blockIdx.x * (tbytes / 4u), tbytes, coff, tile0, s_ctx);
}

}  // namespace mx
