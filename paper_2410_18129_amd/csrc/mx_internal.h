// Internal interface between the C ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mx {

// Device context arrays, limb-major: limb i of context c at arr[i * stride + c].
struct CtxDev {
  uint32_t* n;   // modulus N
  uint32_t* np;  // N' = -N^{-1} mod R
  uint32_t* r2;  // R^2 mod N
  uint32_t* r1;  // R mod N (Montgomery form of 1)
  uint32_t count;
  uint32_t stride;
};

// Launchers of one size class (one instantiation of the kernel templates).
// Workspace: ws_rows(modexp, w) 32-bit words per instance, laid out limb-major
// with `tstride` instances per row (ws_bytes = rows * tstride * 4 < 2 GiB);
// `coff` is added to the instance index to find its context when cidx is NULL.
// impl: 0 = the class's default kernels, 1 = block-level schoolbook over
// 37-limb blocks (available when has_block; the default above 2048 bits),
// 2 = block kernels with a one-level Karatsuba product (when has_kara).
// redc: one of Redc below; kRedcCios with has_cios (impl 0 in the register-resident classes, the
// block-word CIOS with one lane per instance above 2048 bits); kRedcKara as the ABI checks.
enum Redc : int { kRedcTrunc = 0, kRedcPlain = 1, kRedcCios = 2, kRedcKara = 3 };
struct ClassOps {
  int bits;
  int limbs;
  bool has_block;
  bool has_kara;
  bool has_cios;
  hipError_t (*ctx_init)(const uint64_t* mods, const CtxDev& ctx, hipStream_t st);
  uint32_t (*ws_rows)(int impl, bool modexp, uint32_t w);
  hipError_t (*mont)(int impl, int redc, bool sqr, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* a,
                     const uint64_t* b, uint64_t* out, uint32_t count, uint32_t* ws, uint32_t tstride,
                     uint32_t ws_bytes, uint32_t coff, hipStream_t st);
  hipError_t (*modexp)(int impl, int redc, const CtxDev& ctx, const uint32_t* cidx, const uint64_t* base,
                       const uint64_t* ex, uint32_t ebits, uint32_t ewords, uint32_t w, uint64_t* out,
                       uint32_t count, uint32_t* ws, uint32_t tstride, uint32_t ws_bytes, uint32_t coff,
                       hipStream_t st);
  // Two exponentiation batches of `count` instances each in one launch (nullptr where not
  // built): batch 0 on ctx0 with exponents ex0, batch 1 on ctx1 with ex1; bases and outputs
  // are one array of 2 count instances (batch 1 from instance count on), cidx indexes both
  // contexts; ws holds 2 ceil(count/64) tile regions of ws_rows(0, true, w) 64 words.
  hipError_t (*modexp_pair)(bool trunc, const CtxDev& ctx0, const CtxDev& ctx1, const uint32_t* cidx,
                            const uint64_t* base, const uint64_t* ex0, const uint64_t* ex1, uint32_t ebits,
                            uint32_t ewords, uint32_t w, uint64_t* out, uint32_t count, uint32_t* ws,
                            uint32_t ws_bytes, hipStream_t st);
};

// Largest workspace one launch may use: a buffer descriptor spans < 2 GiB.
constexpr size_t kMaxWsBytes = 0x7FFFFFFFull;

// Size classes built into the library.
#define MX_FOR_EACH_CLASS(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(3072) X(4096)

#define MX_DECL_CLASS(B) const ClassOps* class_ops_##B();
MX_FOR_EACH_CLASS(MX_DECL_CLASS)
#undef MX_DECL_CLASS

// nullptr for an unsupported class
inline const ClassOps* class_ops(uint32_t bits) {
  switch (bits) {
#define MX_CASE(B) \
  case B:          \
    return class_ops_##B();
    MX_FOR_EACH_CLASS(MX_CASE)
#undef MX_CASE
    default:
      return nullptr;
  }
}

}  // namespace mx
