// Issue-rate probe for gfx950: the denominator of the library's roofline.
//
// Part 1 (throughput): each lane runs 8 independent chains of one VALU
// instruction, 16 blocks of 256 threads per compute unit, and the rate is
// compared with 256 CUs x 64 lanes x 2.4 GHz (one lane-op per lane per cycle).
// Part 2 (waves per SIMD): one workgroup per CU (each holds more than half
// of the CU's LDS) of 4, 8 or 16 wavefronts, so each SIMD runs exactly 1, 2 or
// 4 of them; 1..16 independent chains; cycles per instruction per SIMD.
// Only ALU instructions are issued from inline assembly; the results are
// stored so nothing is optimised away.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <utility>

#define CHK(x)                                                                    \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);       \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

enum Op { kMad64, kMulLo, kMulHi, kMadU24, kFmaF64, kAddCo, kLshlAdd64, kAdd3, kDpp, kMad64Rot4, kMad64Rot8, kNumOps };
static const char* kNames[] = {"v_mad_u64_u32",  "v_mul_lo_u32",   "v_mul_hi_u32", "v_mad_u32_u24", "v_fma_f64",
                               "v_add_co_u32",   "v_lshl_add_u64", "v_add3_u32",   "v_mov_b32_dpp",
                               "v_mad_u64_u32, carry-out over 4 SGPR pairs",
                               "v_mad_u64_u32, carry-out over 8 SGPR pairs"};

// v_mad_u64_u32 whose carry-out goes to SGPR pair k (s[40+2k : 41+2k]), k in 0..7
template <int K>
__device__ __forceinline__ uint64_t mad_sd(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t r;
  if constexpr (K == 0) asm volatile("v_mad_u64_u32 %0, s[40:41], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s40", "s41");
  if constexpr (K == 1) asm volatile("v_mad_u64_u32 %0, s[42:43], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s42", "s43");
  if constexpr (K == 2) asm volatile("v_mad_u64_u32 %0, s[44:45], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s44", "s45");
  if constexpr (K == 3) asm volatile("v_mad_u64_u32 %0, s[46:47], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s46", "s47");
  if constexpr (K == 4) asm volatile("v_mad_u64_u32 %0, s[48:49], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s48", "s49");
  if constexpr (K == 5) asm volatile("v_mad_u64_u32 %0, s[50:51], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s50", "s51");
  if constexpr (K == 6) asm volatile("v_mad_u64_u32 %0, s[52:53], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s52", "s53");
  if constexpr (K == 7) asm volatile("v_mad_u64_u32 %0, s[54:55], %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c) : "s54", "s55");
  return r;
}

template <int M, int I>
__device__ __forceinline__ uint64_t mad_rot(uint32_t a, uint32_t b, uint64_t c) {
  return mad_sd<I % M>(a, b, c);
}

template <int M, int... I>
__device__ __forceinline__ void rot_all(const uint32_t* a, const uint32_t* b, uint64_t* c,
                                        std::integer_sequence<int, I...>) {
  ((c[I] = mad_rot<M, I>(a[I], b[I], c[I])), ...);
}

template <int OP, int CH, int ITERS, int UNROLL>
__device__ __forceinline__ uint64_t chains(uint32_t seed) {
  uint32_t a[CH], b[CH];
  uint64_t c[CH];
  double d[CH], e[CH];
  for (int i = 0; i < CH; ++i) {
    a[i] = seed + threadIdx.x * 7u + i;
    b[i] = a[i] * 3u + 1u;
    c[i] = a[i];
    d[i] = (double)a[i];
    e[i] = (double)b[i];
  }
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      if constexpr (OP == kMad64Rot4 || OP == kMad64Rot8) {
        constexpr int M = OP == kMad64Rot4 ? 4 : 8;
        rot_all<M>(a, b, c, std::make_integer_sequence<int, CH>{});
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        if constexpr (OP == kMad64) {
          uint64_t r;
          asm volatile("v_mad_u64_u32 %0, s[40:41], %1, %2, %3" : "=v"(r) : "v"(a[i]), "v"(b[i]), "v"(c[i]) : "s40", "s41");
          c[i] = r;
        }
        if constexpr (OP == kMulLo) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b[i]));
        if constexpr (OP == kMulHi) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b[i]));
        if constexpr (OP == kMadU24) asm volatile("v_mad_u32_u24 %0, %0, %1, %0" : "+v"(a[i]) : "v"(b[i]));
        if constexpr (OP == kFmaF64) asm volatile("v_fma_f64 %0, %0, %1, %0" : "+v"(d[i]) : "v"(e[i]));
        if constexpr (OP == kAddCo) asm volatile("v_add_co_u32 %0, vcc, %0, %1" : "+v"(a[i]) : "v"(b[i]) : "vcc");
        if constexpr (OP == kLshlAdd64) asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(c[i]) : "v"((uint64_t)b[i]));
        if constexpr (OP == kAdd3) asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(a[i]) : "v"(b[i]));
        if constexpr (OP == kDpp)
          asm volatile("v_mov_b32_dpp %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf" : "=v"(a[i]) : "v"(b[i]));
      }
    }
  }
  uint64_t s = 0;
  for (int i = 0; i < CH; ++i) s += c[i] + a[i] + (uint64_t)d[i];
  return s;
}

template <int OP, int CH, int ITERS, int UNROLL>
__global__ void k_probe(uint64_t* out, uint32_t seed) {
  extern __shared__ uint32_t pin[];  // sized by the launch to keep one workgroup per CU
  if (seed == 0) pin[threadIdx.x] = 0;  // never taken: keeps the allocation live
  out[blockIdx.x * blockDim.x + threadIdx.x] = chains<OP, CH, ITERS, UNROLL>(seed);
}

template <int OP, int CH, int ITERS, int UNROLL>
static int timed(uint64_t* buf, int blocks, int threads, size_t lds, double* ms_out) {
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  if (lds > 0)
    CHK(hipFuncSetAttribute((const void*)k_probe<OP, CH, ITERS, UNROLL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_probe<OP, CH, ITERS, UNROLL>), dim3(blocks), dim3(threads), lds, 0, buf, 1u);
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  CHK(hipEventRecord(e0));
  hipLaunchKernelGGL((k_probe<OP, CH, ITERS, UNROLL>), dim3(blocks), dim3(threads), lds, 0, buf, 1u);
  CHK(hipEventRecord(e1));
  CHK(hipEventSynchronize(e1));
  float ms = 0;
  CHK(hipEventElapsedTime(&ms, e0, e1));
  *ms_out = ms;
  CHK(hipEventDestroy(e0));
  CHK(hipEventDestroy(e1));
  return 0;
}

template <int OP>
static int throughput(uint64_t* buf, int cus) {
  const int blocks = cus * 16;
  double ms;
  if (timed<OP, 8, 256, 8>(buf, blocks, 256, 0, &ms)) return 1;
  const double ops = (double)blocks * 256 * 256 * 8 * 8;
  const double rate = ops / (ms * 1e-3);
  printf("| %s | %.2f | %.3f |\n", kNames[OP], rate * 1e-12, rate / (256.0 * 64 * 2.4e9));
  return 0;
}

template <int OP, int CH>
static int per_simd(uint64_t* buf, int cus, int waves_per_simd) {
  double ms;
  const size_t lds = 96 * 1024;  // more than half of the 160 KB: one workgroup per CU
  if (timed<OP, CH, 2048, 64 / CH>(buf, cus, 256 * waves_per_simd, lds, &ms)) return 1;
  const double cyc = ms * 1e-3 * 2.4e9 / (2048.0 * 64 * waves_per_simd);
  printf("| %s | %d | %d | %.2f |\n", kNames[OP], waves_per_simd, CH, cyc);
  return 0;
}

int main() {
  hipDeviceProp_t p;
  CHK(hipGetDeviceProperties(&p, 0));
  printf("device %s, %d CUs, clock %d kHz, LDS per workgroup %zu B\n\n", p.gcnArchName, p.multiProcessorCount,
         p.clockRate, (size_t)p.sharedMemPerBlock);
  uint64_t* buf;
  CHK(hipMalloc(&buf, (size_t)p.multiProcessorCount * 16 * 256 * sizeof(uint64_t)));
  printf("Throughput, 8 independent chains per lane, %d blocks x 256 threads\n\n", p.multiProcessorCount * 16);
  printf("| instruction | T lane-ops/s | fraction of 256 x 64 x 2.4 GHz |\n|---|---|---|\n");
  int rc = 0;
  rc |= throughput<kMad64>(buf, p.multiProcessorCount);
  rc |= throughput<kMulLo>(buf, p.multiProcessorCount);
  rc |= throughput<kMulHi>(buf, p.multiProcessorCount);
  rc |= throughput<kMadU24>(buf, p.multiProcessorCount);
  rc |= throughput<kFmaF64>(buf, p.multiProcessorCount);
  rc |= throughput<kAddCo>(buf, p.multiProcessorCount);
  rc |= throughput<kLshlAdd64>(buf, p.multiProcessorCount);
  rc |= throughput<kAdd3>(buf, p.multiProcessorCount);
  rc |= throughput<kDpp>(buf, p.multiProcessorCount);
  rc |= throughput<kMad64Rot8>(buf, p.multiProcessorCount);
  const int cu = p.multiProcessorCount;
  if (p.sharedMemPerBlock < 96 * 1024) {
    printf("LDS per workgroup below 96 KB: cannot pin one workgroup per CU\n");
    CHK(hipFree(buf));
    return rc;
  }
  printf("\nOne workgroup per CU, 1/2/4 wavefronts per SIMD: SIMD cycles per wavefront instruction\n\n");
  printf("| instruction | waves per SIMD | independent chains | cycles |\n|---|---|---|---|\n");
  rc |= per_simd<kMad64, 1>(buf, cu, 1);
  rc |= per_simd<kMad64, 4>(buf, cu, 1);
  rc |= per_simd<kMad64, 16>(buf, cu, 1);
  rc |= per_simd<kMad64, 4>(buf, cu, 2);
  rc |= per_simd<kMad64, 16>(buf, cu, 2);
  rc |= per_simd<kMad64, 4>(buf, cu, 4);
  rc |= per_simd<kMad64Rot4, 8>(buf, cu, 1);
  rc |= per_simd<kMad64Rot8, 8>(buf, cu, 1);
  rc |= per_simd<kMad64Rot8, 16>(buf, cu, 1);
  rc |= per_simd<kLshlAdd64, 4>(buf, cu, 1);
  rc |= per_simd<kMulLo, 4>(buf, cu, 1);
  rc |= per_simd<kMulHi, 4>(buf, cu, 1);
  rc |= per_simd<kMadU24, 4>(buf, cu, 1);
  rc |= per_simd<kAddCo, 4>(buf, cu, 1);
  rc |= per_simd<kAdd3, 4>(buf, cu, 1);
  rc |= per_simd<kFmaF64, 4>(buf, cu, 1);
  CHK(hipFree(buf));
  return rc;
}
