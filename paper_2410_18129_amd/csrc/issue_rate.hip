// Issue-rate probe for gfx950: the denominator of the library's roofline.
//
// Part 1 (throughput): each lane runs 8 independent chains of one VALU
// instruction, 16 blocks of 256 threads per compute unit, and the rate is
// compared with 256 CUs x 64 lanes x 2.4 GHz (one lane-op per lane per cycle).
// Part 2 (one wavefront per SIMD): 1024 blocks of 64 threads, 1..16
// independent chains, cycles per instruction per wavefront.
// Only ALU instructions are issued from inline assembly; the results are
// stored so nothing is optimised away.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define CHK(x)                                                                    \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);       \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

enum Op { kMad64, kMulLo, kMulHi, kMadU24, kFmaF64, kAddCo, kLshlAdd64, kAdd3, kDpp, kNumOps };
static const char* kNames[] = {"v_mad_u64_u32",  "v_mul_lo_u32",   "v_mul_hi_u32", "v_mad_u32_u24", "v_fma_f64",
                               "v_add_co_u32",   "v_lshl_add_u64", "v_add3_u32",   "v_mov_b32_dpp"};

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
  out[blockIdx.x * blockDim.x + threadIdx.x] = chains<OP, CH, ITERS, UNROLL>(seed);
}

template <int OP, int CH, int ITERS, int UNROLL>
static int timed(uint64_t* buf, int blocks, int threads, double* ms_out) {
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  hipLaunchKernelGGL((k_probe<OP, CH, ITERS, UNROLL>), dim3(blocks), dim3(threads), 0, 0, buf, 1u);
  CHK(hipDeviceSynchronize());
  CHK(hipEventRecord(e0));
  hipLaunchKernelGGL((k_probe<OP, CH, ITERS, UNROLL>), dim3(blocks), dim3(threads), 0, 0, buf, 1u);
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
  if (timed<OP, 8, 256, 8>(buf, blocks, 256, &ms)) return 1;
  const double ops = (double)blocks * 256 * 256 * 8 * 8;
  const double rate = ops / (ms * 1e-3);
  printf("| %s | %.2f | %.3f |\n", kNames[OP], rate * 1e-12, rate / (256.0 * 64 * 2.4e9));
  return 0;
}

template <int OP, int CH>
static int single_wave(uint64_t* buf) {
  double ms;
  if (timed<OP, CH, 2048, 64 / CH>(buf, 1024, 64, &ms)) return 1;
  const double cyc = ms * 1e-3 * 2.4e9 / (2048.0 * 64);
  printf("| %s | %d | %.2f |\n", kNames[OP], CH, cyc);
  return 0;
}

int main() {
  hipDeviceProp_t p;
  CHK(hipGetDeviceProperties(&p, 0));
  printf("device %s, %d CUs, clock %d kHz\n\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
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
  printf("\nOne wavefront per SIMD (1024 blocks x 64 threads): cycles per instruction per wavefront\n\n");
  printf("| instruction | independent chains | cycles |\n|---|---|---|\n");
  rc |= single_wave<kMad64, 1>(buf);
  rc |= single_wave<kMad64, 2>(buf);
  rc |= single_wave<kMad64, 4>(buf);
  rc |= single_wave<kMad64, 16>(buf);
  rc |= single_wave<kMadU24, 1>(buf);
  rc |= single_wave<kMadU24, 4>(buf);
  rc |= single_wave<kAddCo, 4>(buf);
  rc |= single_wave<kFmaF64, 4>(buf);
  CHK(hipFree(buf));
  return rc;
}
