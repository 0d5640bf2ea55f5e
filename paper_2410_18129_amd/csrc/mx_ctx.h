// Host-side context object shared by the ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/montexp.h"
#include "mx_internal.h"

// Records a printf-style message for mont_last_error() and returns st.
mx_status mx_fail(mx_status st, const char* fmt, ...);

// Montgomery contexts of one size class (definition of the opaque mont_ctx).
struct mont_ctx {
  const mx::ClassOps* ops = nullptr;
  uint32_t bits = 0;
  uint32_t limbs = 0;
  uint32_t count = 0;
  int device = 0;
  mx::CtxDev dev{};
  void* mem = nullptr;
  size_t bytes = 0;
  // per-instance workspace owned by the context (grow-only; guarded by ws_mu)
  std::mutex ws_mu;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // the two half-size intermediates of rsa_crt_batch when this is the context
  // of the first primes (grow-only; guarded by crt_mu, which is taken before ws_mu)
  std::mutex crt_mu;
  void* crt = nullptr;
  size_t crt_bytes = 0;
};

