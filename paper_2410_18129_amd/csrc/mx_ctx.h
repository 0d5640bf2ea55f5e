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
  // library-owned workspace (guarded by ws_mu): sized by mont_ctx_init and grown only by
  // mont_ctx_reserve, never inside a batch call.  ws_done is recorded after the last work enqueued
  // on it; every batch call that uses it first makes its stream wait for ws_done, so calls on
  // different streams take turns on the workspace instead of racing on it.
  std::mutex ws_mu;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipEvent_t ws_done = nullptr;
};

