// gptr.h -- global-address-space view of a pointer value read from memory.
//
// A pointer loaded from a descriptor (in LDS or in global memory) is
// generic, and every access through it becomes a flat instruction, which
// the compiler can only wait for with both memory counters drained: each
// load then completes before the next one issues.  tc_global rebuilds the
// (wave-uniform) address from its integer value directly in the global
// address space, leaving no generic origin for the optimiser to fold the
// cast back into, so every use becomes a global access.  The value must be
// the same in every active lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename T>
__device__ __forceinline__ T* tc_global(T* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(v >> 32));
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
