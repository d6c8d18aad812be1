// Global-to-LDS copies (gfx950 global_load_lds, 16 bytes per lane) for
// kernels that stream an operand through an LDS ring.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cnmf {

// LDS byte address of a pointer into a __shared__ array
__device__ __forceinline__ uint32_t lds_addr(const uint8_t* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t*)p;
}

// 16 bytes per lane from global memory into LDS: lane l's bytes land at
// lds_base + 16 l (lds_base wave-uniform).  Written in asm so that the
// compiler, which would otherwise wait for every such load in flight before
// any LDS read, leaves the waiting to the explicit counts of the caller (the
// instruction writes no registers).  M0 holds the LDS base; the compiler
// reserves M0 and warns that it does not restore it across the statement,
// which is harmless only while nothing else in the calling kernels uses M0
// (true of the kernels that call this: M0 appears in their code only here).
__device__ __forceinline__ void dma16(const void* gptr, uint32_t lds_base) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gptr), "s"(lds_base)
      : "memory", "m0");
}

// 4 bytes per lane (no alignment beyond the element's): lane l's bytes land
// at lds_base + 4 l.
__device__ __forceinline__ void dma4(const void* gptr, uint32_t lds_base) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dword %0, off"
      :
      : "v"(gptr), "s"(lds_base)
      : "memory", "m0");
}

}  // namespace cnmf
