// Host stand-in for the few HIP names fft.hpp uses, so that its radix butterflies can be
// compiled with the host compiler and checked on the CPU (tests/test_fft_host.py).  The
// wave-level LDS ordering builtins become no-ops: only code that never touches LDS is run.
#pragma once
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
struct float2 {
  float x, y;
};
inline float2 make_float2(float a, float b) { return float2{a, b}; }
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)0)
inline void __syncthreads() {}
