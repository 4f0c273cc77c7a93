// LDS bank-conflict probe for gfx950: one wavefront per block writes (wr_k<P>) or reads
// (rd_k<P>) one float2 per lane at the LDS index pattern P, 2048 times, so that rocprofv3's
// SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE / SQ_INSTS_LDS per kernel give the cycles one
// 8-byte access of that pattern costs.  The patterns are generic strides and the lane-address
// patterns of the 1024-point transform's exchanges and column staging (fft.hpp), before and
// after their paddings were chosen.  The measurement behind the LDS paddings of fft.hpp;
// summarised by `python -m paper_2604_02624_amd.profiling lds <counter csv>`.
//
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         lds_bank_probe.hip -o lds_bank_probe
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                      \
  do {                                                                             \
    hipError_t e = (x);                                                            \
    if (e != hipSuccess) {                                                         \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e), __LINE__);    \
      std::exit(1);                                                                \
    }                                                                              \
  } while (0)

constexpr int kIters = 2048;
constexpr int kSlots = 9216;  // float2 per block (72 KB); every pattern stays below it
constexpr int kPatterns = 12;

// LDS index (in float2) of lane i under pattern p
__host__ __device__ inline int pattern(int p, int i) {
  switch (p) {
    case 0: return i;                                   // linear
    case 1: return 2 * i;                               // stride 2
    case 2: return 4 * i;                               // stride 4
    case 3: return 16 * i;                              // stride 16
    case 4: return (i % 16) + 32 * (i / 16);            // 16-lane runs 32 apart
    case 5: return (i % 4) + 64 * (i / 4);              // 4-lane runs 64 apart
    case 6: { const int a = 8 * i; return a + (a >> 5); }             // 1024 stage-0 write, shift 5
    case 7: { const int a = 8 * i; return a + (a >> 4); }             // 1024 stage-0 write, shift 4
    case 8: { const int a = (i / 8) * 64 + i % 8; return a + (a >> 5); }     // stage-1 write, shift 5
    case 9: { const int a = (i / 8) * 64 + i % 8; return a + (a / 64) * 8; } // stage-1, 8 per 64
    case 10: return (i % 8) * 1148 + i / 8;             // column staging, 1148-slot regions
    case 11: return (i % 8) * 1146 + i / 8;             // column staging, 1146-slot regions
    default: return i;
  }
}

template <int P>
__global__ void __launch_bounds__(64) wr_k(float2* out) {
  __shared__ float2 buf[kSlots];
  const int a = pattern(P, threadIdx.x);
  float2 v = make_float2(static_cast<float>(threadIdx.x), 1.f);
  for (int it = 0; it < kIters; ++it) {
    buf[a] = v;
    v.x += 1.f;
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): one access in flight at a time
    __builtin_amdgcn_wave_barrier();
  }
  __builtin_amdgcn_wave_barrier();
  out[blockIdx.x * 64 + threadIdx.x] = buf[threadIdx.x];
}

template <int P>
__global__ void __launch_bounds__(64) rd_k(float2* out) {
  __shared__ float2 buf[kSlots];
  for (int i = threadIdx.x; i < kSlots; i += 64) buf[i] = make_float2(static_cast<float>(i), 0.f);
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  const int a = pattern(P, threadIdx.x);
  float2 acc = make_float2(0.f, 0.f);
  for (int it = 0; it < kIters; ++it) {
    const float2 u = buf[a + (it & 1)];
    acc.x += u.x;
    acc.y += u.y;
  }
  out[blockIdx.x * 64 + threadIdx.x] = acc;
}

template <int P>
void run(float2* out, int blocks) {
  if constexpr (P < kPatterns) {
    wr_k<P><<<blocks, 64>>>(out);
    CK(hipGetLastError());
    rd_k<P><<<blocks, 64>>>(out);
    CK(hipGetLastError());
    run<P + 1>(out, blocks);
  }
}

int main() {
  for (int p = 0; p < kPatterns; ++p)
    for (int i = 0; i < 64; ++i)
      if (pattern(p, i) + 1 >= kSlots) {
        std::printf("pattern %d leaves the buffer\n", p);
        return 1;
      }
  const int blocks = 4096;
  float2* out;
  CK(hipMalloc(&out, sizeof(float2) * blocks * 64));
  run<0>(out, blocks);
  CK(hipDeviceSynchronize());
  CK(hipFree(out));
  std::printf("done\n");
  return 0;
}
