// Device code of the propagation passes for gfx950: row pass, column pass (transform and
// matrix-core forms), transfer-function table.  Included by the per-transform-length
// translation units (dpx_pass.hip), which instantiate the kernels of one length each.
//
// One propagation over a gap (Section 4, Eq. 4/5 via the angular spectrum) is split in two
// passes over a [N rows][M columns] complex plane per wavelength ("spec"):
//   row pass    : transform along x (the N non-zero rows of the zero-padded plane only)
//   column pass : transform along y, multiply by the transfer function, inverse along y,
//                 keep the N aperture rows
// and the next row pass starts with the inverse transform along x.  Zero padding is placed
// at the high end of each axis instead of centring it: a circular convolution commutes with
// shifts, so cropping the same corner returns the same N x N field.
#pragma once

#include <hip/hip_runtime.h>

#include "dpx_internal.hpp"
#include "fft.hpp"
#include "phase.hpp"

namespace dpx {

// Word 3 of a raw buffer resource on gfx9: 32-bit data format, no stride or swizzle.
constexpr int kBufferRsrcWord3 = 0x00020000;

// One 8-byte load through a buffer resource: byte offset = voff (per lane) + soff (scalar).
__device__ __forceinline__ float2 buffer_load_c64(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

// Eq. 1 with the +j reading: t = exp(-ca h) exp(+i 2 pi rt h); phase argument in double.
__device__ __forceinline__ float2 transmission(float h, const WlConst& c) {
  asm volatile("" : "+v"(h));  // the FP64 height stays per wavelength (as in opaque_lane_row)
  const double hd = static_cast<double>(h);
  float2 t = cis_turns(c.rt * hd);
  if (c.ca != 0.0) {
    const float a = expf(-static_cast<float>(c.ca * hd));
    t.x *= a;
    t.y *= a;
  }
  return t;
}

template <int M, int MODE>
constexpr int row_block_threads() { return row_threads_for(Geo<M>::P, MODE); }

// ------------------------------------------------------------------------------------------
// Row pass.  A block owns G = 256 / P consecutive rows (one transform group per row) and
// loops over a run of wavelengths, so the row's heights stay in registers.
// ------------------------------------------------------------------------------------------
// Block (bx, by) of a row pass: rows row_lo + bx G .. + G - 1, wavelength block by.
// lds_all: G exchange regions; tw: room for the twiddle table (both in LDS).
template <int M, int PAD, int MODE, int V = 0>
__device__ __forceinline__ void row_body(const RowArgs& a, int bx, int by, float2* lds_all, float2* tw) {
  constexpr int kRowThreads = row_block_threads<M, MODE>();
  constexpr int E = Geo<M>::E;
  constexpr int P = Geo<M>::P;
  constexpr int G = kRowThreads / P;
  constexpr int EN = E / PAD;  // registers that hold x < N
  constexpr bool HALF = (PAD == 2);
  constexpr int RG = Geo<M>::ROW_REGION;
  stage_twiddles<M, V>(tw, a.tw, threadIdx.x, kRowThreads);
  __syncthreads();

  const int N = M / PAD;
  const int g = threadIdx.x / P;
  const int j0 = threadIdx.x % P;
  float2* lds = lds_all + g * RG;
  const int y_raw = a.row_lo + bx * G + g;
  const bool active = y_raw < a.row_hi;
  const int y = active ? y_raw : a.row_lo;
  const size_t plane = static_cast<size_t>(N) * M;
  const size_t nn = static_cast<size_t>(N) * N;

  const int wb = a.w_begin + by * a.w_per_block;
  const int we = min(wb + a.w_per_block, a.w_begin + a.w_count);

  float hreg[EN];
  if constexpr (MODE == ROW_FWD_FIRST || MODE == ROW_FWD_MID || MODE == ROW_ADJ_MID ||
                MODE == ROW_ADJ_LAST || MODE == ROW_ADJ_LAST_U) {
    const bool read_h = MODE != ROW_FWD_FIRST || !a.no_layer;
#pragma unroll
    for (int t = 0; t < EN; ++t) hreg[t] = read_h ? a.h[static_cast<size_t>(y) * N + j0 + P * t] : 0.f;
  }

  if constexpr (MODE == ROW_FWD_FIRST) {
    float2 uin[EN];
#pragma unroll
    for (int t = 0; t < EN; ++t)
      uin[t] = a.u_in ? a.u_in[static_cast<size_t>(y) * N + j0 + P * t] : make_float2(1.f, 0.f);
    for (int w = wb; w < we; ++w) {
      const WlConst c = a.wl[w];
      const int wc = w - a.w_begin;
      float2 reg[E];
      if (a.no_layer) {
#pragma unroll
        for (int t = 0; t < EN; ++t) reg[t] = uin[t];
      } else {
#pragma unroll
        for (int t = 0; t < EN; ++t) reg[t] = cmul(uin[t], transmission(hreg[t], c));
      }
      if (a.store_ckpt && !a.ckpt_first && active) {
        float2* ck = a.ckpt + (static_cast<size_t>(a.layer - a.ckpt_first) * a.ckpt_w_stride + wc) * nn +
                     static_cast<size_t>(y) * N;
#pragma unroll
        for (int t = 0; t < EN; ++t) ck[j0 + P * t] = reg[t];
      }
      fft<M, false, HALF, V, XPad<M>::ROWS>(reg, lds, j0, tw);
      if (active) {
        float2* dst = a.spec + wc * plane + static_cast<size_t>(y) * M;
#pragma unroll
        for (int t = 0; t < E; ++t) dst[j0 + P * t] = reg[t];
      }
    }
  } else if constexpr (MODE == ROW_FWD_MID) {
    for (int w = wb; w < we; ++w) {
      const WlConst c = a.wl[w];
      const int wc = w - a.w_begin;
      float2* row = a.spec + wc * plane + static_cast<size_t>(y) * M;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false, V, XPad<M>::ROWS>(reg, lds, j0, tw);
#pragma unroll
      for (int t = 0; t < EN; ++t) reg[t] = cmul(reg[t], transmission(hreg[t], c));
      if (a.store_ckpt && active) {
        float2* ck = a.ckpt + (static_cast<size_t>(a.layer - a.ckpt_first) * a.ckpt_w_stride + wc) * nn +
                     static_cast<size_t>(y) * N;
#pragma unroll
        for (int t = 0; t < EN; ++t) ck[j0 + P * t] = reg[t];
      }
      fft<M, false, HALF, V, XPad<M>::ROWS>(reg, lds, j0, tw);
      if (active) {
#pragma unroll
        for (int t = 0; t < E; ++t) row[j0 + P * t] = reg[t];
      }
    }
  } else if constexpr (MODE == ROW_FWD_LAST) {
    const int F = a.fov;
    const int x0 = (N - F) / 2;
    for (int w = wb; w < we; ++w) {
      const int wc = w - a.w_begin;
      const float2* row = a.spec + wc * plane + static_cast<size_t>(y) * M;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false, V, XPad<M>::ROWS>(reg, lds, j0, tw);
      if (active) {
        float2* dst = a.ofov + static_cast<size_t>(wc) * F * F + static_cast<size_t>(y - x0) * F;
#pragma unroll
        for (int t = 0; t < EN; ++t) {
          const int x = j0 + P * t;
          if (x >= x0 && x < x0 + F) dst[x - x0] = reg[t];
        }
      }
    }
  } else if constexpr (MODE == ROW_ADJ_SEED) {
    const int F = a.fov, b = a.bin, T = F / b;
    const int x0 = (N - F) / 2;
    for (int w = wb; w < we; ++w) {
      const int wc = w - a.w_begin;
      const float2* o = a.ofov + static_cast<size_t>(wc) * F * F + static_cast<size_t>(y - x0) * F;
      const float* d = a.dl_di + static_cast<size_t>(w) * T * T + static_cast<size_t>((y - x0) / b) * T;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < EN; ++t) {
        const int x = j0 + P * t;
        if (x >= x0 && x < x0 + F) {
          const float s = 2.0f * d[(x - x0) / b];
          reg[t] = cscale(o[x - x0], s);
        } else {
          reg[t] = make_float2(0.f, 0.f);
        }
      }
      fft<M, false, HALF, V, XPad<M>::ROWS>(reg, lds, j0, tw);
      if (active) {
        float2* dst = a.spec + wc * plane + static_cast<size_t>(y) * M;
#pragma unroll
        for (int t = 0; t < E; ++t) dst[j0 + P * t] = reg[t];
      }
    }
  } else {  // ROW_ADJ_MID, ROW_ADJ_LAST, ROW_ADJ_LAST_U
    // ROW_ADJ_LAST_U: the input field meets the first layer directly, so the field after the
    // first transmission is u_in t_0(h); the pass rebuilds it from the input and the heights
    // with the same operations as the first forward pass (so the same bits) instead of
    // reading back a stored copy.  u_in is read where it is used, not held in registers.
    constexpr bool REBUILD = (MODE == ROW_ADJ_LAST_U);
    const float2* urow = (REBUILD && a.u_in) ? a.u_in + static_cast<size_t>(y) * N : nullptr;
    float acc[EN];
#pragma unroll
    for (int t = 0; t < EN; ++t) acc[t] = 0.f;
    for (int w = wb; w < we; ++w) {
      const WlConst c = a.wl[w];
      const int wc = w - a.w_begin;
      float2* row = a.spec + wc * plane + static_cast<size_t>(y) * M;
      const float2* ck = REBUILD ? nullptr
                                 : a.ckpt + (static_cast<size_t>(a.layer - a.ckpt_first) * a.ckpt_w_stride + wc) * nn +
                                       static_cast<size_t>(y) * N;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false, V, XPad<M>::ROWS>(reg, lds, j0, tw);
      const float ct = static_cast<float>(c.ct);
      const float ca = static_cast<float>(c.ca);
#pragma unroll
      for (int t = 0; t < EN; ++t) {
        const float2 gv = reg[t];
        float2 v;
        if constexpr (REBUILD) {
          const float2 u = urow ? urow[j0 + P * t] : make_float2(1.f, 0.f);
          v = cmul(u, transmission(hreg[t], c));
        } else {
          v = ck[j0 + P * t];
        }
        // conj(g) v; acc += -ct Im - ca Re
        const float re = fmaf(gv.x, v.x, gv.y * v.y);
        const float im = fmaf(gv.x, v.y, -(gv.y * v.x));
        acc[t] = fmaf(-ct, im, fmaf(-ca, re, acc[t]));
        if constexpr (MODE == ROW_ADJ_MID) reg[t] = cmulc(gv, transmission(hreg[t], c));
      }
      if constexpr (MODE == ROW_ADJ_MID) {
        fft<M, false, HALF, V, XPad<M>::ROWS>(reg, lds, j0, tw);
        if (active) {
#pragma unroll
          for (int t = 0; t < E; ++t) row[j0 + P * t] = reg[t];
        }
      }
    }
    if (active) {
      float* dst = a.dh_part +
                   (static_cast<size_t>(a.chunk_base + by) * a.layers + a.layer) * nn +
                   static_cast<size_t>(y) * N;
      if (a.accumulate) {
#pragma unroll
        for (int t = 0; t < EN; ++t) dst[j0 + P * t] += acc[t];
      } else {
#pragma unroll
        for (int t = 0; t < EN; ++t) dst[j0 + P * t] = acc[t];
      }
    }
  }
}

template <int M, int PAD, int MODE, int V = 0>
__global__ void __launch_bounds__((row_block_threads<M, MODE>())) row_kernel(RowArgs a) {
  __shared__ float2 lds_all[row_block_threads<M, MODE>() / Geo<M>::P * Geo<M>::ROW_REGION];
  __shared__ float2 tw[twiddle_count<M, V>()];
  row_body<M, PAD, MODE, V>(a, blockIdx.x, blockIdx.y, lds_all, tw);
}

// The same pass with at least three wavefronts per SIMD (a cap of 168 registers): the forward
// middle pass at transform 1600 fits it without spilling, and three of its 240-thread blocks
// then share a CU instead of two.
template <int M, int PAD, int MODE>
__global__ void __launch_bounds__((row_block_threads<M, MODE>())) __attribute__((amdgpu_waves_per_eu(3)))
row_kernel_w3(RowArgs a) {
  __shared__ float2 lds_all[row_block_threads<M, MODE>() / Geo<M>::P * Geo<M>::ROW_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  row_body<M, PAD, MODE>(a, blockIdx.x, blockIdx.y, lds_all, tw);
}

// One launch of a row pass for several designs of the same transform length and mode: each
// block finds its design's task, patches the per-call buffers into the design's arguments
// and runs the same body as the single-design kernel.
template <int M, int PAD, int MODE>
__global__ void __launch_bounds__((row_block_threads<M, MODE>())) row_group_kernel(GroupArgs g) {
  __shared__ float2 lds_all[row_block_threads<M, MODE>() / Geo<M>::P * Geo<M>::ROW_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  const int ti = group_task(g, blockIdx.x);
  const RowTask& t = static_cast<const RowTask*>(g.tasks)[ti];
  const int local = static_cast<int>(blockIdx.x) - g.block0[ti];
  if (local >= t.nblocks) return;  // alignment padding between tasks
  RowArgs a = t.a;
  a.h = g.call.h ? g.call.h + t.h_off : nullptr;
  a.u_in = g.call.u_in ? g.call.u_in + t.u_off : nullptr;
  a.dl_di = g.call.dl_di ? g.call.dl_di + t.img_off : nullptr;
  row_body<M, PAD, MODE>(a, local % t.gx, local / t.gx, lds_all, tw);
}

// The lane's first row index, opaque to the optimiser: the per-element row terms of the
// transfer function (ky, ky^2, their conversions to FP64) are the same for every wavelength, and
// left visible the compiler keeps all E of them live across the wavelength loop, which spills.
// Derived from this value they are recomputed per wavelength (a few integer operations).
__device__ __forceinline__ int opaque_lane_row(int j0) {
  asm volatile("" : "+v"(j0));
  return j0;
}

// H(kx, ky) / M^2 with the conjugate for the adjoint; 0 outside the propagating disc.  zrev is
// the phase in revolutions per unit of sqrt(q); outside the disc q is replaced by the smallest
// normal double (one maximum instead of two selects) and the result by 0.
template <int M, bool CONJ>
__device__ __forceinline__ float2 transfer(double zrev, double base, int ky) {
  const int kys = ky < M / 2 ? ky : ky - M;
  const double q = base - static_cast<double>(kys * kys);
  const float2 hh = cis_turns_hw<M * M>(zrev * sqrt_pos(fmax(q, kMinNormalF64)));
  return q > 0.0 ? (CONJ ? conjf2(hh) : hh) : make_float2(0.f, 0.f);
}

// ------------------------------------------------------------------------------------------
// Column pass.  A block owns TX adjacent columns of one wavelength's plane: it stages the
// [rows][TX] tile through LDS (coalesced 8*TX-byte row segments), each transform group
// then runs forward FFT -> transfer function -> inverse FFT on its column in registers, and
// the kept rows go back through the same LDS tile.
// ------------------------------------------------------------------------------------------
// Where a column pass takes the transfer function from: evaluated for every element, evaluated
// for the rows ky <= M/2 and shared with the mirrored rows across lanes, or read from the
// plan's table; a translated gap evaluates every element with its translation ramp folded into
// the phase; the band-limited spectrum evaluates every element inside the band.
constexpr int kHEval = 0, kHMirror = 1, kHTable = 2, kHShift = 3, kHBand = 4;

// XCD-aware order of a column pass's blocks.  Consecutive blocks go to the eight XCDs in turn,
// so blocks L and L + 8 of every run of 16 share an XCD and its L2; they take neighbouring
// column tiles of the same wavelength block, so the two halves of each 128-byte row segment
// meet in one L2 instead of being fetched twice.  Blocks are numbered L = bx + gx by from a
// multiple of 16 in launch order; with an even tile count gx a pair never straddles two
// wavelength blocks; a tail of fewer than 16 blocks keeps its order.
__device__ __forceinline__ void col_block_item(int L, int total, int gx, int& bx, int& by) {
  int item = L;
  if ((gx & 1) == 0 && L < (total & ~15)) {
    const int r = L & 15;
    item = (L & ~15) + ((r & 7) << 1) + (r >> 3);
  }
  bx = item % gx;
  by = item / gx;
}

// Block (bx, by) of a column pass: column tile bx, wavelength block by.
template <int M, int PAD, bool CONJ, int TX, int HM, bool FULL, int V = 0>
__device__ __forceinline__ void col_body(const ColArgs& a, int bx, int by, float2* tile, float2* tw) {
  constexpr int E = Geo<M>::E;
  constexpr int P = Geo<M>::P;
  constexpr int NT = TX * P;
  constexpr int LD = Geo<M>::COL_REGION;  // one column's staging rows / exchange region
  constexpr int EN = E / PAD;
  constexpr bool HALF = (PAD == 2);
  static_assert(NT / TX == P, "staging rows per pass");

  const int N = M / PAD;
  const int kx0 = bx * TX;
  const int cc = threadIdx.x % TX;
  const int yy = threadIdx.x / TX;
  const int g = threadIdx.x / P;
  const int j0 = threadIdx.x % P;
  float2* lds = tile + g * LD;
  const int kx = kx0 + g;
  const int kxs = kx < M / 2 ? kx : kx - M;
  // staged rows of tile column c start SKEW (c / 2) slots into its region (bank spread of the
  // staging with block-padded regions); the transforms' exchanges use the region from slot 0
  constexpr int SKEW = XPad<M>::SKEW;
  float2* lds_in = lds + SKEW * (g >> 1);
  float2* stg = tile + cc * LD + SKEW * (cc >> 1);

  // The block runs a.col_wpb wavelengths.  With zero padding the staged rows of the next one
  // are loaded into registers while the current one is transformed, so their latency is
  // hidden; without it those registers would not fit next to the full-length transform (nor
  // next to the band-limited source's per-element band tests) and the rows go straight to LDS.
  // Row k of a lane is one buffer load at the lane's 32-bit byte offset plus the scalar offset
  // k P M 8, so no per-row address stays live.
  constexpr bool PREFETCH = HALF && HM != kHBand;
  const int wb = by * a.col_wpb;
  const int we = min(wb + a.col_wpb, a.w_count);
  const unsigned voff = static_cast<unsigned>((((FULL ? 0 : a.in_lo) + yy) * M + kx0 + cc) * 8);
  // The plane's base address is the same in every lane; reading it through readfirstlane
  // keeps the descriptor in scalar registers (a descriptor left in vector registers makes
  // the compiler wrap every load in a loop over the distinct descriptors of the wavefront).
  auto plane = [&](int w) {
    const uint64_t base = reinterpret_cast<uint64_t>(a.spec + static_cast<size_t>(w) * N * M);
    const uint64_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(base)));
    const uint64_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(base >> 32)));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>((hi << 32) | lo), 0, N * M * 8,
                                             kBufferRsrcWord3);
  };
  // FULL: the pass reads and keeps every aperture row (all passes but the first adjoint and
  // the last forward one), so the row-range tests drop out.
  const int in_lo = FULL ? 0 : a.in_lo, in_hi = FULL ? N : a.in_hi;
  const int out_lo = FULL ? 0 : a.out_lo, out_hi = FULL ? N : a.out_hi;
  float2 pre[PREFETCH ? EN : 1];
  auto fetch = [&](int w) {
    const auto rs = plane(w);
#pragma unroll
    for (int k = 0; k < EN; ++k) {
      const int y = in_lo + yy + k * P;
      pre[PREFETCH ? k : 0] = (y < in_hi) ? buffer_load_c64(rs, voff, k * P * M * 8) : make_float2(0.f, 0.f);
      if constexpr (!PREFETCH) {
        if (y < in_hi) stg[y] = pre[0];
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < EN; ++k) {
      const int y = in_lo + yy + k * P;
      if (y < in_hi) stg[y] = pre[k];
    }
  };
  // With every row in and out, the tile elements a thread stages for the next wavelength are
  // exactly those it copies out for the current one, so the staging follows the copy-out
  // without a barrier between them.
  constexpr bool STAGE_AFTER_STORE = FULL && PREFETCH;
  if constexpr (PREFETCH) fetch(wb);
  stage_twiddles<M, V>(tw, a.tw, threadIdx.x, NT);
  if constexpr (STAGE_AFTER_STORE) stage();

  // the twiddles of one stage stay in registers for the block's wavelengths (fewer LDS reads;
  // loaded after the first barrier, which also orders the table's staging) where the transfer
  // function leaves room for them: the evaluated, table and translated sources would spill
  constexpr bool TREG = (HM == kHMirror || HM == kHBand);
  float2 treg[RegTwiddles<M, V>::N];
  for (int w = wb; w < we; ++w) {
    if constexpr (!STAGE_AFTER_STORE) {
      if constexpr (PREFETCH) stage();
      else fetch(w);
    }
    __syncthreads();
    if (TREG && w == wb) load_register_twiddles<M, V>(treg, tw, j0);
    if constexpr (PREFETCH) {
      if (w + 1 < we) fetch(w + 1);
    }

    const WlConst c = a.wl[a.w_begin + w];
    float2 reg[E];
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int y = j0 + P * t;
      reg[t] = (y >= in_lo && y < in_hi) ? lds_in[y] : make_float2(0.f, 0.f);
    }
    group_sync<M>();
    fft_sel<M, false, HALF, V, TREG>(reg, lds, j0, tw, treg);

    // transfer function H = exp(+i 2 pi z sqrt(q)) / M^2 on the propagating disc, else 0:
    // read from the plan's table of H(|kx|, |ky|) when there is one, else evaluated here.
    const double base = c.q0 - static_cast<double>(kxs * kxs);
    auto H = [&](int ky) { return transfer<M, CONJ>(a.zrev, base, ky); };
    if constexpr (HM == kHEval) {
      // the product is selected, not H: outside the disc the element becomes +0 and the compiler
      // branches the evaluation over runs of rows that lie wholly outside (a wavefront's rows are
      // consecutive ky), which at long wavelengths on a fine pitch are most of the plane
      const int jv = opaque_lane_row(j0);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int ky = jv + P * t;
        const int kys = ky < M / 2 ? ky : ky - M;
        const double q = base - static_cast<double>(kys * kys);
        const float2 hh = cis_turns_hw<M * M>(a.zrev * sqrt_pos(fmax(q, kMinNormalF64)));
        reg[t] = q > 0.0 ? cmul(reg[t], CONJ ? conjf2(hh) : hh) : make_float2(0.f, 0.f);
      }
    } else if constexpr (HM == kHBand) {
      // band-limited angular spectrum: H = 0 where |kx| or |ky| exceeds the band limit
      // sqrt(q0 / (4 zrev^2 + 1)) (in frequency indices), beyond which the sampled phase aliases
      const double lim = c.q0 / (4.0 * a.zrev * a.zrev + 1.0);
      const bool col_in = static_cast<double>(kxs * kxs) <= lim;
      const int jv = opaque_lane_row(j0);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int ky = jv + P * t;
        const int kys = ky < M / 2 ? ky : ky - M;
        const bool in = col_in && static_cast<double>(kys * kys) <= lim;
        reg[t] = in ? cmul(reg[t], H(ky)) : make_float2(0.f, 0.f);
      }
    } else if constexpr (HM == kHTable) {
      // table row of |kx|: every lane reads its E values (rows ky and M - ky share an entry)
      constexpr int HS = M / 2 + 1;
      const float2* hrow = a.htab + (static_cast<size_t>(a.w_begin + w) * HS + (kxs < 0 ? -kxs : kxs)) * HS;
      float2 hv[E];
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int ky = j0 + P * t;
        hv[t] = hrow[ky <= M / 2 ? ky : M - ky];
      }
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = cmul(reg[t], CONJ ? conjf2(hv[t]) : hv[t]);
    } else if constexpr (HM == kHShift) {
      // translated gap: H times the ramp exp(-i 2 pi (kx sx + ky sy)) (signed indices) is one
      // phase per element, z sqrt(q) - kx sx - ky sy in revolutions, reduced in FP64 like H's
      // own; conjugated for the adjoint.  Per element, so no lane holds ramp state and the
      // next wavelength's rows still fit in registers.
      const double px = static_cast<double>(kxs) * a.sx;
      const int jv = opaque_lane_row(j0);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int ky = jv + P * t;
        const int kys = ky < M / 2 ? ky : ky - M;
        const double q = base - static_cast<double>(kys * kys);
        const double ph = a.zrev * sqrt_pos(fmax(q, kMinNormalF64)) - fma(static_cast<double>(kys), a.sy, px);
        const float2 hh = cis_turns_hw<M * M>(ph);
        reg[t] = q > 0.0 ? cmul(reg[t], CONJ ? conjf2(hh) : hh) : make_float2(0.f, 0.f);
      }
    } else if constexpr (HM == kHMirror) {
      // H depends on ky^2 only: lane j0 holds ky = j0 + P t, and for t >= E/2 the row M - ky
      // is register E-1-t of lane P - j0 (lane 0 mirrors onto its own register E - t), so
      // each lane evaluates E/2 + 1 rows and fetches the others across lanes.  Streamed so
      // that only two evaluations are live at a time: step u applies row u and the mirrored
      // row E-1-u (whose value lane 0 takes from its own evaluation u+1).
      constexpr int EH = E / 2;
      const int lane = threadIdx.x & 63;
      const int src = ((lane - j0) + ((P - j0) & (P - 1))) << 2;
      float2 cur = H(j0);
#pragma unroll
      for (int u = 0; u < EH; ++u) {
        const float2 nxt = H(j0 + P * (u + 1));
        reg[u] = cmul(reg[u], cur);
        float2 m;
        m.x = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(cur.x)));
        m.y = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(cur.y)));
        if (j0 == 0) m = nxt;
        reg[E - 1 - u] = cmul(reg[E - 1 - u], m);
        cur = nxt;
      }
    }
    fft_sel<M, true, false, V, TREG>(reg, lds, j0, tw, treg);
    group_sync<M>();
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int y = j0 + P * t;
      if (y >= out_lo && y < out_hi) lds_in[y] = reg[t];
    }
    __syncthreads();
    float2* sp = a.spec + static_cast<size_t>(w) * N * M + kx0 + cc;
    if constexpr (FULL) {
#pragma unroll
      for (int k = 0; k < EN; ++k) sp[static_cast<size_t>(yy + k * P) * M] = stg[yy + k * P];
    } else {
      for (int y = out_lo + yy; y < out_hi; y += P) sp[static_cast<size_t>(y) * M] = stg[y];
    }
    if constexpr (STAGE_AFTER_STORE) {
      if (w + 1 < we) stage();
    } else {
      __syncthreads();  // the next wavelength's staging overwrites the tile
    }
  }
}

template <int M, int PAD, bool CONJ, int TX, int HM, bool FULL, int V = 0>
__global__ void __launch_bounds__(TX * Geo<M>::P) __attribute__((amdgpu_waves_per_eu(4)))
col_kernel(ColArgs a) {
  __shared__ float2 tile[TX * Geo<M>::COL_REGION];
  __shared__ float2 tw[twiddle_count<M, V>()];
  int bx, by;
  col_block_item(static_cast<int>(blockIdx.x + gridDim.x * blockIdx.y), static_cast<int>(gridDim.x * gridDim.y),
                 static_cast<int>(gridDim.x), bx, by);
  col_body<M, PAD, CONJ, TX, HM, FULL, V>(a, bx, by, tile, tw);
}

// One launch of a column pass for several designs of the same transform length (see
// row_group_kernel); every task starts at a multiple of 16 blocks.
template <int M, int PAD, bool CONJ, int TX, int HM, bool FULL>
__global__ void __launch_bounds__(TX * Geo<M>::P) __attribute__((amdgpu_waves_per_eu(4)))
col_group_kernel(GroupArgs g) {
  __shared__ float2 tile[TX * Geo<M>::COL_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  const int ti = group_task(g, blockIdx.x);
  const ColTask& t = static_cast<const ColTask*>(g.tasks)[ti];
  const int local = static_cast<int>(blockIdx.x) - g.block0[ti];
  if (local >= t.nblocks) return;
  const ColArgs a = t.a;
  int bx, by;
  col_block_item(local, t.nblocks, t.gx, bx, by);
  col_body<M, PAD, CONJ, TX, HM, FULL>(a, bx, by, tile, tw);
}

// H / M^2 of one gap for every wavelength on the quarter plane |kx|, |ky| <= M/2 (H depends on
// kx^2 + ky^2 only); block (|kx|, w), threads over |ky|.
template <int M>
__global__ void __launch_bounds__(256) transfer_table_kernel(const WlConst* __restrict__ wl, double zrev,
                                                             float2* __restrict__ out) {
  constexpr int HS = M / 2 + 1;
  const int kx = blockIdx.x;
  const int w = blockIdx.y;
  const double base = wl[w].q0 - static_cast<double>(kx * kx);
  float2* row = out + (static_cast<size_t>(w) * HS + kx) * HS;
  for (int ky = threadIdx.x; ky < HS; ky += blockDim.x) row[ky] = transfer<M, false>(zrev, base, ky);
}

// ------------------------------------------------------------------------------------------
// Column pass as two complex matrix products on the FP32 matrix cores (v_mfma_f32_16x16x4_f32):
//   Z = F S            F[ky][y] = exp(-2 pi i ky y / M)  (M x N, shared by every wavelength)
//   Z <- H . Z / M^2   (transfer function on the fly, as in the transform kernels)
//   Out = F^H Z        (N x M, keeps the aperture rows)
// for a tile of 16 columns of one wavelength.  S and Z live in LDS as separate real and
// imaginary planes; the DFT matrix is read from a table built on the host in double
// precision: FT[y][ky] (step 1, lanes read 16 consecutive ky) and F[ky][y] (step 3).
// Operand layout of the 16x16x4 instruction: lane l holds A[l%16][l/16], B[l/16][l%16] and
// D[4(l/16)+r][l%16], r = 0..3.
// ------------------------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 16;
// threads per block: the LDS tiles of long transforms allow one block per CU, so those get
// eight wavefronts to keep two per SIMD
constexpr int gemm_threads(int M) { return M >= 256 ? 512 : 256; }

template <int M, int PAD, bool CONJ>
__global__ void __launch_bounds__(gemm_threads(M)) colgemm_kernel(ColArgs a, const float2* __restrict__ dft) {
  constexpr int N = M / PAD;
  constexpr int TN = kGemmTile;
  constexpr int kGemmThreads = gemm_threads(M);
  constexpr int WAVES = kGemmThreads / 64;
  __shared__ float sr[N * TN], si[N * TN];
  __shared__ float zr[M * TN], zi[M * TN];
  const float2* __restrict__ FT = dft;           // [N][M]
  const float2* __restrict__ F = dft + M * N;    // [M][N]

  const int kx0 = blockIdx.x * TN;
  float2* spec = a.spec + static_cast<size_t>(blockIdx.y) * N * M;
  const WlConst c = a.wl[a.w_begin + blockIdx.y];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  // stage rows [in_lo, in_hi) of the 16 columns (zeros elsewhere)
  for (int i = tid; i < N * TN; i += kGemmThreads) {
    const int y = i / TN, cc = i % TN;
    float2 v = make_float2(0.f, 0.f);
    if (y >= a.in_lo && y < a.in_hi) v = spec[static_cast<size_t>(y) * M + kx0 + cc];
    sr[i] = v.x;
    si[i] = v.y;
  }
  __syncthreads();

  // step 1: Z = F S, K = N.  A wave takes its row tiles of ky two at a time, so four
  // accumulator chains are in flight on the matrix core and the S operand is read once per
  // k step for both.
  {
    const int kx = kx0 + lr;
    const int kxs = kx < M / 2 ? kx : kx - M;
    const double base = c.q0 - static_cast<double>(kxs * kxs);
    for (int t0 = wave; t0 < M / 16; t0 += 2 * WAVES) {
      const int t1 = t0 + WAVES;
      const bool two = t1 < M / 16;
      v4f re0 = {0.f, 0.f, 0.f, 0.f}, im0 = re0, re1 = re0, im1 = re0;
#pragma unroll 4
      for (int k0 = 0; k0 < N; k0 += 4) {
        const float br = sr[(k0 + lk) * TN + lr], bi = si[(k0 + lk) * TN + lr];
        const float2 f0 = FT[(k0 + lk) * M + t0 * 16 + lr];
        re0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.x, br, re0, 0, 0, 0);
        re0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-f0.y, bi, re0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.x, bi, im0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.y, br, im0, 0, 0, 0);
        if (two) {
          const float2 f1 = FT[(k0 + lk) * M + t1 * 16 + lr];
          re1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.x, br, re1, 0, 0, 0);
          re1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-f1.y, bi, re1, 0, 0, 0);
          im1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.x, bi, im1, 0, 0, 0);
          im1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.y, br, im1, 0, 0, 0);
        }
      }
      // H at (kx0 + lr, ky0 + 4 lk + r)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int ky = t0 * 16 + 4 * lk + r;
        float2 z = cmul(make_float2(re0[r], im0[r]), transfer<M, CONJ>(a.zrev, base, ky));
        zr[ky * TN + lr] = z.x;
        zi[ky * TN + lr] = z.y;
        if (two) {
          ky = t1 * 16 + 4 * lk + r;
          z = cmul(make_float2(re1[r], im1[r]), transfer<M, CONJ>(a.zrev, base, ky));
          zr[ky * TN + lr] = z.x;
          zi[ky * TN + lr] = z.y;
        }
      }
    }
  }
  __syncthreads();

  // step 3: Out = F^H Z for the kept rows, K = M, two row tiles of y at a time
  for (int t0 = wave; t0 < N / 16; t0 += 2 * WAVES) {
    const int t1 = t0 + WAVES;
    const bool use0 = t0 * 16 < a.out_hi && t0 * 16 + 16 > a.out_lo;
    const bool use1 = t1 < N / 16 && t1 * 16 < a.out_hi && t1 * 16 + 16 > a.out_lo;
    if (!use0 && !use1) continue;
    v4f re0 = {0.f, 0.f, 0.f, 0.f}, im0 = re0, re1 = re0, im1 = re0;
#pragma unroll 4
    for (int k0 = 0; k0 < M; k0 += 4) {
      const float br = zr[(k0 + lk) * TN + lr], bi = zi[(k0 + lk) * TN + lr];
      // A[y][ky] = conj(F[ky][y]): lane (lr, lk) needs y = y0 + lr, ky = k0 + lk
      if (use0) {
        const float2 f0 = F[(k0 + lk) * N + t0 * 16 + lr];
        re0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.x, br, re0, 0, 0, 0);
        re0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.y, bi, re0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f0.x, bi, im0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_16x16x4f32(-f0.y, br, im0, 0, 0, 0);
      }
      if (use1) {
        const float2 f1 = F[(k0 + lk) * N + t1 * 16 + lr];
        re1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.x, br, re1, 0, 0, 0);
        re1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.y, bi, re1, 0, 0, 0);
        im1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f1.x, bi, im1, 0, 0, 0);
        im1 = __builtin_amdgcn_mfma_f32_16x16x4f32(-f1.y, br, im1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int y = t0 * 16 + 4 * lk + r;
      if (use0 && y >= a.out_lo && y < a.out_hi)
        spec[static_cast<size_t>(y) * M + kx0 + lr] = make_float2(re0[r], im0[r]);
      y = t1 * 16 + 4 * lk + r;
      if (use1 && y >= a.out_lo && y < a.out_hi)
        spec[static_cast<size_t>(y) * M + kx0 + lr] = make_float2(re1[r], im1[r]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// LDS-resident path for short transforms.  A block owns one wavelength.  Its N aperture rows
// live in LDS with a row stride equal to a row transform's exchange region, so every row
// transforms in place; a batch of CB columns at a time gathers its column from the rows and
// exchanges through regions of its own.  Every step is the one the multi-kernel path takes
// (same transforms, transmission, transfer function, products, partial-sum order), so the
// results are the same bits.
// ------------------------------------------------------------------------------------------
template <int M, int PAD>
struct LdsGeo {
  static constexpr int N = M / PAD;
  static constexpr int P = Geo<M>::P;
  static constexpr int RS = Geo<M>::ROW_REGION;               // row stride of the plane
  static constexpr int CS = Geo<M>::COL_REGION;               // column exchange region
  static constexpr int RB = kLdsThreads / P;                  // rows transformed at once
  static constexpr int CB = RB < M ? RB : M;                  // columns transformed at once
  static constexpr long long LDS_BYTES = 8LL * (static_cast<long long>(N) * RS + CB * CS + twiddle_count<M>());
  static constexpr bool FITS = LDS_BYTES <= 160 * 1024;
  // the forward's window field (F <= N) is staged in the column regions for the binning
  static_assert(M > 128 || !FITS || static_cast<long long>(CB) * CS >= static_cast<long long>(N) * N,
                "window staging");
};

// forward rows of one layer: FIRST = input field times t_0, else inverse row transform of the
// plane row, crop, times t_layer; checkpoint; zero-padded forward row transform in place
template <int M, int PAD, bool FIRST>
__device__ __forceinline__ void lds_rows_forward(const LdsArgs& a, const WlConst& c, int w, int layer,
                                                 float2* plane, const float2* tw) {
  using G = LdsGeo<M, PAD>;
  constexpr int E = Geo<M>::E, P = G::P, N = G::N, EN = E / PAD;
  constexpr bool HALF = (PAD == 2);
  const int g = threadIdx.x / P, j0 = threadIdx.x % P;
  const size_t nn = static_cast<size_t>(N) * N;
  for (int y = g; y < N; y += G::RB) {
    float2* row = plane + y * G::RS;
    const float* hrow = a.h + (static_cast<size_t>(layer) * N + y) * N;
    float2 reg[E];
    if constexpr (FIRST) {
#pragma unroll
      for (int t = 0; t < EN; ++t) {
        const float2 u = a.u_in ? a.u_in[static_cast<size_t>(y) * N + j0 + P * t] : make_float2(1.f, 0.f);
        reg[t] = cmul(u, transmission(hrow[j0 + P * t], c));
      }
    } else {
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false>(reg, row, j0, tw);
#pragma unroll
      for (int t = 0; t < EN; ++t) reg[t] = cmul(reg[t], transmission(hrow[j0 + P * t], c));
    }
    float2* ck = a.ckpt + (static_cast<size_t>(layer) * a.W + w) * nn + static_cast<size_t>(y) * N;
#pragma unroll
    for (int t = 0; t < EN; ++t) ck[j0 + P * t] = reg[t];
    fft<M, false, HALF>(reg, row, j0, tw);
#pragma unroll
    for (int t = 0; t < E; ++t) row[j0 + P * t] = reg[t];
  }
}

// column transforms of one gap: rows [in_lo, in_hi) in, H or conj(H), rows [0, N) back
template <int M, int PAD, bool CONJ>
__device__ __forceinline__ void lds_columns(const WlConst& c, double zrev, int in_lo, int in_hi,
                                            float2* plane, float2* xch, const float2* tw) {
  using G = LdsGeo<M, PAD>;
  constexpr int E = Geo<M>::E, P = G::P, N = G::N, EN = E / PAD;
  constexpr bool HALF = (PAD == 2);
  const int g = threadIdx.x / P, j0 = threadIdx.x % P;
  if (g >= G::CB) return;
  float2* xr = xch + g * G::CS;
  for (int kx = g; kx < M; kx += G::CB) {
    float2 reg[E];
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int y = j0 + P * t;
      reg[t] = (y >= in_lo && y < in_hi) ? plane[y * G::RS + kx] : make_float2(0.f, 0.f);
    }
    fft<M, false, HALF>(reg, xr, j0, tw);
    const int kxs = kx < M / 2 ? kx : kx - M;
    const double base = c.q0 - static_cast<double>(kxs * kxs);
#pragma unroll
    for (int t = 0; t < E; ++t) reg[t] = cmul(reg[t], transfer<M, CONJ>(zrev, base, j0 + P * t));
    fft<M, true, false>(reg, xr, j0, tw);
#pragma unroll
    for (int t = 0; t < EN; ++t) plane[(j0 + P * t) * G::RS + kx] = reg[t];
  }
}

template <int M, int PAD>
__global__ void __launch_bounds__(kLdsThreads) lds_forward_kernel(LdsArgs a) {
  using G = LdsGeo<M, PAD>;
  constexpr int E = Geo<M>::E, P = G::P, N = G::N, EN = E / PAD;
  __shared__ float2 plane[N * G::RS];
  __shared__ float2 xch[G::CB * G::CS];
  __shared__ float2 tw[twiddle_count<M>()];
  stage_twiddles<M>(tw, a.tw, threadIdx.x, kLdsThreads);
  __syncthreads();
  const int w = blockIdx.x;
  const WlConst c = a.wl[w];
  lds_rows_forward<M, PAD, true>(a, c, w, 0, plane, tw);
  __syncthreads();
  for (int l = 0; l < a.K; ++l) {
    lds_columns<M, PAD, false>(c, a.zrev[l], 0, N, plane, xch, tw);
    __syncthreads();
    if (l + 1 < a.K) {
      lds_rows_forward<M, PAD, false>(a, c, w, l + 1, plane, tw);
      __syncthreads();
    }
  }
  // last inverse row transforms on the window rows: output field, and its intensity in bins
  const int F = a.fov, x0 = (N - F) / 2, T = F / a.bin;
  const int g = threadIdx.x / P, j0 = threadIdx.x % P;
  float2* win = xch;  // the column regions are free now
  for (int y = x0 + g; y < x0 + F; y += G::RB) {
    float2* row = plane + y * G::RS;
    float2 reg[E];
#pragma unroll
    for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
    fft<M, true, false>(reg, row, j0, tw);
    float2* dst = a.ofov + static_cast<size_t>(w) * F * F + static_cast<size_t>(y - x0) * F;
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int x = j0 + P * t;
      if (x >= x0 && x < x0 + F) {
        dst[x - x0] = reg[t];
        win[(y - x0) * F + x - x0] = reg[t];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < T * T; i += kLdsThreads)
    bin_intensity_body(win, a.intensity + static_cast<size_t>(w) * T * T, 1, F, a.bin, i);
}

template <int M, int PAD>
__global__ void __launch_bounds__(kLdsThreads) lds_adjoint_kernel(LdsArgs a) {
  using G = LdsGeo<M, PAD>;
  constexpr int E = Geo<M>::E, P = G::P, N = G::N, EN = E / PAD;
  constexpr bool HALF = (PAD == 2);
  __shared__ float2 plane[N * G::RS];
  __shared__ float2 xch[G::CB * G::CS];
  __shared__ float2 tw[twiddle_count<M>()];
  stage_twiddles<M>(tw, a.tw, threadIdx.x, kLdsThreads);
  __syncthreads();
  const int w = blockIdx.x;
  const WlConst c = a.wl[w];
  const int F = a.fov, b = a.bin, T = F / b, x0 = (N - F) / 2;
  const int g = threadIdx.x / P, j0 = threadIdx.x % P;
  const size_t nn = static_cast<size_t>(N) * N;
  // seed 2 (dL/dI) o on the window rows, forward row transform
  for (int y = x0 + g; y < x0 + F; y += G::RB) {
    float2* row = plane + y * G::RS;
    const float2* o = a.ofov + static_cast<size_t>(w) * F * F + static_cast<size_t>(y - x0) * F;
    const float* d = a.dl_di + static_cast<size_t>(w) * T * T + static_cast<size_t>((y - x0) / b) * T;
    float2 reg[E];
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int x = j0 + P * t;
      if (x >= x0 && x < x0 + F) {
        const float s = 2.0f * d[(x - x0) / b];
        reg[t] = cscale(o[x - x0], s);
      } else {
        reg[t] = make_float2(0.f, 0.f);
      }
    }
    fft<M, false, HALF>(reg, row, j0, tw);
#pragma unroll
    for (int t = 0; t < E; ++t) row[j0 + P * t] = reg[t];
  }
  __syncthreads();
  const float ct = static_cast<float>(c.ct), ca = static_cast<float>(c.ca);
  for (int l = a.K - 1; l >= 0; --l) {
    lds_columns<M, PAD, true>(c, a.zrev[l], l == a.K - 1 ? x0 : 0, l == a.K - 1 ? x0 + F : N, plane, xch, tw);
    __syncthreads();
    for (int y = g; y < N; y += G::RB) {
      float2* row = plane + y * G::RS;
      const float* hrow = a.h + (static_cast<size_t>(l) * N + y) * N;
      const float2* ck = a.ckpt + (static_cast<size_t>(l) * a.W + w) * nn + static_cast<size_t>(y) * N;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false>(reg, row, j0, tw);
      float* dst = a.dh_part + (static_cast<size_t>(w) * a.K + l) * nn + static_cast<size_t>(y) * N;
#pragma unroll
      for (int t = 0; t < EN; ++t) {
        const float2 gv = reg[t];
        const float2 v = ck[j0 + P * t];
        // conj(g) v; -ct Im - ca Re
        const float re = fmaf(gv.x, v.x, gv.y * v.y);
        const float im = fmaf(gv.x, v.y, -(gv.y * v.x));
        dst[j0 + P * t] = fmaf(-ct, im, fmaf(-ca, re, 0.f));
        if (l > 0) reg[t] = cmulc(gv, transmission(hrow[j0 + P * t], c));
      }
      if (l > 0) {
        fft<M, false, HALF>(reg, row, j0, tw);
#pragma unroll
        for (int t = 0; t < E; ++t) row[j0 + P * t] = reg[t];
      }
    }
    __syncthreads();
  }
}

}  // namespace dpx
