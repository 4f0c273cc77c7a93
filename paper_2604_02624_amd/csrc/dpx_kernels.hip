// HIP kernels for gfx950: row passes, column passes, intensity binning, loss, reductions.
//
// One propagation over a gap (Section 4, Eq. 4/5 via the angular spectrum) is split in two
// passes over a [N rows][M columns] complex plane per wavelength ("spec"):
//   row pass    : transform along x (the N non-zero rows of the zero-padded plane only)
//   column pass : transform along y, multiply by the transfer function, inverse along y,
//                 keep the N aperture rows
// and the next row pass starts with the inverse transform along x.  Zero padding is placed
// at the high end of each axis instead of centring it: a circular convolution commutes with
// shifts, so cropping the same corner returns the same N x N field.
#include <cmath>
#include <vector>

#include "dpx_internal.hpp"
#include "fft.hpp"
#include "phase.hpp"

namespace dpx {

// Eq. 1 with the +j reading: t = exp(-ca h) exp(+i 2 pi rt h); phase argument in double.
// Word 3 of a raw buffer resource on gfx9: 32-bit data format, no stride or swizzle.
constexpr int kBufferRsrcWord3 = 0x00020000;

// One 8-byte load through a buffer resource: byte offset = voff (per lane) + soff (scalar).
__device__ __forceinline__ float2 buffer_load_c64(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

__device__ __forceinline__ float2 transmission(float h, const WlConst& c) {
  const double hd = static_cast<double>(h);
  float2 t = cis_turns(c.rt * hd);
  if (c.ca != 0.0) {
    const float a = expf(-static_cast<float>(c.ca * hd));
    t.x *= a;
    t.y *= a;
  }
  return t;
}

// Threads per row-pass block: 512 (eight transforms of 1024) where the registers allow two
// such blocks per CU next to their LDS, 256 for the register-heavy adjoint middle pass.
constexpr int row_threads_of_mode(int mode) { return mode == ROW_ADJ_MID ? 256 : 512; }
template <int M, int MODE>
constexpr int row_block_threads() { return row_threads_of_mode(MODE); }

// ------------------------------------------------------------------------------------------
// Row pass.  A block owns G = 256 / P consecutive rows (one transform group per row) and
// loops over a run of wavelengths, so the row's heights stay in registers.
// ------------------------------------------------------------------------------------------
// Block (bx, by) of a row pass: rows row_lo + bx G .. + G - 1, wavelength block by.
// lds_all: G exchange regions; tw: room for the twiddle table (both in LDS).
template <int M, int PAD, int MODE>
__device__ __forceinline__ void row_body(const RowArgs& a, int bx, int by, float2* lds_all, float2* tw) {
  constexpr int kRowThreads = row_block_threads<M, MODE>();
  constexpr int E = Geo<M>::E;
  constexpr int P = Geo<M>::P;
  constexpr int G = kRowThreads / P;
  constexpr int EN = E / PAD;  // registers that hold x < N
  constexpr bool HALF = (PAD == 2);
  constexpr int RG = Geo<M>::ROW_REGION;
  stage_twiddles<M>(tw, a.tw, threadIdx.x, kRowThreads);
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
                MODE == ROW_ADJ_LAST) {
#pragma unroll
    for (int t = 0; t < EN; ++t) hreg[t] = a.h[static_cast<size_t>(y) * N + j0 + P * t];
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
#pragma unroll
      for (int t = 0; t < EN; ++t) reg[t] = cmul(uin[t], transmission(hreg[t], c));
      if (a.store_ckpt && active) {
        float2* ck = a.ckpt + (static_cast<size_t>(a.layer) * a.ckpt_w_stride + wc) * nn +
                     static_cast<size_t>(y) * N;
#pragma unroll
        for (int t = 0; t < EN; ++t) ck[j0 + P * t] = reg[t];
      }
      fft<M, false, HALF>(reg, lds, j0, tw);
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
      fft<M, true, false>(reg, lds, j0, tw);
#pragma unroll
      for (int t = 0; t < EN; ++t) reg[t] = cmul(reg[t], transmission(hreg[t], c));
      if (a.store_ckpt && active) {
        float2* ck = a.ckpt + (static_cast<size_t>(a.layer) * a.ckpt_w_stride + wc) * nn +
                     static_cast<size_t>(y) * N;
#pragma unroll
        for (int t = 0; t < EN; ++t) ck[j0 + P * t] = reg[t];
      }
      fft<M, false, HALF>(reg, lds, j0, tw);
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
      fft<M, true, false>(reg, lds, j0, tw);
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
      fft<M, false, HALF>(reg, lds, j0, tw);
      if (active) {
        float2* dst = a.spec + wc * plane + static_cast<size_t>(y) * M;
#pragma unroll
        for (int t = 0; t < E; ++t) dst[j0 + P * t] = reg[t];
      }
    }
  } else {  // ROW_ADJ_MID, ROW_ADJ_LAST
    float acc[EN];
#pragma unroll
    for (int t = 0; t < EN; ++t) acc[t] = 0.f;
    for (int w = wb; w < we; ++w) {
      const WlConst c = a.wl[w];
      const int wc = w - a.w_begin;
      float2* row = a.spec + wc * plane + static_cast<size_t>(y) * M;
      const float2* ck = a.ckpt + (static_cast<size_t>(a.layer) * a.ckpt_w_stride + wc) * nn +
                         static_cast<size_t>(y) * N;
      float2 reg[E];
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = row[j0 + P * t];
      fft<M, true, false>(reg, lds, j0, tw);
      const float ct = static_cast<float>(c.ct);
      const float ca = static_cast<float>(c.ca);
#pragma unroll
      for (int t = 0; t < EN; ++t) {
        const float2 gv = reg[t];
        const float2 v = ck[j0 + P * t];
        // conj(g) v; acc += -ct Im - ca Re
        const float re = fmaf(gv.x, v.x, gv.y * v.y);
        const float im = fmaf(gv.x, v.y, -(gv.y * v.x));
        acc[t] = fmaf(-ct, im, fmaf(-ca, re, acc[t]));
        if constexpr (MODE == ROW_ADJ_MID) reg[t] = cmulc(gv, transmission(hreg[t], c));
      }
      if constexpr (MODE == ROW_ADJ_MID) {
        fft<M, false, HALF>(reg, lds, j0, tw);
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

template <int M, int PAD, int MODE>
__global__ void __launch_bounds__(row_threads_of_mode(MODE)) row_kernel(RowArgs a) {
  __shared__ float2 lds_all[row_block_threads<M, MODE>() / Geo<M>::P * Geo<M>::ROW_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  row_body<M, PAD, MODE>(a, blockIdx.x, blockIdx.y, lds_all, tw);
}

// Task of a grouped launch that block b belongs to: the last task whose first block is <= b
// (the table of first blocks is a kernel argument, so the search runs on scalar loads).
__device__ __forceinline__ int group_task(const GroupArgs& g, int b) {
  int lo = 0, hi = g.ntasks;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g.block0[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One launch of a row pass for several designs of the same transform length and mode: each
// block finds its design's task, patches the per-call buffers into the design's arguments
// and runs the same body as the single-design kernel.
template <int M, int PAD, int MODE>
__global__ void __launch_bounds__(row_threads_of_mode(MODE)) row_group_kernel(GroupArgs g) {
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

// H(kx, ky) / M^2 with the conjugate for the adjoint; 0 outside the propagating disc
template <int M, bool CONJ>
__device__ __forceinline__ float2 transfer(double zrev, double base, int ky) {
  const int kys = ky < M / 2 ? ky : ky - M;
  const double q = base - static_cast<double>(kys * kys);
  const float2 hh = cis_turns<M * M>(zrev * sqrt_pos(q > 0.0 ? q : 1.0));
  return q > 0.0 ? (CONJ ? conjf2(hh) : hh) : make_float2(0.f, 0.f);
}

// ------------------------------------------------------------------------------------------
// Column pass.  A block owns TX adjacent columns of one wavelength's plane: it stages the
// [rows][TX] tile through LDS (coalesced 8*TX-byte row segments), each transform group
// then runs forward FFT -> transfer function -> inverse FFT on its column in registers, and
// the kept rows go back through the same LDS tile.
// ------------------------------------------------------------------------------------------
// Block (bx, by) of a column pass: column tile bx of gx, wavelength block by.  The blocks of
// one pass are numbered bx + gx by from a multiple of 16 in launch order.
template <int M, int PAD, bool CONJ, int TX, bool MIRROR>
__device__ __forceinline__ void col_body(const ColArgs& a, int bx, int by, int gx, float2* tile, float2* tw) {
  constexpr int E = Geo<M>::E;
  constexpr int P = Geo<M>::P;
  constexpr int NT = TX * P;
  constexpr int LD = Geo<M>::COL_REGION;  // one column's staging rows / exchange region
  constexpr int EN = E / PAD;
  constexpr bool HALF = (PAD == 2);
  static_assert(NT / TX == P, "staging rows per pass");

  const int N = M / PAD;
  // XCD-aware tile order: consecutive blocks go to the eight XCDs in turn, so blocks b and
  // b + 8 of every run of 16 share an XCD and its L2; giving them neighbouring column tiles
  // lets the two halves of each 128-byte row segment meet in the same L2.
  int tile_x = bx;
  if ((gx & 15) == 0) {
    const int r = tile_x & 15;
    tile_x = (tile_x & ~15) + ((r & 7) << 1) + (r >> 3);
  }
  const int kx0 = tile_x * TX;
  const int cc = threadIdx.x % TX;
  const int yy = threadIdx.x / TX;
  const int g = threadIdx.x / P;
  const int j0 = threadIdx.x % P;
  float2* lds = tile + g * LD;
  const int kx = kx0 + g;
  const int kxs = kx < M / 2 ? kx : kx - M;

  // The block runs a.col_wpb wavelengths.  With zero padding the staged rows of the next one
  // are loaded into registers while the current one is transformed, so their latency is
  // hidden; without it those registers would not fit next to the full-length transform and
  // the rows go straight to LDS.  Row k of a lane is one buffer load at the lane's 32-bit
  // byte offset plus the scalar offset k P M 8, so no per-row address stays live.
  constexpr bool PREFETCH = HALF;
  const int wb = by * a.col_wpb;
  const int we = min(wb + a.col_wpb, a.w_count);
  const unsigned voff = static_cast<unsigned>(((a.in_lo + yy) * M + kx0 + cc) * 8);
  auto plane = [&](int w) {
    return __builtin_amdgcn_make_buffer_rsrc(a.spec + static_cast<size_t>(w) * N * M, 0,
                                             N * M * 8, kBufferRsrcWord3);
  };
  float2 pre[PREFETCH ? EN : 1];
  auto fetch = [&](int w) {
    const auto rs = plane(w);
#pragma unroll
    for (int k = 0; k < EN; ++k) {
      const int y = a.in_lo + yy + k * P;
      pre[PREFETCH ? k : 0] = (y < a.in_hi) ? buffer_load_c64(rs, voff, k * P * M * 8) : make_float2(0.f, 0.f);
      if constexpr (!PREFETCH) {
        if (y < a.in_hi) tile[cc * LD + y] = pre[0];
      }
    }
  };
  if constexpr (PREFETCH) fetch(wb);
  stage_twiddles<M>(tw, a.tw, threadIdx.x, NT);

  for (int w = wb; w < we; ++w) {
    if constexpr (PREFETCH) {
#pragma unroll
      for (int k = 0; k < EN; ++k) {
        const int y = a.in_lo + yy + k * P;
        if (y < a.in_hi) tile[cc * LD + y] = pre[k];
      }
    } else {
      fetch(w);
    }
    __syncthreads();
    if constexpr (PREFETCH) {
      if (w + 1 < we) fetch(w + 1);
    }

    const WlConst c = a.wl[a.w_begin + w];
    float2 reg[E];
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int y = j0 + P * t;
      reg[t] = (y >= a.in_lo && y < a.in_hi) ? lds[y] : make_float2(0.f, 0.f);
    }
    wave_sync();
    fft<M, false, HALF>(reg, lds, j0, tw);

    // transfer function H = exp(+i 2 pi z sqrt(q)) / M^2 on the propagating disc, else 0.
    const double base = c.q0 - static_cast<double>(kxs * kxs);
    if constexpr (MIRROR) {
      // H depends on ky^2 only: lane j0 holds ky = j0 + P t, and for t >= E/2 the row M - ky
      // is register E-1-t of lane P - j0 (lane 0 mirrors onto its own register E - t), so
      // each lane evaluates E/2 + 1 rows and fetches the others across lanes.  Streamed so
      // that only two evaluations are live at a time: step u applies row u and the mirrored
      // row E-1-u (whose value lane 0 takes from its own evaluation u+1).
      constexpr int EH = E / 2;
      const int lane = threadIdx.x & 63;
      const int src = ((lane - j0) + ((P - j0) & (P - 1))) << 2;
      float2 cur = transfer<M, CONJ>(a.zrev, base, j0);
#pragma unroll
      for (int u = 0; u < EH; ++u) {
        const float2 nxt = transfer<M, CONJ>(a.zrev, base, j0 + P * (u + 1));
        reg[u] = cmul(reg[u], cur);
        float2 m;
        m.x = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(cur.x)));
        m.y = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(cur.y)));
        if (j0 == 0) m = nxt;
        reg[E - 1 - u] = cmul(reg[E - 1 - u], m);
        cur = nxt;
      }
    } else {
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = cmul(reg[t], transfer<M, CONJ>(a.zrev, base, j0 + P * t));
    }
    fft<M, true, false>(reg, lds, j0, tw);
    wave_sync();
#pragma unroll
    for (int t = 0; t < EN; ++t) {
      const int y = j0 + P * t;
      if (y >= a.out_lo && y < a.out_hi) lds[y] = reg[t];
    }
    __syncthreads();
    float2* sp = a.spec + static_cast<size_t>(w) * N * M + kx0 + cc;
    for (int y = a.out_lo + yy; y < a.out_hi; y += P) sp[static_cast<size_t>(y) * M] = tile[cc * LD + y];
    __syncthreads();  // the next wavelength's staging overwrites the tile
  }
}

template <int M, int PAD, bool CONJ, int TX, bool MIRROR>
__global__ void __launch_bounds__(TX * Geo<M>::P) __attribute__((amdgpu_waves_per_eu(4)))
col_kernel(ColArgs a) {
  __shared__ float2 tile[TX * Geo<M>::COL_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  col_body<M, PAD, CONJ, TX, MIRROR>(a, blockIdx.x, blockIdx.y, gridDim.x, tile, tw);
}

// One launch of a column pass for several designs of the same transform length (see
// row_group_kernel); every task starts at a multiple of 16 blocks.
template <int M, int PAD, bool CONJ, int TX, bool MIRROR>
__global__ void __launch_bounds__(TX * Geo<M>::P) __attribute__((amdgpu_waves_per_eu(4)))
col_group_kernel(GroupArgs g) {
  __shared__ float2 tile[TX * Geo<M>::COL_REGION];
  __shared__ float2 tw[twiddle_count<M>()];
  const int ti = group_task(g, blockIdx.x);
  const ColTask& t = static_cast<const ColTask*>(g.tasks)[ti];
  const int local = static_cast<int>(blockIdx.x) - g.block0[ti];
  if (local >= t.nblocks) return;
  const ColArgs a = t.a;
  col_body<M, PAD, CONJ, TX, MIRROR>(a, local % t.gx, local / t.gx, t.gx, tile, tw);
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
// Small kernels
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void bin_intensity_body(const float2* __restrict__ ofov, float* __restrict__ out,
                                                   int w_count, int fov, int bin, size_t i) {
  const int T = fov / bin;
  const size_t total = static_cast<size_t>(w_count) * T * T;
  if (i >= total) return;
  const int w = static_cast<int>(i / (static_cast<size_t>(T) * T));
  const int r = static_cast<int>(i % (static_cast<size_t>(T) * T));
  const int ty = r / T, tx = r % T;
  const float2* o = ofov + static_cast<size_t>(w) * fov * fov;
  float s = 0.f;
  for (int a = 0; a < bin; ++a)
    for (int b = 0; b < bin; ++b) {
      const float2 v = o[static_cast<size_t>(ty * bin + a) * fov + tx * bin + b];
      s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
    }
  out[i] = s;
}

__global__ void bin_intensity_kernel(const float2* __restrict__ ofov, float* __restrict__ out,
                                     int w_count, int fov, int bin) {
  bin_intensity_body(ofov, out, w_count, fov, bin, static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// grouped: task = one design's window fields -> its intensities in the packed output
__global__ void bin_group_kernel(GroupArgs g, float* __restrict__ out) {
  const int ti = group_task(g, blockIdx.x);
  const BinTask& t = static_cast<const BinTask*>(g.tasks)[ti];
  const int local = static_cast<int>(blockIdx.x) - g.block0[ti];
  bin_intensity_body(t.ofov, out + t.img_off, t.w_count, t.fov, t.bin,
                     static_cast<size_t>(local) * blockDim.x + threadIdx.x);
}

constexpr int kLossThreads = 256;

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kLossThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One block per wavelength w: sums in double in a fixed tree order (bitwise reproducible).
__device__ __forceinline__ void loss_body(const float* __restrict__ I, const float* __restrict__ tau,
                                          float* __restrict__ dl_di, double* __restrict__ per_wl,
                                          int W, int T, int w, double* sh) {
  const int P = T * T;
  const float* Iw = I + static_cast<size_t>(w) * P;
  const float* tw = tau + static_cast<size_t>(w) * P;
  double si = 0.0, st = 0.0;
  for (int p = threadIdx.x; p < P; p += kLossThreads) {
    si += Iw[p];
    st += tw[p];
  }
  const double S = block_sum(si, sh);
  const double St = block_sum(st, sh);
  const double rS = S > 0.0 ? 1.0 / S : 0.0;
  const double rSt = St > 0.0 ? 1.0 / St : 0.0;
  double sd2 = 0.0, sdi = 0.0;
  for (int p = threadIdx.x; p < P; p += kLossThreads) {
    const double ih = Iw[p] * rS;
    const double d = ih - tw[p] * rSt;
    sd2 += d * d;
    sdi += d * ih;
  }
  const double D2 = block_sum(sd2, sh);
  const double inner = block_sum(sdi, sh);
  if (threadIdx.x == 0) per_wl[w] = D2 / P;
  if (dl_di) {
    const double k = 2.0 * rS / (static_cast<double>(W) * P);
    float* gw = dl_di + static_cast<size_t>(w) * P;
    for (int p = threadIdx.x; p < P; p += kLossThreads) {
      const double ih = Iw[p] * rS;
      const double d = ih - tw[p] * rSt;
      gw[p] = static_cast<float>(k * (d - inner));
    }
  }
}

__global__ void __launch_bounds__(kLossThreads)
loss_kernel(const float* __restrict__ I, const float* __restrict__ tau, float* __restrict__ dl_di,
            double* __restrict__ per_wl, int W, int T) {
  __shared__ double sh[kLossThreads];
  loss_body(I, tau, dl_di, per_wl, W, T, blockIdx.x, sh);
}

// grouped: task = one design, one block per wavelength of every design
__global__ void __launch_bounds__(kLossThreads)
loss_group_kernel(GroupArgs g, const float* __restrict__ I, const float* __restrict__ tau,
                  float* __restrict__ dl_di) {
  __shared__ double sh[kLossThreads];
  const int ti = group_task(g, blockIdx.x);
  const LossTask& t = static_cast<const LossTask*>(g.tasks)[ti];
  const int w = static_cast<int>(blockIdx.x) - g.block0[ti];
  loss_body(I + t.img_off, tau + t.img_off, dl_di ? dl_di + t.img_off : nullptr, t.per_wl, t.W, t.T, w, sh);
}

__device__ __forceinline__ void loss_sum_body(const double* __restrict__ per_wl, double* __restrict__ loss,
                                              int W, double* sh) {
  double s = 0.0;
  for (int w = threadIdx.x; w < W; w += kLossThreads) s += per_wl[w];
  const double tot = block_sum(s, sh);
  if (threadIdx.x == 0) *loss = tot / W;
}

__global__ void __launch_bounds__(kLossThreads)
loss_sum_kernel(const double* __restrict__ per_wl, double* __restrict__ loss, int W) {
  __shared__ double sh[kLossThreads];
  loss_sum_body(per_wl, loss, W, sh);
}

// grouped: block i = design i of the plan (tasks in design order)
__global__ void __launch_bounds__(kLossThreads)
loss_sum_group_kernel(const LossTask* __restrict__ tasks, double* __restrict__ loss) {
  __shared__ double sh[kLossThreads];
  const LossTask& t = tasks[blockIdx.x];
  loss_sum_body(t.per_wl, loss + blockIdx.x, t.W, sh);
}

__device__ __forceinline__ void dh_reduce_body(const float* __restrict__ part, float* __restrict__ dh,
                                               int nchunk, int64_t per_chunk, int64_t i) {
  if (i >= per_chunk) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[c * per_chunk + i];
  dh[i] = static_cast<float>(s);
}

__global__ void dh_reduce_kernel(const float* __restrict__ part, float* __restrict__ dh, int nchunk,
                                 int64_t per_chunk) {
  dh_reduce_body(part, dh, nchunk, per_chunk, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// grouped: task = one design's gradient slots -> its dL/dh in the packed output
__global__ void dh_group_kernel(GroupArgs g, float* __restrict__ dl_dh) {
  const int ti = group_task(g, blockIdx.x);
  const DhTask& t = static_cast<const DhTask*>(g.tasks)[ti];
  const int local = static_cast<int>(blockIdx.x) - g.block0[ti];
  dh_reduce_body(t.part, dl_dh + t.h_off, t.nslots, t.per,
                 static_cast<int64_t>(local) * blockDim.x + threadIdx.x);
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
template <int M, int PAD>
static hipError_t row_dispatch_mode(int mode, const RowArgs& a, dim3 grid, hipStream_t s) {
  switch (mode) {
#define DPX_ROW(MD) \
  case MD: row_kernel<M, PAD, MD><<<grid, row_block_threads<M, MD>(), 0, s>>>(a); break;
    DPX_ROW(ROW_FWD_FIRST)
    DPX_ROW(ROW_FWD_MID)
    DPX_ROW(ROW_FWD_LAST)
    DPX_ROW(ROW_ADJ_SEED)
    DPX_ROW(ROW_ADJ_MID)
    DPX_ROW(ROW_ADJ_LAST)
#undef DPX_ROW
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M>
static hipError_t row_dispatch_pad(int pad, int mode, const RowArgs& a, dim3 grid, hipStream_t s) {
  if (pad == 2) return row_dispatch_mode<M, 2>(mode, a, grid, s);
  if (pad == 1) return row_dispatch_mode<M, 1>(mode, a, grid, s);
  return hipErrorInvalidValue;
}

#define DPX_FOR_EACH_M(X) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)

template <int M>
static void twiddle_table(std::vector<float2>& out) {
  out.assign(twiddle_count<M>() > 0 ? twiddle_count<M>() : 1, make_float2(1.f, 0.f));
  int ns = Plan<M>::R[0];
  for (int st = 1; st < Plan<M>::NST; ++st) {
    const int R = Plan<M>::R[st];
    const int L = ns * R;
    const int off = twiddle_offset<M>(st);
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < ns; ++k) {
        const double ang = 6.283185307179586476925286766559 * static_cast<double>((r * k) % L) /
                           static_cast<double>(L);
        out[off + (r - 1) * ns + k] = make_float2(static_cast<float>(std::cos(ang)),
                                                  static_cast<float>(-std::sin(ang)));
      }
    ns = L;
  }
}

void build_dft_table(int M, int pad, std::vector<float2>& out) {
  const int N = M / pad;
  out.assign(static_cast<size_t>(2) * M * N, make_float2(0.f, 0.f));
  for (int ky = 0; ky < M; ++ky)
    for (int y = 0; y < N; ++y) {
      const long long m = (static_cast<long long>(ky) * y) % M;
      const double ang = 6.283185307179586476925286766559 * static_cast<double>(m) / M;
      const float2 v = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(-std::sin(ang)));
      out[static_cast<size_t>(y) * M + ky] = v;              // FT[y][ky]
      out[static_cast<size_t>(M) * N + static_cast<size_t>(ky) * N + y] = v;  // F[ky][y]
    }
}

void build_twiddle_table(int M, std::vector<float2>& out) {
  switch (M) {
#define DPX_CASE(m) case m: twiddle_table<m>(out); return;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      out.clear();
  }
}

bool fft_size_supported(int M) {
  switch (M) {
#define DPX_CASE(m) case m:
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    return true;
    default:
      return false;
  }
}

int row_lanes_per_transform(int M) {
  switch (M) {
#define DPX_CASE(m) case m: return Geo<m>::P;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return 0;
  }
}

int row_rows_per_block(int M, int mode) {
  const int P = row_lanes_per_transform(M);
  if (P == 0) return 0;
  return row_threads_of_mode(mode) / P;
}

hipError_t launch_row(int M, int pad, int mode, const RowArgs& a, int n_row_blocks, int n_w_blocks,
                      hipStream_t s) {
  dim3 grid(n_row_blocks, n_w_blocks);
  switch (M) {
#define DPX_CASE(m) case m: return row_dispatch_pad<m>(pad, mode, a, grid, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Column-pass variants (0-3 give the same results bit for bit; 4 differs by rounding):
//   0: 8-column tiles, 1: 16-column tiles, 2: 8-column tiles + mirrored H rows,
//   3: 16-column tiles + mirrored H rows, 4: DFT as complex matrix products on the matrix
//   cores (transform lengths up to 512).
// Tiles must be whole wavefronts: with fewer than 8 lanes per transform, 8-column tiles
// fall back to 16 columns.
const char* const kColVariantNames[kColVariants] = {"tile8", "tile16", "tile8+mirror",
                                                    "tile16+mirror", "dft-gemm-mfma"};

// built-in choice when no variant is forced and no autotuning is asked for
int default_col_variant(int M) { return M >= 512 ? 2 : 3; }

template <int M, int PAD, int TX, bool MIRROR>
static hipError_t col_launch(bool conj, const ColArgs& a, int w_count, hipStream_t s) {
  dim3 grid(M / TX, (w_count + a.col_wpb - 1) / a.col_wpb);
  if (conj)
    col_kernel<M, PAD, true, TX, MIRROR><<<grid, TX * Geo<M>::P, 0, s>>>(a);
  else
    col_kernel<M, PAD, false, TX, MIRROR><<<grid, TX * Geo<M>::P, 0, s>>>(a);
  return hipGetLastError();
}

template <int M, int PAD>
static hipError_t col_dispatch_variant(int variant, bool conj, const ColArgs& a, int w_count,
                                       hipStream_t s) {
  const bool t8 = col_tile_width(M, variant) == 8;
  const bool mirror = variant >= 2;
  if (t8) return mirror ? col_launch<M, PAD, 8, true>(conj, a, w_count, s)
                        : col_launch<M, PAD, 8, false>(conj, a, w_count, s);
  return mirror ? col_launch<M, PAD, 16, true>(conj, a, w_count, s)
                : col_launch<M, PAD, 16, false>(conj, a, w_count, s);
}

template <int M>
static hipError_t col_dispatch(int pad, bool conj, int variant, const ColArgs& a, int w_count,
                               hipStream_t s) {
  if (pad == 2) return col_dispatch_variant<M, 2>(variant, conj, a, w_count, s);
  if (pad == 1) return col_dispatch_variant<M, 1>(variant, conj, a, w_count, s);
  return hipErrorInvalidValue;
}

template <int M, int PAD>
static hipError_t colgemm_launch(bool conj, const ColArgs& a, const float2* dft, int w_count, hipStream_t s) {
  if constexpr (M <= 512 && M % 16 == 0 && (M / PAD) % 16 == 0) {
    dim3 grid(M / kGemmTile, w_count);
    if (conj)
      colgemm_kernel<M, PAD, true><<<grid, gemm_threads(M), 0, s>>>(a, dft);
    else
      colgemm_kernel<M, PAD, false><<<grid, gemm_threads(M), 0, s>>>(a, dft);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

bool col_variant_supported(int M, int pad, int variant) {
  if (variant < 0 || variant >= kColVariants) return false;
  if (variant == 4) return M <= 512 && M % 16 == 0 && (M / pad) % 16 == 0;
  return true;
}

hipError_t launch_col(int M, int pad, bool conj, int variant, const ColArgs& a, int w_count,
                      hipStream_t s) {
  if (!col_variant_supported(M, pad, variant)) return hipErrorInvalidValue;
  if (variant == 4) {
    ColArgs one = a;
    one.col_wpb = 1;
    switch (M) {
#define DPX_CASE(m) \
  case m: return pad == 2 ? colgemm_launch<m, 2>(conj, one, a.dft, w_count, s) : colgemm_launch<m, 1>(conj, one, a.dft, w_count, s);
      DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (M) {
#define DPX_CASE(m) case m: return col_dispatch<m>(pad, conj, variant, a, w_count, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_bin_intensity(const float2* ofov, float* out, int w_count, int fov, int bin,
                                hipStream_t s) {
  const int T = fov / bin;
  const size_t total = static_cast<size_t>(w_count) * T * T;
  const int th = 256;
  bin_intensity_kernel<<<static_cast<unsigned>((total + th - 1) / th), th, 0, s>>>(ofov, out, w_count,
                                                                                 fov, bin);
  return hipGetLastError();
}

hipError_t launch_loss(const float* I, const float* tau, float* dl_di, double* per_wl, int W, int T,
                       hipStream_t s) {
  loss_kernel<<<W, kLossThreads, 0, s>>>(I, tau, dl_di, per_wl, W, T);
  return hipGetLastError();
}

hipError_t launch_loss_sum(const double* per_wl, double* loss, int W, hipStream_t s) {
  loss_sum_kernel<<<1, kLossThreads, 0, s>>>(per_wl, loss, W);
  return hipGetLastError();
}

hipError_t launch_dh_reduce(const float* part, float* dh, int nchunk, int64_t per_chunk,
                            hipStream_t s) {
  const int th = 256;
  dh_reduce_kernel<<<static_cast<unsigned>((per_chunk + th - 1) / th), th, 0, s>>>(part, dh, nchunk,
                                                                                 per_chunk);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Grouped launchers: the grid is block0[ntasks] blocks
// ------------------------------------------------------------------------------------------
static unsigned group_grid(const GroupArgs& g) { return static_cast<unsigned>(g.block0[g.ntasks]); }

template <int M, int PAD>
static hipError_t row_group_mode(int mode, const GroupArgs& g, hipStream_t s) {
  switch (mode) {
#define DPX_ROW(MD) \
  case MD: row_group_kernel<M, PAD, MD><<<group_grid(g), row_block_threads<M, MD>(), 0, s>>>(g); break;
    DPX_ROW(ROW_FWD_FIRST)
    DPX_ROW(ROW_FWD_MID)
    DPX_ROW(ROW_FWD_LAST)
    DPX_ROW(ROW_ADJ_SEED)
    DPX_ROW(ROW_ADJ_MID)
    DPX_ROW(ROW_ADJ_LAST)
#undef DPX_ROW
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_group(int M, int pad, int mode, const GroupArgs& g, hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks) return hipErrorInvalidValue;
  switch (M) {
#define DPX_CASE(m) \
  case m: return pad == 2 ? row_group_mode<m, 2>(mode, g, s) : pad == 1 ? row_group_mode<m, 1>(mode, g, s) : hipErrorInvalidValue;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int col_tile_width(int M, int variant) {
  const int P = row_lanes_per_transform(M);
  return ((variant == 0 || variant == 2) && 8 * P >= 64) ? 8 : 16;
}

template <int M, int PAD, int TX, bool MIRROR>
static hipError_t col_group_tx(bool conj, const GroupArgs& g, hipStream_t s) {
  if (conj)
    col_group_kernel<M, PAD, true, TX, MIRROR><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
  else
    col_group_kernel<M, PAD, false, TX, MIRROR><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
  return hipGetLastError();
}

template <int M, int PAD>
static hipError_t col_group_variant(int variant, bool conj, const GroupArgs& g, hipStream_t s) {
  const bool t8 = col_tile_width(M, variant) == 8;
  const bool mirror = variant >= 2;
  if (t8) return mirror ? col_group_tx<M, PAD, 8, true>(conj, g, s) : col_group_tx<M, PAD, 8, false>(conj, g, s);
  return mirror ? col_group_tx<M, PAD, 16, true>(conj, g, s) : col_group_tx<M, PAD, 16, false>(conj, g, s);
}

hipError_t launch_col_group(int M, int pad, bool conj, int variant, const GroupArgs& g, hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks || variant < 0 || variant > 3) return hipErrorInvalidValue;
  switch (M) {
#define DPX_CASE(m) \
  case m: return pad == 2 ? col_group_variant<m, 2>(variant, conj, g, s) : pad == 1 ? col_group_variant<m, 1>(variant, conj, g, s) : hipErrorInvalidValue;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_bin_group(const GroupArgs& g, float* out, hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks) return hipErrorInvalidValue;
  bin_group_kernel<<<group_grid(g), kGroupThreads, 0, s>>>(g, out);
  return hipGetLastError();
}

hipError_t launch_loss_group(const GroupArgs& g, const float* I, const float* tau, float* dl_di,
                             hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks) return hipErrorInvalidValue;
  loss_group_kernel<<<group_grid(g), kLossThreads, 0, s>>>(g, I, tau, dl_di);
  return hipGetLastError();
}

hipError_t launch_loss_sum_group(const LossTask* tasks, int ntasks, double* loss, hipStream_t s) {
  if (ntasks < 1) return hipErrorInvalidValue;
  loss_sum_group_kernel<<<ntasks, kLossThreads, 0, s>>>(tasks, loss);
  return hipGetLastError();
}

hipError_t launch_dh_group(const GroupArgs& g, float* dl_dh, hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks) return hipErrorInvalidValue;
  dh_group_kernel<<<group_grid(g), kGroupThreads, 0, s>>>(g, dl_dh);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  fill_zero_kernel<<<static_cast<unsigned>((n + th - 1) / th), th, 0, s>>>(p, n);
  return hipGetLastError();
}

}  // namespace dpx
