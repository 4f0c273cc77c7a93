// Host/device shared descriptions of one launch of each pass.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dpx {

// Per-wavelength constants, built on the host in double precision (paper Eq. 1 and the
// transfer function of the gap):
//   rt = (n - n_m) / lambda                 [1/m]   phase of t in revolutions per metre
//   ca = 2 pi kappa / lambda                [1/m]   absorption of t per metre
//   q0 = (M dx n_m / lambda)^2              [-]     squared radius of the propagating disc
//                                                   in units of the frequency grid step
//   ct = 2 pi (n - n_m) / lambda            [1/m]   phase per metre (gradient)
struct WlConst {
  double rt, ca, q0, ct;
};

enum RowMode : int {
  ROW_FWD_FIRST = 0,  // u_in * t_0 -> checkpoint -> pad -> row FFT
  ROW_FWD_MID = 1,    // row IFFT -> crop -> * t_l -> checkpoint -> pad -> row FFT
  ROW_FWD_LAST = 2,   // row IFFT -> crop to the field of view -> output field
  ROW_ADJ_SEED = 3,   // 2 dL/dI o on the field of view -> pad -> row FFT
  ROW_ADJ_MID = 4,    // row IFFT -> crop -> dL/dh_l partial -> * conj(t_l) -> pad -> row FFT
  ROW_ADJ_LAST = 5,   // row IFFT -> crop -> dL/dh_0 partial
  ROW_ADJ_LAST_U = 6, // the same with the field after layer 0 rebuilt as u_in * t_0 (no
                      // checkpoint slab for layer 0: the input meets layer 0 directly)
};

// timer kind (dpx_pass) of a row-pass mode
constexpr int row_pass_kind(int mode) { return 2 + (mode == ROW_ADJ_LAST_U ? ROW_ADJ_LAST : mode); }

// Threads per row-pass block: 512 (eight transforms of 1024) where the registers allow two
// such blocks per CU next to their LDS, 256 for the register-heavy adjoint middle pass.
constexpr int row_threads_of_mode(int mode) { return mode == ROW_ADJ_MID ? 256 : 512; }
// Threads of a row-pass block for P lanes per transform: the mode's count when transforms tile
// a wavefront; three or so whole transforms (about 256 threads) when one spans wavefronts.
constexpr int row_threads_for(int P, int mode) {
  return (P <= 64 && 64 % P == 0) ? row_threads_of_mode(mode) : (256 / P) * P;
}

struct RowArgs {
  float2* spec;              // [wc][N][M] row-transformed planes of the current chunk
  const float* h;            // [N][N] heights of the layer used by this pass
  const float2* u_in;        // [N][N] or null (unit plane wave)
  float2* ckpt;              // [K - ckpt_first][wc][N][N] fields after each transmission
                             // (chunk-local w); slab 0 holds layer ckpt_first
  float2* ofov;              // [wc][F][F] output field on the field of view
  const float* dl_di;        // [W][T][T] (global w)
  float* dh_part;            // [nchunk][K][N][N] per-chunk dL/dh partial sums
  const WlConst* wl;         // [W] (global w)
  const float2* tw;          // per-stage twiddle table of the transform length
  int n, fov, bin, layer, layers;
  int row_lo, row_hi;        // rows this pass processes
  int w_begin, w_count;      // global wavelength range of this launch (chunk)
  int w_per_block;           // wavelengths each block loops over
  int chunk_base;            // global chunk index of blockIdx.y == 0 (dL/dh partials)
  int ckpt_w_stride;         // wavelengths in one checkpoint layer slab
  int store_ckpt;
  int accumulate;            // dL/dh partials: add to the slot instead of overwriting it
  int no_layer;              // ROW_FWD_FIRST only: u_in passes unchanged (the input plane before
                             // an input gap: no transmission, h not read)
  int ckpt_first;            // 1: layer 0 has no checkpoint slab (ROW_ADJ_LAST_U rebuilds
                             // u_in t_0(h) from u_in and h)
};

struct ColArgs {
  float2* spec;              // [wc][N][M]
  const WlConst* wl;         // [W] (global w)
  const float2* tw;          // per-stage twiddle table of the transform length
  double zrev;               // z / (M dx): revolutions per unit of sqrt(q)
  double sx, sy;             // lateral translation of the gap / (M dx): revolutions per signed
                             // frequency index (0, 0 unless the plan has a misalignment)
  int band_limited;          // band-limited angular spectrum (per-element H evaluation only)
  int n;
  int in_lo, in_hi;          // rows holding non-zero input (others read as zero)
  int out_lo, out_hi;        // rows whose output is kept
  int w_begin;               // global wavelength of chunk-local wavelength 0
  int w_count;               // wavelengths in this launch
  int col_wpb;               // wavelengths each block runs (>= 1)
  const float2* dft;         // DFT matrices of the transform (matrix-core variant only)
  const float2* htab;        // [W][M/2+1][M/2+1] H(|kx|, |ky|) / M^2 of this gap, or null:
                             // evaluate H in the kernel (global w)
};

// ------------------------------------------------------------------------------------------
// LDS-resident path for short transforms (M <= 128): one block per wavelength keeps its plane
// in LDS and runs every layer of the forward (with the intensity binning) or of the adjoint
// (with the dL/dh partials) in one launch.
// ------------------------------------------------------------------------------------------
struct LdsArgs {
  const WlConst* wl;         // [W]
  const float2* tw;          // per-stage twiddle table of the transform length
  const double* zrev;        // [K] z_l / (M dx)
  const float* h;            // [K][N][N] heights of the design
  const float2* u_in;        // [N][N] or null (unit plane wave)
  float2* ckpt;              // [K][W][N][N] fields after each transmission
  float2* ofov;              // [W][F][F] output field on the field of view
  float* intensity;          // [W][T][T] (forward)
  const float* dl_di;        // [W][T][T] (adjoint)
  float* dh_part;            // [W][K][N][N] dL/dh of each wavelength (adjoint)
  int K, fov, bin, W;
};

// Intensity of output i of a [w_count][T][T] image set: sum of |o|^2 over the b x b bin of the
// [w_count][fov][fov] window field (fused multiply-adds in a fixed order)
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

constexpr int kLdsThreads = 512;
// whether the LDS-resident kernels are built for this transform length and pad
bool lds_path_supported(int M, int pad);
hipError_t launch_lds(int M, int pad, bool adjoint, const LdsArgs& a, hipStream_t s);

// ------------------------------------------------------------------------------------------
// Grouped launches: one launch of a pass for several designs that share the transform length
// (and pad, mode, column variant).  Each design is a task owning a contiguous run of blocks
// of a one-dimensional grid; the first block of every task travels in the kernel argument
// (kMaxGroupTasks per launch), the tasks' arguments in a device array built at plan
// creation.  Buffers the caller passes per call (heights, input field, dL/dI, outputs) are
// offsets in the tasks and base pointers in the launch.
// ------------------------------------------------------------------------------------------
constexpr int kMaxGroupTasks = 64;

struct CallBuffers {
  const float* h;            // packed heights (all designs)
  const float2* u_in;        // packed input fields or null
  const float* dl_di;        // packed dL/dI or null
};

struct GroupArgs {
  const void* tasks;         // RowTask / ColTask / BinTask / LossTask / DhTask [ntasks]
  CallBuffers call;
  int ntasks;
  int block0[kMaxGroupTasks + 1];  // first block of each task; block0[ntasks] = grid size
};

struct RowTask {
  RowArgs a;                 // h, u_in, dl_di unset: taken from the call plus the offsets
  int64_t h_off, u_off, img_off;
  int gx;                    // row blocks (x extent of the design's own grid)
  int nblocks;               // gx times the wavelength blocks
};

struct ColTask {
  ColArgs a;
  int gx;                    // column tiles
  int nblocks;               // gx times the wavelength blocks
};

struct BinTask {
  const float2* ofov;        // [W][F][F] window field
  int64_t img_off;           // offset of the design's intensities in the packed output
  int w_count, fov, bin;
};

struct LossTask {
  int64_t img_off;           // offset of the design's images in the packed buffers
  double* per_wl;            // [W] per-wavelength loss of the design
  int W, T;
};

struct DhTask {
  const float* part;         // [nslots][K][N][N] gradient slots
  int64_t h_off;             // offset of the design's heights in the packed dL/dh
  int64_t per;               // K N N
  int nslots;
};

constexpr int kGroupThreads = 256;  // threads per block of the grouped binning / reduction

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

// Supported transform lengths; the pass launchers of each live in their own translation unit.
#define DPX_FOR_EACH_M(X) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024) X(1600)
#define DPX_DECLARE_PASS_LAUNCHERS(m)                                                                   \
  hipError_t launch_row_##m(int pad, int mode, int plan, const RowArgs& a, int n_row_blocks,             \
                            int n_w_blocks, hipStream_t s);                                             \
  hipError_t launch_row_group_##m(int pad, int mode, const GroupArgs& g, hipStream_t s);                \
  hipError_t launch_col_##m(int pad, bool conj, int variant, int plan, const ColArgs& a, int w_count,    \
                            hipStream_t s);                                                             \
  void twiddle_table_##m(int plan, std::vector<float2>& out);                                           \
  hipError_t launch_col_group_##m(int pad, bool conj, int variant, bool table, bool full,               \
                                  const GroupArgs& g, hipStream_t s);                                   \
  hipError_t launch_transfer_table_##m(const WlConst* wl, int W, double zrev, float2* out, hipStream_t s); \
  hipError_t launch_lds_##m(int pad, bool adjoint, const LdsArgs& a, hipStream_t s);                     \
  bool lds_supported_##m(int pad);
DPX_FOR_EACH_M(DPX_DECLARE_PASS_LAUNCHERS)
#undef DPX_DECLARE_PASS_LAUNCHERS

hipError_t launch_row_group(int M, int pad, int mode, const GroupArgs& g, hipStream_t s);
// table: every task's arguments carry a transfer table (else none does); full: every task reads
// and keeps all its aperture rows
hipError_t launch_col_group(int M, int pad, bool conj, int variant, bool table, bool full, const GroupArgs& g,
                            hipStream_t s);
hipError_t launch_bin_group(const GroupArgs& g, float* out, hipStream_t s);
hipError_t launch_loss_group(const GroupArgs& g, const float* I, const float* tau, float* dl_di,
                             hipStream_t s);
hipError_t launch_loss_sum_group(const LossTask* tasks, int ntasks, double* loss, hipStream_t s);
hipError_t launch_dh_group(const GroupArgs& g, float* dl_dh, hipStream_t s);
int col_tile_width(int M, int variant);  // columns per block of a transform variant (0-3)

// launchers (dpx_kernels.hip); each returns a hipError_t from the launch
// plan: the radix plan of the transforms (0 .. radix_plan_count(M) - 1)
hipError_t launch_row(int M, int pad, int mode, int plan, const RowArgs& a, int n_row_blocks, int n_w_blocks,
                      hipStream_t s);
constexpr int kColVariants = 5;
bool col_variant_supported(int M, int pad, int variant);
// host: FT[y][ky] then F[ky][y] (F = exp(-2 pi i ky y / M), y < M / pad) for the matrix-core
// column pass
void build_dft_table(int M, int pad, std::vector<float2>& out);
extern const char* const kColVariantNames[kColVariants];
int default_col_variant(int M);
hipError_t launch_col(int M, int pad, bool conj, int variant, int plan, const ColArgs& a, int w_count,
                      hipStream_t s);
// fills out[w][|kx|][|ky|] (w < W, |kx|, |ky| <= M/2) with H / M^2 of the gap z = zrev M dx,
// by the same device function the column pass evaluates
hipError_t launch_transfer_table(int M, const WlConst* wl, int W, double zrev, float2* out, hipStream_t s);
hipError_t launch_bin_intensity(const float2* ofov, float* out, int w_count, int fov, int bin,
                                hipStream_t s);
hipError_t launch_loss(const float* I, const float* tau, float* dl_di, double* per_wl, int W, int T,
                       hipStream_t s);
hipError_t launch_loss_sum(const double* per_wl, double* loss, int W, hipStream_t s);
// most wavelengths dpx_loss_static takes (its partials live in a fixed device array)
constexpr int kStaticLossMaxWl = 65536;
// device address of that array on the current device (looked up once per device)
hipError_t static_loss_scratch(double** out);
hipError_t launch_dh_reduce(const float* part, float* dh, int nchunk, int64_t per_chunk,
                            hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
// adds the number of NaN and infinite values among x[0..n) to *count (integer atomics)
hipError_t launch_count_nonfinite(const float* x, int64_t n, unsigned* count, hipStream_t s);
hipError_t launch_count_nonfinite(const double* x, int64_t n, unsigned* count, hipStream_t s);

// Adam on theta with h = h_max sigmoid(theta) (see adam_sigmoid_kernel)
struct AdamArgs {
  float lr, b1, b2, eps, h_max;
  float omb1, omb2;  // 1 - b1, 1 - b2 (formed in double)
  float c1, c2;      // 1 / (1 - b1^t), 1 / (1 - b2^t)
};
hipError_t launch_quantize(const float* h, float* out, int64_t n, float scale, float step, float kmax,
                           hipStream_t s);
hipError_t launch_adam_sigmoid(float* theta, float* h, const float* dl_dh, float* m, float* v, int64_t n,
                               const AdamArgs& a, hipStream_t s);
// per-wavelength PSNR of one design's [W][T][T] images -> out [W]
hipError_t launch_psnr(const float* I, const float* tau, double* out, int W, int T, hipStream_t s);

bool fft_size_supported(int M);
// host: per-stage twiddle table of the length-M transform (layout in fft.hpp)
void build_twiddle_table(int M, int plan, std::vector<float2>& out);
// radix plans of a transform length (plan 0 is the built-in one; the others run the evaluated
// and mirrored transfer functions of untranslated full-spectrum gaps, per-design schedule only)
int radix_plan_count(int M);
const char* radix_plan_name(int M, int plan);
int row_lanes_per_transform(int M);  // P = M / E
int row_rows_per_block(int M, int mode);  // rows (transforms) per row-pass block

}  // namespace dpx
