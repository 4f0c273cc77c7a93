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
};

struct RowArgs {
  float2* spec;              // [wc][N][M] row-transformed planes of the current chunk
  const float* h;            // [N][N] heights of the layer used by this pass
  const float2* u_in;        // [N][N] or null (unit plane wave)
  float2* ckpt;              // [K][wc][N][N] fields after each transmission (chunk-local w)
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
};

struct ColArgs {
  float2* spec;              // [wc][N][M]
  const WlConst* wl;         // [W] (global w)
  const float2* tw;          // per-stage twiddle table of the transform length
  double zrev;               // z / (M dx): revolutions per unit of sqrt(q)
  int n;
  int in_lo, in_hi;          // rows holding non-zero input (others read as zero)
  int out_lo, out_hi;        // rows whose output is kept
  int w_begin;               // global wavelength of chunk-local wavelength 0
  int w_count;               // wavelengths in this launch
  int col_wpb;               // wavelengths each block runs (>= 1)
  const float2* dft;         // DFT matrices of the transform (matrix-core variant only)
};

// launchers (dpx_kernels.hip); each returns a hipError_t from the launch
hipError_t launch_row(int M, int pad, int mode, const RowArgs& a, int n_row_blocks, int n_w_blocks,
                      hipStream_t s);
constexpr int kColVariants = 5;
bool col_variant_supported(int M, int pad, int variant);
// host: FT[y][ky] then F[ky][y] (F = exp(-2 pi i ky y / M), y < M / pad) for the matrix-core
// column pass
void build_dft_table(int M, int pad, std::vector<float2>& out);
extern const char* const kColVariantNames[kColVariants];
int default_col_variant(int M);
hipError_t launch_col(int M, int pad, bool conj, int variant, const ColArgs& a, int w_count,
                      hipStream_t s);
hipError_t launch_bin_intensity(const float2* ofov, float* out, int w_count, int fov, int bin,
                                hipStream_t s);
hipError_t launch_loss(const float* I, const float* tau, float* dl_di, double* per_wl, int W, int T,
                       hipStream_t s);
hipError_t launch_loss_sum(const double* per_wl, double* loss, int W, hipStream_t s);
hipError_t launch_dh_reduce(const float* part, float* dh, int nchunk, int64_t per_chunk,
                            hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);

bool fft_size_supported(int M);
// host: per-stage twiddle table of the length-M transform (layout in fft.hpp)
void build_twiddle_table(int M, std::vector<float2>& out);
int row_lanes_per_transform(int M);  // P = M / E
int row_rows_per_block(int M, int mode);  // rows (transforms) per row-pass block

}  // namespace dpx
