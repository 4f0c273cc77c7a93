// HIP kernels for gfx950 that do not depend on the transform length (intensity binning, loss,
// gradient reduction), host-side tables (stage twiddles, DFT matrices), and the dispatch of
// the per-length pass launchers (dpx_pass.hip, one translation unit per length).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "dpx_internal.hpp"
#include "fft.hpp"

namespace dpx {

// ------------------------------------------------------------------------------------------
// Small kernels
// ------------------------------------------------------------------------------------------

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

// Fixed device array for the per-wavelength loss partials of dpx_loss_static (callers that cannot
// allocate): every GPU the library runs on holds one copy until the process ends.  Host code
// never passes the array's name to a kernel (in host code it is a stand-in, not a device
// address); static_loss_scratch() returns the device address, looked up once per device.
static __device__ __align__(256) double scratch[kStaticLossMaxWl];

constexpr int kMaxScratchDevices = 64;

hipError_t static_loss_scratch(double** out) {
  static std::mutex mu;
  static void* ptr[kMaxScratchDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = p;
  }
  *out = static_cast<double*>(ptr[dev]);
  return hipSuccess;
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

// ------------------------------------------------------------------------------------------
// Training support (Section 4: Adam with the optimizer library's defaults; heights bounded to
// [0, h_max] through a sigmoid of an unconstrained variable)
// ------------------------------------------------------------------------------------------
// One Adam step on theta with h = h_max sigmoid(theta):
//   g = dL/dh * h_max s (1 - s),  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   theta -= lr (m c1) / (sqrt(v c2) + eps)  with c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t),
// then h = h_max sigmoid(theta).  Arithmetic in single precision; 1 - b1, 1 - b2 and the bias
// corrections come from the host, formed in double.
// Phase bit depth: the nearest of the levels k step, k = 0 .. kmax (ties to even), the level
// index decided in single precision as rint(h scale), clamped to the end levels.
__global__ void quantize_kernel(const float* h, float* out, int64_t n, float scale, float step, float kmax) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float k = fminf(fmaxf(rintf(h[i] * scale), 0.0f), kmax);
  out[i] = k * step;
}

__global__ void adam_sigmoid_kernel(float* __restrict__ theta, float* __restrict__ h, const float* __restrict__ dl_dh,
                                    float* __restrict__ m, float* __restrict__ v, int64_t n, AdamArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float th = theta[i];
  // s (1 - s) = e / (1 + e)^2 with e = exp(-|theta|): even in theta, no cancellation near
  // s = 1 and no overflow for large |theta|.
  const float e = expf(-fabsf(th));
  const float ope = 1.0f + e;
  const float g = dl_dh[i] * (a.h_max * (e / (ope * ope)));
  const float mi = fmaf(a.b1, m[i], a.omb1 * g);
  const float vi = fmaf(a.b2, v[i], a.omb2 * (g * g));
  m[i] = mi;
  v[i] = vi;
  const float t2 = th - a.lr * (mi * a.c1) / (sqrtf(vi * a.c2) + a.eps);
  theta[i] = t2;
  h[i] = a.h_max / (1.0f + expf(-t2));
}

// Per-wavelength PSNR of the intensity image against its target, both normalised to unit sum
// (as in the loss): 10 log10(max_p tau^2 / mean_p (I - tau)^2), in double; one block per
// wavelength of one design ([W][T][T] images, out [W]).
__global__ void __launch_bounds__(kLossThreads)
psnr_kernel(const float* __restrict__ I, const float* __restrict__ tau, double* __restrict__ out, int T) {
  __shared__ double sh[kLossThreads];
  const int w = blockIdx.x;
  const int P = T * T;
  const float* Iw = I + static_cast<size_t>(w) * P;
  const float* tw = tau + static_cast<size_t>(w) * P;
  double si = 0.0, st = 0.0, mx = 0.0;
  for (int p = threadIdx.x; p < P; p += kLossThreads) {
    si += Iw[p];
    st += tw[p];
    mx = fmax(mx, static_cast<double>(tw[p]));
  }
  const double S = block_sum(si, sh);
  const double St = block_sum(st, sh);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kLossThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double tmax = sh[0];
  __syncthreads();
  const double rS = S > 0.0 ? 1.0 / S : 0.0;
  const double rSt = St > 0.0 ? 1.0 / St : 0.0;
  double sd2 = 0.0;
  for (int p = threadIdx.x; p < P; p += kLossThreads) {
    const double d = Iw[p] * rS - tw[p] * rSt;
    sd2 += d * d;
  }
  const double mse = block_sum(sd2, sh) / P;
  if (threadIdx.x == 0) {
    const double peak = tmax * rSt;
    out[w] = (mse > 0.0) ? 10.0 * log10(peak * peak / mse) : INFINITY;
  }
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Counts the NaN and infinite values of x (grid-stride); one integer atomic per lane that
// found any, so the count is exact and independent of the launch shape.
template <typename T>
__global__ void __launch_bounds__(256) count_nonfinite_kernel(const T* __restrict__ x, int64_t n,
                                                              unsigned* __restrict__ count) {
  unsigned c = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    c += isfinite(x[i]) ? 0u : 1u;
  if (c) atomicAdd(count, c);
}


// ------------------------------------------------------------------------------------------
// Host-side tables and sizes
// ------------------------------------------------------------------------------------------
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

void build_twiddle_table(int M, int plan, std::vector<float2>& out) {
  switch (M) {
#define DPX_CASE(m) case m: twiddle_table_##m(plan, out); return;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      out.clear();
  }
}
int radix_plan_count(int M) { return fft_size_supported(M) ? radix_plans(M) : 0; }
template <int m, int v>
static void radix_name(char* buf, size_t cap) {
  int n = 0;
  for (int st = 0; st < Radix<m, v>::NST; ++st)
    n += snprintf(buf + n, cap - n, st ? "x%d" : "%d", Radix<m, v>::R[st]);
}
// "16x16x4": the radices of plan `plan` of length M (empty for an unknown pair)
const char* radix_plan_name(int M, int plan) {
  static thread_local char buf[32];
  buf[0] = 0;
  if (plan < 0 || plan >= radix_plan_count(M)) return buf;
  switch (M) {
#define DPX_CASE(m) \
  case m:           \
    if (plan == 0) radix_name<m, 0>(buf, sizeof(buf)); \
    break;
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default: break;
  }
  if (M == 512 && plan == 1) radix_name<512, 1>(buf, sizeof(buf));
  if (M == 512 && plan == 2) radix_name<512, 2>(buf, sizeof(buf));
  if (M == 1024 && plan == 1) radix_name<1024, 1>(buf, sizeof(buf));
  if (M == 1024 && plan == 2) radix_name<1024, 2>(buf, sizeof(buf));
  return buf;
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
  return row_threads_for(P, mode) / P;
}

namespace {
// the lanes of one transform lie in one wavefront (else its LDS exchanges take block barriers,
// tiles are 4 or 8 columns wide and H has no cross-lane mirrored form)
bool wave_local(int M) {
  const int P = row_lanes_per_transform(M);
  return P > 0 && P <= 64 && 64 % P == 0;
}
}  // namespace

// Column-pass variants (0-3 give the same results bit for bit; 4 differs by rounding):
//   0: 8-column tiles, 1: 16-column tiles, 2: 8-column tiles + mirrored H rows,
//   3: 16-column tiles + mirrored H rows, 4: DFT as complex matrix products on the matrix
//   cores (transform lengths up to 512).
// Tiles must be whole wavefronts: with fewer than 8 lanes per transform, 8-column tiles
// fall back to 16 columns.
const char* const kColVariantNames[kColVariants] = {"tile8", "tile16", "tile8+mirror",
                                                    "tile16+mirror", "dft-gemm-mfma"};

// built-in choice when no variant is forced and no autotuning is asked for: the mirrored forms
// where transforms stay in one wavefront; at 1600 the wide tile (8 columns, 10 waves per CU in
// one block) beats the narrow one, which the registers hold to one 5-wave block per CU
int default_col_variant(int M) { return !wave_local(M) ? 1 : M >= 512 ? 2 : 3; }

bool col_variant_supported(int M, int pad, int variant) {
  if (variant < 0 || variant >= kColVariants) return false;
  if (variant == 4) return M <= 512 && M % 16 == 0 && (M / pad) % 16 == 0;
  if (!wave_local(M)) return variant <= 1;
  return true;
}

int col_tile_width(int M, int variant) {
  const int P = row_lanes_per_transform(M);
  if (!wave_local(M)) return variant == 0 ? 4 : 8;
  return ((variant == 0 || variant == 2) && 8 * P >= 64) ? 8 : 16;
}


// ------------------------------------------------------------------------------------------
// Dispatch to the per-length launchers
// ------------------------------------------------------------------------------------------
hipError_t launch_row(int M, int pad, int mode, int plan, const RowArgs& a, int n_row_blocks, int n_w_blocks,
                      hipStream_t s) {
  switch (M) {
#define DPX_CASE(m) case m: return launch_row_##m(pad, mode, plan, a, n_row_blocks, n_w_blocks, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_row_group(int M, int pad, int mode, const GroupArgs& g, hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks) return hipErrorInvalidValue;
  switch (M) {
#define DPX_CASE(m) case m: return launch_row_group_##m(pad, mode, g, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_col(int M, int pad, bool conj, int variant, int plan, const ColArgs& a, int w_count,
                      hipStream_t s) {
  if (!col_variant_supported(M, pad, variant)) return hipErrorInvalidValue;
  switch (M) {
#define DPX_CASE(m) case m: return launch_col_##m(pad, conj, variant, plan, a, w_count, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_col_group(int M, int pad, bool conj, int variant, bool table, bool full, const GroupArgs& g,
                            hipStream_t s) {
  if (g.ntasks < 1 || g.ntasks > kMaxGroupTasks || variant < 0 || variant > 3) return hipErrorInvalidValue;
  switch (M) {
#define DPX_CASE(m) case m: return launch_col_group_##m(pad, conj, variant, table, full, g, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

bool lds_path_supported(int M, int pad) {
  switch (M) {
#define DPX_CASE(m) case m: return lds_supported_##m(pad);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return false;
  }
}

hipError_t launch_lds(int M, int pad, bool adjoint, const LdsArgs& a, hipStream_t s) {
  switch (M) {
#define DPX_CASE(m) case m: return launch_lds_##m(pad, adjoint, a, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_transfer_table(int M, const WlConst* wl, int W, double zrev, float2* out, hipStream_t s) {
  switch (M) {
#define DPX_CASE(m) case m: return launch_transfer_table_##m(wl, W, zrev, out, s);
    DPX_FOR_EACH_M(DPX_CASE)
#undef DPX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------------------
// Small kernels: launchers
// ------------------------------------------------------------------------------------------
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

static unsigned group_grid(const GroupArgs& g) { return static_cast<unsigned>(g.block0[g.ntasks]); }

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

hipError_t launch_quantize(const float* h, float* out, int64_t n, float scale, float step, float kmax,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  quantize_kernel<<<static_cast<unsigned>((n + th - 1) / th), th, 0, s>>>(h, out, n, scale, step, kmax);
  return hipGetLastError();
}

hipError_t launch_adam_sigmoid(float* theta, float* h, const float* dl_dh, float* m, float* v, int64_t n,
                               const AdamArgs& a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  adam_sigmoid_kernel<<<static_cast<unsigned>((n + th - 1) / th), th, 0, s>>>(theta, h, dl_dh, m, v, n, a);
  return hipGetLastError();
}

hipError_t launch_psnr(const float* I, const float* tau, double* out, int W, int T, hipStream_t s) {
  if (W <= 0) return hipSuccess;
  psnr_kernel<<<W, kLossThreads, 0, s>>>(I, tau, out, T);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  fill_zero_kernel<<<static_cast<unsigned>((n + th - 1) / th), th, 0, s>>>(p, n);
  return hipGetLastError();
}

template <typename T>
hipError_t count_nonfinite(const T* x, int64_t n, unsigned* count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int th = 256;
  const int64_t blocks = std::min<int64_t>((n + th - 1) / th, 4096);
  count_nonfinite_kernel<T><<<static_cast<unsigned>(blocks), th, 0, s>>>(x, n, count);
  return hipGetLastError();
}
hipError_t launch_count_nonfinite(const float* x, int64_t n, unsigned* count, hipStream_t s) {
  return count_nonfinite(x, n, count, s);
}
hipError_t launch_count_nonfinite(const double* x, int64_t n, unsigned* count, hipStream_t s) {
  return count_nonfinite(x, n, count, s);
}

}  // namespace dpx
