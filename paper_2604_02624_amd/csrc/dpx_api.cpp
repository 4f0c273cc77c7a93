// C ABI of the dpx library: plan creation (validation, per-wavelength constants, twiddle
// tables, workspace), and the forward / loss / backward call sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <limits>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/dpx.h"
#include "dpx_internal.hpp"

using dpx::ColArgs;
using dpx::RowArgs;
using dpx::WlConst;

namespace {

thread_local std::string g_last_error;

dpx_status fail(dpx_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

dpx_status ok() {
  g_last_error.clear();
  return DPX_OK;
}

#define DPX_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(DPX_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Design {
  int N, M, K, W, F, b, T, pad;
  double dx, n_m;
  std::vector<double> wl, n_mat, kappa, z;
  std::vector<double> dz, sx, sy;  // per gap: axial jitter, lateral translation (metres)
  double z_in = 0.0;               // input plane -> layer 1 (0: u_in is the field at layer 1)
  bool band = false;               // band-limited angular spectrum
  int64_t h_off, u_off, img_off;
  // launch geometry
  int wl_chunk;      // wavelengths per chunk (spec buffer depth per lane)
  int nchunks;       // ceil(W / wl_chunk)
  int lanes;         // chunks run on this many streams at once (chunk c on lane c % lanes)
  int w_per_block;   // wavelengths per row-pass block
  int slots_per_lane;  // dL/dh partial slots of one lane = ceil(wl_chunk / w_per_block)
  int nslots;        // lanes * slots_per_lane
  int row_group;     // rows per row-pass block
  int col_variant;   // column-pass kernel variant
  int row_plan = 0;  // radix plans of the row and column transforms
  int col_plan = 0;
  bool lds = false;  // forward and adjoint as one LDS-resident launch each
  // 1: the input field meets layer 0 directly, so its field after the first transmission,
  // u_in t_0(h), is rebuilt by the last adjoint pass and gets no checkpoint slab
  int ck_first = 0;
  // transfer-function tables: one [W][M/2+1][M/2+1] table per distinct gap; zslot[l] is the
  // table of layer l's gap (empty: H is evaluated in the column pass)
  int nzslots = 0;
  std::vector<int> zslot;
  int64_t table_bytes = 0;
  // device memory
  float2* htab = nullptr;
  double* d_zrev = nullptr;  // [K] z_l / (M dx) (LDS-resident path)
  WlConst* d_wl = nullptr;
  float2* spec = nullptr;
  float2* ckpt = nullptr;
  float2* ofov = nullptr;
  float* dh_part = nullptr;
  double* per_wl = nullptr;
  int64_t bytes = 0;
};

}  // namespace

struct TimedLaunch {
  int pass;
  hipEvent_t start, stop;
  int64_t bytes;
  double flops;
  int instance = -1;  // a second timer kind the launch also counts toward (full-plane column passes)
};

struct PassTotals {
  double ms = 0.0;
  int64_t launches = 0;
  int64_t bytes = 0;
  double flops = 0.0;
};

// One launch of the grouped schedule.  g.tasks points into the plan's task buffer; g.call is
// filled per call.
enum GroupKind { GK_ROW, GK_COL, GK_BIN, GK_LOSS, GK_DH };
struct GroupLaunch {
  GroupKind kind;
  int M = 0, pad = 0, mode = 0, variant = 0;
  bool conj = false;
  bool table = false;      // column launches: the tasks read transfer tables
  bool full = false;       // column launches: every task reads and keeps all aperture rows
  dpx::GroupArgs g{};
  int pass = -1;           // DPX_PASS_* of row / column launches (timers)
  int64_t bytes = 0;       // algorithmic bytes (without the input field)
  int64_t u_bytes = 0;     // extra bytes when an input field is passed
  double flops = 0.0;
};

struct dpx_plan {
  std::vector<Design> designs;
  std::vector<hipStream_t> aux;   // lanes 1..L-1 (lane 0 is the caller's stream)
  hipEvent_t ev_fork = nullptr, ev_offset = nullptr;
  std::vector<hipEvent_t> ev_join;
  // independent designs spread over `dstreams` streams (the caller's plus aux[0..]);
  // design i runs on stream design_stream[i]
  int dstreams = 1;
  std::vector<int> design_stream;
  // HIP-graph replay (opts.use_graph): one executable graph per call kind and pointer set,
  // replayed on a plan-owned stream joined to the caller's stream by events
  hipStream_t gstream = nullptr;
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  std::map<std::array<uintptr_t, 5>, hipGraphExec_t> graphs;
  std::vector<std::array<uintptr_t, 5>> graph_order;
  bool timing = false;
  std::vector<TimedLaunch> pending;
  PassTotals totals[DPX_PASS_COUNT];
  dpx_opts opts;
  int device = 0;
  std::map<int, float2*> twiddles;
  std::map<int, float2*> dft;      // matrix-core column pass: key M * 4 + pad
  // grouped schedule (opts.schedule): every pass of every design as one launch per transform
  // length, mode and variant; task arrays in one device buffer
  bool grouped = false;
  // one forward / backward launch list per partition of the designs (partition k runs on
  // stream k, as design_stream assigns); the loss is one list over all designs
  std::vector<std::vector<GroupLaunch>> g_fwd, g_bwd;
  std::vector<GroupLaunch> g_loss;
  void* d_tasks = nullptr;
  const dpx::LossTask* d_loss_tasks = nullptr;
  // opts.check_finite: counters of non-finite output values, one per output of a call
  unsigned* d_nonfinite = nullptr;
  int64_t h_total = 0, img_total = 0;
  int64_t bytes = 0;
  bool fwd_valid = false;
  const float* last_h = nullptr;
  const float* last_u = nullptr;
};

#define DPX_TRY(expr)                   \
  do {                                  \
    dpx_status s_ = (expr);             \
    if (s_ != DPX_OK) return s_;        \
  } while (0)

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

dpx_status check_wavelengths(int i, const double* wl, const double* n_mat, const double* kappa, int n) {
  if (!wl || !n_mat) return fail(DPX_E_ARG, "design %d: wl, n_mat and z are required", i);
  for (int w = 0; w < n; ++w) {
    if (!finite_pos(wl[w])) return fail(DPX_E_ARG, "design %d: wl[%d] must be > 0", i, w);
    if (!std::isfinite(n_mat[w])) return fail(DPX_E_ARG, "design %d: n_mat[%d] not finite", i, w);
    if (kappa && !(std::isfinite(kappa[w]) && kappa[w] >= 0.0))
      return fail(DPX_E_ARG, "design %d: kappa[%d] must be finite and >= 0", i, w);
  }
  return DPX_OK;
}

dpx_status validate(const dpx_design* ds, int32_t nd, const dpx_opts* o) {
  if (!ds) return fail(DPX_E_ARG, "designs is NULL");
  if (nd < 1) return fail(DPX_E_ARG, "n_designs must be >= 1 (got %d)", nd);
  if (o) {
    if (o->checkpoint_mode != 0 && o->checkpoint_mode != 1)
      return fail(DPX_E_ARG, "checkpoint_mode must be 0 or 1");
    if (o->wl_chunk < 0) return fail(DPX_E_ARG, "wl_chunk must be >= 0");
    if (o->streams < 0 || o->streams > 8) return fail(DPX_E_ARG, "streams must be in [0, 8]");
    if (o->schedule < 0 || o->schedule > 2) return fail(DPX_E_ARG, "schedule must be 0, 1 or 2");
    if (o->transfer_table < 0 || o->transfer_table > 2)
      return fail(DPX_E_ARG, "transfer_table must be 0, 1 or 2");
    if (o->small_path < 0 || o->small_path > 1) return fail(DPX_E_ARG, "small_path must be 0 or 1");
    if (o->max_workspace_bytes < 0) return fail(DPX_E_ARG, "max_workspace_bytes must be >= 0");
    if (o->force_variant < -1 || o->force_variant >= dpx::kColVariants)
      return fail(DPX_E_ARG, "force_variant must be -1 or a variant index below %d", dpx::kColVariants);
    if (o->force_plan < -1) return fail(DPX_E_ARG, "force_plan must be -1 or a radix plan index");
  }
  for (int i = 0; i < nd; ++i) {
    const dpx_design& d = ds[i];
    if (d.n < 2 || d.n % 2) return fail(DPX_E_ARG, "design %d: n must be even and >= 2 (got %d)", i, d.n);
    if (d.layers < 1) return fail(DPX_E_ARG, "design %d: layers must be >= 1", i);
    if (d.n_wl < 1) return fail(DPX_E_ARG, "design %d: n_wl must be >= 1", i);
    if (d.fov < 1 || d.fov > d.n || (d.n - d.fov) % 2)
      return fail(DPX_E_ARG, "design %d: fov must be in [1, n] with n - fov even (n=%d fov=%d)", i,
                  d.n, d.fov);
    if (d.bin < 1 || d.fov % d.bin) return fail(DPX_E_ARG, "design %d: fov %% bin must be 0", i);
    if (d.pad != 1 && d.pad != 2) return fail(DPX_E_ARG, "design %d: pad must be 1 or 2", i);
    if (!finite_pos(d.dx)) return fail(DPX_E_ARG, "design %d: dx must be finite and > 0", i);
    if (!finite_pos(d.n_medium)) return fail(DPX_E_ARG, "design %d: n_medium must be > 0", i);
    if (!d.z) return fail(DPX_E_ARG, "design %d: wl, n_mat and z are required", i);
    DPX_TRY(check_wavelengths(i, d.wl, d.n_mat, d.kappa, d.n_wl));
    for (int l = 0; l < d.layers; ++l)
      if (!(std::isfinite(d.z[l]) && d.z[l] >= 0.0))
        return fail(DPX_E_ARG, "design %d: z[%d] must be finite and >= 0", i, l);
    if (!(std::isfinite(d.z_in) && d.z_in >= 0.0))
      return fail(DPX_E_ARG, "design %d: z_in must be finite and >= 0", i);
    if (d.band_limited != 0 && d.band_limited != 1) return fail(DPX_E_ARG, "design %d: band_limited must be 0 or 1", i);
    if (d.band_limited && o && (o->force_variant > 1 || o->transfer_table == 2))
      return fail(DPX_E_UNSUPPORTED,
                  "design %d: the band-limited spectrum runs the per-element column variants (0, 1), "
                  "without transfer tables", i);
    const int M = d.pad * d.n;
    if (o && o->force_variant >= 0 && dpx::fft_size_supported(M) &&
        !dpx::col_variant_supported(M, d.pad, o->force_variant))
      return fail(DPX_E_UNSUPPORTED, "design %d: column variant %d is not built for transform length %d", i,
                  o->force_variant, M);
    if (o && o->force_plan > 0 && dpx::fft_size_supported(M) && o->force_plan >= dpx::radix_plan_count(M))
      return fail(DPX_E_UNSUPPORTED, "design %d: transform length %d has %d radix plan(s), no plan %d", i, M,
                  dpx::radix_plan_count(M), o->force_plan);
    if (o && o->force_plan > 0 && (d.band_limited || o->transfer_table == 2 || o->schedule == 2 || o->small_path))
      return fail(DPX_E_UNSUPPORTED,
                  "design %d: radix plans other than 0 run the per-design schedule without transfer "
                  "tables, band limit or the LDS-resident path", i);
    if (!dpx::fft_size_supported(M))
      return fail(DPX_E_UNSUPPORTED,
                  "design %d: transform length pad*n = %d is not built (64, 96, 128, 192, 256, "
                  "384, 512, 1024, 1600)",
                  i, M);
  }
  return DPX_OK;
}

// Geometry and byte counts for one design (host only).
void layout_design(const dpx_design& src, const dpx_opts& o, Design& d) {
  d.N = src.n;
  d.pad = src.pad;
  d.M = src.pad * src.n;
  d.K = src.layers;
  d.W = src.n_wl;
  d.F = src.fov;
  d.b = src.bin;
  d.T = src.fov / src.bin;
  d.dx = src.dx;
  d.n_m = src.n_medium;
  d.z_in = src.z_in;
  d.band = src.band_limited != 0;
  d.row_group = dpx::row_rows_per_block(d.M, dpx::ROW_FWD_MID);
  const int row_blocks = (d.N + d.row_group - 1) / d.row_group;
  // wavelengths per chunk: everything at once unless asked otherwise (recompute mode
  // defaults to chunks of 64).  Concurrent lanes run chunks of wavelengths on several
  // streams, so that one chunk's column pass (arithmetic-bound) can run beside another
  // chunk's row pass (memory-bound); measured on the large workload, two lanes share the chip
  // without shortening the step, so the automatic choice is one lane (more on request).
  const int lanes_wanted = o.streams > 0 ? o.streams : 1;
  int chunk = o.wl_chunk > 0 ? o.wl_chunk
                             : (o.checkpoint_mode == 1 ? 64 : (d.W + 2 * lanes_wanted - 1) / (2 * lanes_wanted));
  if (lanes_wanted == 1 && o.wl_chunk <= 0 && o.checkpoint_mode == 0) chunk = d.W;
  chunk = std::max(1, std::min(chunk, d.W));
  // wavelengths per row-pass block: enough blocks to fill the chip (about 2048), at most 16
  int wpb = static_cast<int>(std::max<int64_t>(1, static_cast<int64_t>(chunk) * row_blocks / 2048));
  wpb = std::min(wpb, 16);
  if (chunk < d.W) {
    // chunks must hold whole blocks so every chunk maps onto the same partial slots
    chunk = std::max(wpb, chunk / wpb * wpb);
  }
  // LDS-resident path for short transforms (opts.small_path = 1): every wavelength is one
  // block with one dL/dh slot, the whole design one chunk
  d.lds = o.small_path == 1 && o.checkpoint_mode == 0 && o.streams <= 1 && o.force_variant < 0 &&
          src.z_in == 0.0 && src.band_limited == 0 &&
          o.transfer_table != 2 && dpx::lds_path_supported(d.M, d.pad);
  if (d.lds) {
    chunk = d.W;
    wpb = 1;
  }
  d.wl_chunk = chunk;
  d.nchunks = (d.W + chunk - 1) / chunk;
  d.lanes = std::max(1, std::min(lanes_wanted, d.nchunks));
  d.w_per_block = wpb;
  d.slots_per_lane = (chunk + wpb - 1) / wpb;
  d.nslots = d.lanes * d.slots_per_lane;
  d.col_variant = o.force_variant >= 0 ? o.force_variant : dpx::default_col_variant(d.M);
  // the band-limited spectrum is applied by the per-element evaluation: the mirrored variants'
  // tile widths without the mirror
  if (src.band_limited && d.col_variant >= 2 && d.col_variant <= 3) d.col_variant -= 2;
  // transfer tables (opts.transfer_table: 2 = always; 0 automatic and 1 = never: measured on
  // MI355X, reading H costs the column pass more load traffic and latency than evaluating it
  // saves arithmetic)
  d.table_bytes = 0;
  {
    std::vector<double> zs;
    d.zslot.assign(d.K, 0);
    for (int l = 0; l < d.K; ++l) {
      int k = 0;
      while (k < static_cast<int>(zs.size()) && zs[k] != src.z[l]) ++k;
      if (k == static_cast<int>(zs.size())) zs.push_back(src.z[l]);
      d.zslot[l] = k;
    }
    const int64_t hs = d.M / 2 + 1;
    const int64_t tb = static_cast<int64_t>(zs.size()) * d.W * hs * hs * 8;
    d.nzslots = static_cast<int>(zs.size());
    d.table_bytes = tb;
  }
  const int64_t nn = static_cast<int64_t>(d.N) * d.N;
  const int ck_w = (o.checkpoint_mode == 1) ? d.lanes * d.wl_chunk : d.W;
  const int of_w = ck_w;
  d.ck_first = (src.z_in == 0.0 && !d.lds) ? 1 : 0;
  d.bytes = static_cast<int64_t>(d.lanes) * d.wl_chunk * d.N * d.M * 8  // spec
            + static_cast<int64_t>(d.K - d.ck_first) * ck_w * nn * 8  // checkpoints
            + static_cast<int64_t>(of_w) * d.F * d.F * 8      // output field
            + static_cast<int64_t>(d.nslots) * d.K * nn * 4   // dL/dh partials
            + static_cast<int64_t>(d.W) * 8                   // per-wavelength loss
            + static_cast<int64_t>(d.W) * sizeof(WlConst)
            + static_cast<int64_t>(d.K) * 8;                  // gap table
  const bool want = o.transfer_table == 2;
  if (want) {
    d.bytes += d.table_bytes;
  } else {
    d.table_bytes = 0;
    d.nzslots = 0;
    d.zslot.clear();
  }
}

void free_design(Design& d) {
  hipFree(d.d_wl);
  hipFree(d.spec);
  hipFree(d.ckpt);
  hipFree(d.ofov);
  hipFree(d.dh_part);
  hipFree(d.per_wl);
  hipFree(d.htab);
  hipFree(d.d_zrev);
  d.htab = nullptr;
  d.d_zrev = nullptr;
  d.d_wl = nullptr;
  d.spec = d.ckpt = d.ofov = nullptr;
  d.dh_part = nullptr;
  d.per_wl = nullptr;
}

template <typename T>
dpx_status dev_alloc(T** p, int64_t bytes, const char* what) {
  if (bytes <= 0) {
    *p = nullptr;
    return DPX_OK;
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(bytes));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(DPX_E_NOMEM, "hipMalloc of %lld bytes for %s failed: %s", static_cast<long long>(bytes),
                what, hipGetErrorString(e));
  }
  return DPX_OK;
}

dpx_status check_ptr(const void* p, size_t align, const char* name) {
  if (!p) return fail(DPX_E_ARG, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % align)
    return fail(DPX_E_ARG, "%s is not %zu-byte aligned", name, align);
  return DPX_OK;
}

dpx_status sticky_check() {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DPX_E_DEVICE, "pending HIP error: %s", hipGetErrorString(e));
  }
  return DPX_OK;
}

float2* spec_of_lane(const Design& d, int lane) {
  return d.spec + static_cast<int64_t>(lane) * d.wl_chunk * d.N * d.M;
}

// opts.check_finite: counts the NaN and infinite values of a call's outputs on its stream,
// waits for them and reports the first output that holds any
struct OutputSpan {
  const void* p;
  int64_t n;
  bool f64;
  const char* name;
};

dpx_status check_outputs(dpx_plan* p, std::initializer_list<OutputSpan> outs, hipStream_t s) {
  if (!p->opts.check_finite) return DPX_OK;
  const int k = static_cast<int>(outs.size());
  hipError_t e = dpx::launch_fill_zero(reinterpret_cast<float*>(p->d_nonfinite), k, s);
  int i = 0;
  for (const auto& o : outs) {
    if (e == hipSuccess && o.p)
      e = o.f64 ? dpx::launch_count_nonfinite(static_cast<const double*>(o.p), o.n, p->d_nonfinite + i, s)
                : dpx::launch_count_nonfinite(static_cast<const float*>(o.p), o.n, p->d_nonfinite + i, s);
    ++i;
  }
  unsigned counts[8] = {};
  if (e == hipSuccess) e = hipMemcpyAsync(counts, p->d_nonfinite, k * sizeof(unsigned), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "non-finite scan failed: %s", hipGetErrorString(e));
  i = 0;
  for (const auto& o : outs) {
    if (counts[i])
      return fail(DPX_E_NONFINITE, "%s holds %u NaN or infinite value(s) of %lld", o.name, counts[i],
                  static_cast<long long>(o.n));
    ++i;
  }
  return DPX_OK;
}

// key of a twiddle table in dpx_plan::twiddles
int tw_key(int M, int plan) { return M * 8 + plan; }

// the radix plan a column launch runs: the design's, unless its transfer function comes from a
// source that only plan 0 has (tables, band limit, translated gaps)
int col_plan_of(const Design& d, const ColArgs& c) {
  if (c.htab || c.band_limited || c.sx != 0.0 || c.sy != 0.0) return 0;
  return d.col_plan;
}

// launch arguments for chunk [w0, w0 + wc) running on lane `lane`
RowArgs row_args(const dpx_plan* p, const Design& d, int w0, int wc, int lane) {
  RowArgs a{};
  a.wl = d.d_wl;
  a.tw = p->twiddles.at(tw_key(d.M, d.row_plan));
  a.n = d.N;
  a.fov = d.F;
  a.bin = d.b;
  a.layers = d.K;
  a.w_begin = w0;
  a.w_count = wc;
  a.w_per_block = d.w_per_block;
  a.chunk_base = lane * d.slots_per_lane;
  a.spec = spec_of_lane(d, lane);
  const int64_t nn = static_cast<int64_t>(d.N) * d.N;
  a.ckpt_first = d.ck_first;
  if (p->opts.checkpoint_mode == 1) {
    a.ckpt = d.ckpt ? d.ckpt + static_cast<int64_t>(lane) * (d.K - d.ck_first) * d.wl_chunk * nn : nullptr;
    a.ckpt_w_stride = d.wl_chunk;
    a.ofov = d.ofov + static_cast<int64_t>(lane) * d.wl_chunk * d.F * d.F;
  } else {
    a.ckpt = d.ckpt ? d.ckpt + w0 * nn : nullptr;
    a.ckpt_w_stride = d.W;
    a.ofov = d.ofov + static_cast<int64_t>(w0) * d.F * d.F;
  }
  a.dh_part = d.dh_part;
  return a;
}

dpx_status timer_begin(dpx_plan* p, hipStream_t s, TimedLaunch& t) {
  if (!p->timing) return DPX_OK;
  DPX_HIP(hipEventCreate(&t.start));
  DPX_HIP(hipEventCreate(&t.stop));
  DPX_HIP(hipEventRecord(t.start, s));
  return DPX_OK;
}

dpx_status timer_end(dpx_plan* p, hipStream_t s, TimedLaunch& t) {
  if (!p->timing) return DPX_OK;
  DPX_HIP(hipEventRecord(t.stop, s));
  p->pending.push_back(t);
  return DPX_OK;
}

// conventional operation count of one complex transform of length m: 5 m log2 m
double fft_flops(int m) { return 5.0 * m * std::log2(static_cast<double>(m)); }

// algorithmic floating-point work of one launch: transforms at the conventional count plus
// 6 flops per complex product (transmission, transfer function, gradient term)
double row_flops(const Design& d, int mode, int wc, int rows) {
  const double per_row_fft = fft_flops(d.M);
  switch (mode) {
    case dpx::ROW_FWD_FIRST: return static_cast<double>(wc) * rows * (per_row_fft + 6.0 * d.N);
    case dpx::ROW_FWD_MID: return static_cast<double>(wc) * rows * (2 * per_row_fft + 6.0 * d.N);
    case dpx::ROW_FWD_LAST: return static_cast<double>(wc) * rows * per_row_fft;
    case dpx::ROW_ADJ_SEED: return static_cast<double>(wc) * rows * per_row_fft;
    case dpx::ROW_ADJ_MID: return static_cast<double>(wc) * rows * (2 * per_row_fft + 12.0 * d.N);
    case dpx::ROW_ADJ_LAST: return static_cast<double>(wc) * rows * (per_row_fft + 6.0 * d.N);
    case dpx::ROW_ADJ_LAST_U: return static_cast<double>(wc) * rows * (per_row_fft + 12.0 * d.N);
    default: return 0.0;
  }
}

// the last adjoint row pass: rebuilding layer 0's field from u_in and h when it has no
// checkpoint slab
int adj_last_mode(const Design& d) { return d.ck_first ? dpx::ROW_ADJ_LAST_U : dpx::ROW_ADJ_LAST; }

// algorithmic bytes of one row-pass launch (every operand read or written once)
int64_t row_bytes(const Design& d, int mode, int wc, int nwb, bool accumulate, bool has_u) {
  const int64_t nn = static_cast<int64_t>(d.N) * d.N;
  const int64_t row = static_cast<int64_t>(d.M) * 8;  // one spectrum row
  const int64_t fov = static_cast<int64_t>(d.F) * d.F * 8;
  const int64_t part = nwb * nn * 4 * (accumulate ? 2 : 1);
  switch (mode) {
    // the first pass stores no checkpoint (layer 0's is rebuilt, or the pass only carries the
    // input plane to an input gap, reading no heights)
    case dpx::ROW_FWD_FIRST: return wc * d.N * row + (d.z_in > 0.0 ? 0 : 4 * nn) + (has_u ? 8 * nn : 0);
    case dpx::ROW_FWD_MID: return wc * (2 * d.N * row + 8 * nn) + 4 * nn;
    case dpx::ROW_FWD_LAST: return wc * (d.F * row + fov);
    case dpx::ROW_ADJ_SEED: return wc * (fov + 4 * d.T * d.T + d.F * row);
    case dpx::ROW_ADJ_MID: return wc * (2 * d.N * row + 8 * nn) + 4 * nn + part;
    case dpx::ROW_ADJ_LAST: return wc * (d.N * row + 8 * nn) + 4 * nn + part;
    case dpx::ROW_ADJ_LAST_U: return wc * d.N * row + 4 * nn + part + (has_u ? 8 * nn : 0);
    default: return 0;
  }
}

dpx_status run_row(dpx_plan* p, const Design& d, int mode, RowArgs a, int row_lo, int row_hi, hipStream_t s) {
  a.row_lo = row_lo;
  a.row_hi = row_hi;
  const int rg = dpx::row_rows_per_block(d.M, mode);
  const int nrb = (row_hi - row_lo + rg - 1) / rg;
  const int nwb = (a.w_count + d.w_per_block - 1) / d.w_per_block;
  TimedLaunch t{dpx::row_pass_kind(mode), nullptr, nullptr,
                row_bytes(d, mode, a.w_count, nwb, a.accumulate != 0, a.u_in != nullptr),
                row_flops(d, mode, a.w_count, row_hi - row_lo)};
  DPX_TRY(timer_begin(p, s, t));
  hipError_t e = dpx::launch_row(d.M, d.pad, mode, d.row_plan, a, nrb, nwb, s);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "row pass (mode %d) launch failed: %s", mode, hipGetErrorString(e));
  DPX_TRY(timer_end(p, s, t));
  return DPX_OK;
}

ColArgs col_args(const dpx_plan* p, const Design& d, int lane, int layer, int w0, int wc, int in_lo,
                 int in_hi, int out_lo, int out_hi) {
  ColArgs c{};
  c.spec = spec_of_lane(d, lane);
  c.wl = d.d_wl;
  c.tw = nullptr;  // set below, once the transfer-function source is known
  // layer -1: the input gap (no misalignment, transfer function evaluated in the pass)
  const double md = static_cast<double>(d.M) * d.dx;
  c.zrev = (layer < 0 ? d.z_in : d.z[layer] + d.dz[layer]) / md;
  c.sx = layer < 0 ? 0.0 : d.sx[layer] / md;
  c.sy = layer < 0 ? 0.0 : d.sy[layer] / md;
  c.band_limited = d.band ? 1 : 0;
  c.n = d.N;
  c.in_lo = in_lo;
  c.in_hi = in_hi;
  c.out_lo = out_lo;
  c.out_hi = out_hi;
  c.w_begin = w0;
  c.w_count = wc;
  {
    auto it = p->dft.find(d.M * 4 + d.pad);
    c.dft = it == p->dft.end() ? nullptr : it->second;
  }
  // two wavelengths per column block (the second one's rows are prefetched while the first
  // is transformed; measured best of 1, 2, 4, 8 on the large workload) when that still
  // leaves several blocks per CU
  c.col_wpb = (static_cast<int64_t>(wc) * (d.M / 8) >= 2 * 8192) ? 2 : 1;
  const int64_t hs = d.M / 2 + 1;
  c.htab = (d.htab && layer >= 0) ? d.htab + static_cast<int64_t>(d.zslot[layer]) * d.W * hs * hs : nullptr;
  c.tw = p->twiddles.at(tw_key(d.M, col_plan_of(d, c)));
  return c;
}

// algorithmic bytes of a column launch: staged rows in and kept rows out, plus every entry of
// the wavelengths' transfer tables once when the plan has them
int64_t col_bytes(const Design& d, int wc, int in_lo, int in_hi, int out_lo, int out_hi) {
  const int64_t hs = d.M / 2 + 1;
  return static_cast<int64_t>(wc) * d.M * 8 * ((in_hi - in_lo) + (out_hi - out_lo)) +
         (d.htab ? static_cast<int64_t>(wc) * hs * hs * 8 : 0);
}

double col_flops(const Design& d, int wc) {
  return static_cast<double>(wc) * d.M * (2 * fft_flops(d.M) + 6.0 * d.M);
}

dpx_status run_col(dpx_plan* p, const Design& d, int lane, int layer, bool conj, int w0, int wc,
                   int in_lo, int in_hi, int out_lo, int out_hi, hipStream_t s) {
  const ColArgs c = col_args(p, d, lane, layer, w0, wc, in_lo, in_hi, out_lo, out_hi);
  TimedLaunch t{conj ? DPX_PASS_COL_ADJ : DPX_PASS_COL_FWD, nullptr, nullptr,
                col_bytes(d, wc, in_lo, in_hi, out_lo, out_hi), col_flops(d, wc)};
  if (in_lo == 0 && in_hi == d.N && out_lo == 0 && out_hi == d.N)
    t.instance = conj ? DPX_PASS_COL_ADJ_FULL : DPX_PASS_COL_FWD_FULL;
  DPX_TRY(timer_begin(p, s, t));
  hipError_t e = dpx::launch_col(d.M, d.pad, conj, d.col_variant, col_plan_of(d, c), c, wc, s);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "column pass launch failed: %s", hipGetErrorString(e));
  DPX_TRY(timer_end(p, s, t));
  return DPX_OK;
}

int64_t h_off_layer(const Design& d, int l) { return d.h_off + static_cast<int64_t>(l) * d.N * d.N; }

// forward over one chunk of wavelengths [w0, w0 + wc) on lane `lane`; leaves the output
// field in ofov.  `after_first` (may be null) is recorded on s after the first launch.
dpx_status forward_chunk(dpx_plan* p, const Design& d, const float* h, const float* u_in,
                         int w0, int wc, int lane, hipStream_t s, hipEvent_t after_first) {
  const int fo = (d.N - d.F) / 2;
  RowArgs a = row_args(p, d, w0, wc, lane);
  a.u_in = u_in ? reinterpret_cast<const float2*>(u_in) + d.u_off : nullptr;
  a.layer = 0;
  if (d.z_in > 0.0) {
    // input plane: u_in to the spectrum unchanged, across the input gap, then layer 0 as a
    // middle pass (row inverse transform, transmission, checkpoint, row transform)
    a.no_layer = 1;
    a.store_ckpt = 0;
    a.h = nullptr;
    DPX_TRY(run_row(p, d, dpx::ROW_FWD_FIRST, a, 0, d.N, s));
    if (after_first) DPX_HIP(hipEventRecord(after_first, s));
    DPX_TRY(run_col(p, d, lane, -1, false, w0, wc, 0, d.N, 0, d.N, s));
    a.no_layer = 0;
    a.store_ckpt = 1;
    a.h = h + h_off_layer(d, 0);
    DPX_TRY(run_row(p, d, dpx::ROW_FWD_MID, a, 0, d.N, s));
  } else {
    a.store_ckpt = d.ck_first ? 0 : 1;
    a.h = h + h_off_layer(d, 0);
    DPX_TRY(run_row(p, d, dpx::ROW_FWD_FIRST, a, 0, d.N, s));
    if (after_first) DPX_HIP(hipEventRecord(after_first, s));
    a.store_ckpt = 1;
  }
  for (int l = 0; l < d.K; ++l) {
    const bool last = (l == d.K - 1);
    DPX_TRY(run_col(p, d, lane, l, false, w0, wc, 0, d.N, last ? fo : 0, last ? fo + d.F : d.N, s));
    if (!last) {
      a.layer = l + 1;
      a.h = h + h_off_layer(d, l + 1);
      DPX_TRY(run_row(p, d, dpx::ROW_FWD_MID, a, 0, d.N, s));
    } else {
      DPX_TRY(run_row(p, d, dpx::ROW_FWD_LAST, a, fo, fo + d.F, s));
    }
  }
  return DPX_OK;
}

// adjoint over one chunk on lane `lane`; dL/dh partials go to the lane's own slots, added to
// what the lane's earlier chunks left there when `accumulate` is set
dpx_status adjoint_chunk(dpx_plan* p, const Design& d, const float* h, const float* u_in, const float* dl_di,
                         int w0, int wc, int lane, bool accumulate, hipStream_t s,
                         hipEvent_t after_first) {
  const int fo = (d.N - d.F) / 2;
  RowArgs a = row_args(p, d, w0, wc, lane);
  a.u_in = u_in ? reinterpret_cast<const float2*>(u_in) + d.u_off : nullptr;  // rebuilt layer 0
  a.dl_di = dl_di + d.img_off;
  a.store_ckpt = 0;
  a.accumulate = accumulate ? 1 : 0;
  DPX_TRY(run_row(p, d, dpx::ROW_ADJ_SEED, a, fo, fo + d.F, s));
  if (after_first) DPX_HIP(hipEventRecord(after_first, s));
  for (int l = d.K - 1; l >= 0; --l) {
    const bool first = (l == d.K - 1);
    DPX_TRY(run_col(p, d, lane, l, true, w0, wc, first ? fo : 0, first ? fo + d.F : d.N, 0, d.N, s));
    a.layer = l;
    a.h = h + h_off_layer(d, l);
    DPX_TRY(run_row(p, d, l > 0 ? dpx::ROW_ADJ_MID : adj_last_mode(d), a, 0, d.N, s));
  }
  return DPX_OK;
}

// ------------------------------------------------------------------------------------------
// Grouped schedule.  Design i runs the passes FIRST, (column, MID)*, column, LAST forward and
// SEED, (column, ADJ_MID)*, column, ADJ_LAST backward; position k of every design's sequence
// becomes one launch per (transform length, pad, mode or variant), so the passes of all
// designs share launches instead of queueing behind each other.
// ------------------------------------------------------------------------------------------
struct TaskBlob {
  std::vector<char> bytes;
  bool too_many_blocks = false;  // a launch would need more blocks than a grid can hold
  size_t put(const void* src, size_t n) {
    const size_t off = (bytes.size() + 255) / 256 * 256;
    bytes.resize(off + n);
    std::memcpy(bytes.data() + off, src, n);
    return off;
  }
};

// Splits tasks into launches of at most kMaxGroupTasks; each task starts at a multiple of
// `align` blocks.  g.tasks holds the blob offset until the blob is uploaded.
template <typename Task>
void add_group(std::vector<GroupLaunch>& out, const GroupLaunch& proto, const std::vector<Task>& tasks,
               const std::vector<int>& nblocks, const std::vector<int>& align,
               const std::vector<int64_t>& bytes, const std::vector<int64_t>& u_bytes,
               const std::vector<double>& flops, TaskBlob& blob) {
  for (size_t i0 = 0; i0 < tasks.size(); i0 += dpx::kMaxGroupTasks) {
    const size_t n = std::min<size_t>(dpx::kMaxGroupTasks, tasks.size() - i0);
    GroupLaunch L = proto;
    L.g.ntasks = static_cast<int>(n);
    int64_t b = 0;
    for (size_t i = 0; i < n; ++i) {
      const int a = align[i0 + i];
      b = (b + a - 1) / a * a;
      L.g.block0[i] = static_cast<int>(b);
      b += nblocks[i0 + i];
      L.bytes += bytes[i0 + i];
      L.u_bytes += u_bytes[i0 + i];
      L.flops += flops[i0 + i];
    }
    if (b > std::numeric_limits<int>::max()) blob.too_many_blocks = true;
    L.g.block0[n] = static_cast<int>(std::min<int64_t>(b, std::numeric_limits<int>::max()));
    L.g.tasks = reinterpret_cast<const void*>(blob.put(tasks.data() + i0, n * sizeof(Task)));
    out.push_back(L);
  }
}

// Row launches of one position: designs (index, mode, layer, row range) grouped by key.
struct RowItem {
  int design, mode, layer, row_lo, row_hi;
};

void add_row_position(dpx_plan* p, const std::vector<RowItem>& items, std::vector<GroupLaunch>& out,
                      TaskBlob& blob) {
  std::map<std::array<int, 3>, std::vector<RowItem>> by_key;
  for (const auto& it : items) {
    const Design& d = p->designs[it.design];
    by_key[{d.M, d.pad, it.mode}].push_back(it);
  }
  for (const auto& kv : by_key) {
    std::vector<dpx::RowTask> tasks;
    std::vector<int> nb, al;
    std::vector<int64_t> by, ub;
    std::vector<double> fl;
    for (const auto& it : kv.second) {
      const Design& d = p->designs[it.design];
      dpx::RowTask t{};
      t.a = row_args(p, d, 0, d.W, 0);
      t.a.store_ckpt = (it.mode == dpx::ROW_FWD_MID || (it.mode == dpx::ROW_FWD_FIRST && !d.ck_first)) ? 1 : 0;
      t.a.accumulate = 0;
      t.a.layer = it.layer;
      t.a.row_lo = it.row_lo;
      t.a.row_hi = it.row_hi;
      t.h_off = h_off_layer(d, it.layer);
      t.u_off = d.u_off;
      t.img_off = d.img_off;
      const int rg = dpx::row_rows_per_block(d.M, it.mode);
      t.gx = (it.row_hi - it.row_lo + rg - 1) / rg;
      const int nwb = (d.W + d.w_per_block - 1) / d.w_per_block;
      t.nblocks = t.gx * nwb;
      tasks.push_back(t);
      nb.push_back(t.nblocks);
      al.push_back(1);
      by.push_back(row_bytes(d, it.mode, d.W, nwb, false, false));
      const bool reads_u = it.mode == dpx::ROW_FWD_FIRST || it.mode == dpx::ROW_ADJ_LAST_U;
      ub.push_back(reads_u ? 8 * static_cast<int64_t>(d.N) * d.N : 0);
      fl.push_back(row_flops(d, it.mode, d.W, it.row_hi - it.row_lo));
    }
    GroupLaunch proto{};
    proto.kind = GK_ROW;
    proto.M = kv.first[0];
    proto.pad = kv.first[1];
    proto.mode = kv.first[2];
    proto.pass = dpx::row_pass_kind(proto.mode);
    add_group(out, proto, tasks, nb, al, by, ub, fl, blob);
  }
}

// Column launches of one position: (design, layer, input rows, kept rows)
struct ColItem {
  int design, layer, in_lo, in_hi, out_lo, out_hi;
};

void add_col_position(dpx_plan* p, const std::vector<ColItem>& items, bool conj,
                      std::vector<GroupLaunch>& out, TaskBlob& blob) {
  std::map<std::array<int, 5>, std::vector<ColItem>> by_key;
  for (const auto& it : items) {
    const Design& d = p->designs[it.design];
    const bool full = it.in_lo == 0 && it.in_hi == d.N && it.out_lo == 0 && it.out_hi == d.N;
    by_key[{d.M, d.pad, d.col_variant, d.htab ? 1 : 0, full ? 1 : 0}].push_back(it);
  }
  for (const auto& kv : by_key) {
    std::vector<dpx::ColTask> tasks;
    std::vector<int> nb, al;
    std::vector<int64_t> by, ub;
    std::vector<double> fl;
    for (const auto& it : kv.second) {
      const Design& d = p->designs[it.design];
      dpx::ColTask t{};
      t.a = col_args(p, d, 0, it.layer, 0, d.W, it.in_lo, it.in_hi, it.out_lo, it.out_hi);
      t.gx = d.M / dpx::col_tile_width(d.M, d.col_variant);
      t.nblocks = t.gx * ((d.W + t.a.col_wpb - 1) / t.a.col_wpb);
      tasks.push_back(t);
      nb.push_back(t.nblocks);
      // column tiles pair up on an XCD in runs of 16 blocks counted from the task's start
      // (col_block_item), which needs an even tile count
      al.push_back(t.gx % 2 == 0 ? 16 : 1);
      by.push_back(col_bytes(d, d.W, it.in_lo, it.in_hi, it.out_lo, it.out_hi));
      ub.push_back(0);
      fl.push_back(col_flops(d, d.W));
    }
    GroupLaunch proto{};
    proto.kind = GK_COL;
    proto.M = kv.first[0];
    proto.pad = kv.first[1];
    proto.variant = kv.first[2];
    proto.table = kv.first[3] != 0;
    proto.full = kv.first[4] != 0;
    proto.conj = conj;
    proto.pass = conj ? DPX_PASS_COL_ADJ : DPX_PASS_COL_FWD;
    add_group(out, proto, tasks, nb, al, by, ub, fl, blob);
  }
}

template <typename Task>
void add_simple_group(std::vector<GroupLaunch>& out, GroupKind kind, const std::vector<Task>& tasks,
                      const std::vector<int>& nblocks, TaskBlob& blob) {
  GroupLaunch proto{};
  proto.kind = kind;
  const std::vector<int> al(tasks.size(), 1);
  const std::vector<int64_t> z(tasks.size(), 0);
  const std::vector<double> zf(tasks.size(), 0.0);
  add_group(out, proto, tasks, nblocks, al, z, z, zf, blob);
}

// Whether every design can run in the grouped schedule: whole designs in one chunk on one
// lane, stored checkpoints, a transform column variant.
bool groupable(const dpx_plan* p) {
  if (p->opts.checkpoint_mode != 0) return false;
  for (const auto& d : p->designs)
    if (d.nchunks != 1 || d.lanes != 1 || d.col_variant > 3 || d.z_in > 0.0 || d.band || d.row_plan ||
        d.col_plan)
      return false;
  return true;
}

// forward and backward launch lists of the designs `ids`
void build_group_lists(dpx_plan* p, const std::vector<int>& ids, std::vector<GroupLaunch>& fwd,
                       std::vector<GroupLaunch>& bwd, TaskBlob& blob) {
  int kmax = 0;
  for (int i : ids) kmax = std::max(kmax, p->designs[i].K);
  // forward
  for (int j = 0; j <= kmax; ++j) {
    std::vector<RowItem> rows;
    for (int i : ids) {
      const Design& d = p->designs[i];
      if (j > d.K) continue;
      const int fo = (d.N - d.F) / 2;
      if (j == 0) rows.push_back({i, dpx::ROW_FWD_FIRST, 0, 0, d.N});
      else if (j < d.K) rows.push_back({i, dpx::ROW_FWD_MID, j, 0, d.N});
      else rows.push_back({i, dpx::ROW_FWD_LAST, 0, fo, fo + d.F});
    }
    add_row_position(p, rows, fwd, blob);
    if (j == kmax) break;
    std::vector<ColItem> cols;
    for (int i : ids) {
      const Design& d = p->designs[i];
      if (j >= d.K) continue;
      const int fo = (d.N - d.F) / 2;
      const bool last = (j == d.K - 1);
      cols.push_back({i, j, 0, d.N, last ? fo : 0, last ? fo + d.F : d.N});
    }
    add_col_position(p, cols, false, fwd, blob);
  }
  {
    std::vector<dpx::BinTask> bins;
    std::vector<int> nb;
    for (int i : ids) {
      const Design& d = p->designs[i];
      bins.push_back({d.ofov, d.img_off, d.W, d.F, d.b});
      nb.push_back(static_cast<int>((static_cast<int64_t>(d.W) * d.T * d.T + dpx::kGroupThreads - 1) /
                                    dpx::kGroupThreads));
    }
    add_simple_group(fwd, GK_BIN, bins, nb, blob);
  }
  // backward
  {
    std::vector<RowItem> seeds;
    for (int i : ids) {
      const Design& d = p->designs[i];
      const int fo = (d.N - d.F) / 2;
      seeds.push_back({i, dpx::ROW_ADJ_SEED, 0, fo, fo + d.F});
    }
    add_row_position(p, seeds, bwd, blob);
  }
  for (int k = 0; k < kmax; ++k) {
    std::vector<ColItem> cols;
    std::vector<RowItem> rows;
    for (int i : ids) {
      const Design& d = p->designs[i];
      if (k >= d.K) continue;
      const int l = d.K - 1 - k;
      const int fo = (d.N - d.F) / 2;
      cols.push_back({i, l, k == 0 ? fo : 0, k == 0 ? fo + d.F : d.N, 0, d.N});
      rows.push_back({i, l > 0 ? dpx::ROW_ADJ_MID : adj_last_mode(d), l, 0, d.N});
    }
    add_col_position(p, cols, true, bwd, blob);
    add_row_position(p, rows, bwd, blob);
  }
  {
    std::vector<dpx::DhTask> dhs;
    std::vector<int> nb;
    for (int i : ids) {
      const Design& d = p->designs[i];
      const int64_t per = static_cast<int64_t>(d.K) * d.N * d.N;
      dhs.push_back({d.dh_part, d.h_off, per, d.nslots});
      nb.push_back(static_cast<int>((per + dpx::kGroupThreads - 1) / dpx::kGroupThreads));
    }
    add_simple_group(bwd, GK_DH, dhs, nb, blob);
  }
}

dpx_status build_groups(dpx_plan* p) {
  TaskBlob blob;
  const int nd = static_cast<int>(p->designs.size());
  const int parts = std::max(1, p->dstreams);
  p->g_fwd.assign(parts, {});
  p->g_bwd.assign(parts, {});
  for (int k = 0; k < parts; ++k) {
    std::vector<int> ids;
    for (int i = 0; i < nd; ++i)
      if ((p->design_stream.empty() ? 0 : p->design_stream[i]) == k) ids.push_back(i);
    if (!ids.empty()) build_group_lists(p, ids, p->g_fwd[k], p->g_bwd[k], blob);
  }
  // loss: the task array in design order doubles as the table of the per-design sums
  std::vector<dpx::LossTask> losses;
  std::vector<int> lnb;
  for (const auto& d : p->designs) {
    losses.push_back({d.img_off, d.per_wl, d.W, d.T});
    lnb.push_back(d.W);
  }
  add_simple_group(p->g_loss, GK_LOSS, losses, lnb, blob);
  const size_t loss_table = blob.put(losses.data(), losses.size() * sizeof(dpx::LossTask));
  if (blob.too_many_blocks)
    return fail(DPX_E_UNSUPPORTED, "a grouped launch would exceed the grid limit; use schedule 1");
  // upload and turn offsets into device pointers
  const int64_t nbytes = static_cast<int64_t>(blob.bytes.size());
  DPX_TRY(dev_alloc(reinterpret_cast<char**>(&p->d_tasks), nbytes, "grouped-launch tasks"));
  DPX_HIP(hipMemcpy(p->d_tasks, blob.bytes.data(), static_cast<size_t>(nbytes), hipMemcpyHostToDevice));
  p->bytes += nbytes;
  char* base = static_cast<char*>(p->d_tasks);
  auto fix = [&](std::vector<GroupLaunch>& v) {
    for (auto& L : v) L.g.tasks = base + reinterpret_cast<uintptr_t>(L.g.tasks);
  };
  for (auto& v : p->g_fwd) fix(v);
  for (auto& v : p->g_bwd) fix(v);
  fix(p->g_loss);
  p->d_loss_tasks = reinterpret_cast<const dpx::LossTask*>(base + loss_table);
  return DPX_OK;
}

// Enqueues one list of grouped launches on s.  out_f: intensity (binning) or dL/dh (reduction).
dpx_status run_groups(dpx_plan* p, const std::vector<GroupLaunch>& launches, const dpx::CallBuffers& call,
                      float* out_f, hipStream_t s) {
  for (const auto& L : launches) {
    dpx::GroupArgs g = L.g;
    g.call = call;
    TimedLaunch t{L.pass, nullptr, nullptr, L.bytes + (call.u_in ? L.u_bytes : 0), L.flops};
    if (L.kind == GK_COL && L.full) t.instance = L.conj ? DPX_PASS_COL_ADJ_FULL : DPX_PASS_COL_FWD_FULL;
    const bool timed = (L.kind == GK_ROW || L.kind == GK_COL);
    if (timed) DPX_TRY(timer_begin(p, s, t));
    hipError_t e = hipErrorInvalidValue;
    switch (L.kind) {
      case GK_ROW: e = dpx::launch_row_group(L.M, L.pad, L.mode, g, s); break;
      case GK_COL: e = dpx::launch_col_group(L.M, L.pad, L.conj, L.variant, L.table, L.full, g, s); break;
      case GK_BIN: e = dpx::launch_bin_group(g, out_f, s); break;
      case GK_DH: e = dpx::launch_dh_group(g, out_f, s); break;
      case GK_LOSS: break;
    }
    if (e != hipSuccess) return fail(DPX_E_DEVICE, "grouped launch (kind %d, M %d) failed: %s",
                                     static_cast<int>(L.kind), L.M, hipGetErrorString(e));
    if (timed) DPX_TRY(timer_end(p, s, t));
  }
  return DPX_OK;
}

// LDS-resident forward (with the intensity binning) or adjoint (with the dL/dh partials) of a
// whole design in one launch
dpx_status run_lds(dpx_plan* p, const Design& d, bool adjoint, const float* h, const float* u_in,
                   float* intensity, const float* dl_di, hipStream_t s) {
  dpx::LdsArgs a{};
  a.wl = d.d_wl;
  a.tw = p->twiddles.at(tw_key(d.M, 0));
  a.zrev = d.d_zrev;
  a.h = h + d.h_off;
  a.u_in = u_in ? reinterpret_cast<const float2*>(u_in) + d.u_off : nullptr;
  a.ckpt = d.ckpt;
  a.ofov = d.ofov;
  a.intensity = intensity ? intensity + d.img_off : nullptr;
  a.dl_di = dl_di ? dl_di + d.img_off : nullptr;
  a.dh_part = d.dh_part;
  a.K = d.K;
  a.fov = d.F;
  a.bin = d.b;
  a.W = d.W;
  // algorithmic work: every pass of the multi-kernel path, without its spectrum traffic
  double flops = 0.0;
  int64_t bytes = static_cast<int64_t>(d.K) * d.N * d.N * 4 + (u_in ? 8LL * d.N * d.N : 0);
  const int64_t nn = static_cast<int64_t>(d.N) * d.N;
  if (!adjoint) {
    flops += row_flops(d, dpx::ROW_FWD_FIRST, d.W, d.N) + (d.K - 1) * row_flops(d, dpx::ROW_FWD_MID, d.W, d.N) +
             row_flops(d, dpx::ROW_FWD_LAST, d.W, d.F) + d.K * col_flops(d, d.W);
    bytes += static_cast<int64_t>(d.W) * (d.K * nn * 8 + d.F * d.F * 8 + d.T * d.T * 4);
  } else {
    flops += row_flops(d, dpx::ROW_ADJ_SEED, d.W, d.F) + (d.K - 1) * row_flops(d, dpx::ROW_ADJ_MID, d.W, d.N) +
             row_flops(d, dpx::ROW_ADJ_LAST, d.W, d.N) + d.K * col_flops(d, d.W);
    bytes += static_cast<int64_t>(d.W) * (d.K * nn * 8 + d.F * d.F * 8 + d.T * d.T * 4 + d.K * nn * 4);
  }
  TimedLaunch t{adjoint ? DPX_PASS_LDS_ADJ : DPX_PASS_LDS_FWD, nullptr, nullptr, bytes, flops};
  DPX_TRY(timer_begin(p, s, t));
  hipError_t e = dpx::launch_lds(d.M, d.pad, adjoint, a, s);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "LDS-resident pass launch failed: %s", hipGetErrorString(e));
  DPX_TRY(timer_end(p, s, t));
  return DPX_OK;
}

// Chunk c of a design runs on lane c % lanes.  Lane 0 is the caller's stream; the other
// lanes fork from it, start one pass behind lane 0 (so that the column pass of one chunk
// meets the row pass of another), and join back before the call returns.
hipStream_t lane_stream(dpx_plan* p, int lane, hipStream_t s) { return lane == 0 ? s : p->aux[lane - 1]; }

dpx_status fork_lanes(dpx_plan* p, const Design& d, hipStream_t s) {
  if (d.lanes <= 1) return DPX_OK;
  DPX_HIP(hipEventRecord(p->ev_fork, s));
  for (int l = 1; l < d.lanes; ++l) DPX_HIP(hipStreamWaitEvent(p->aux[l - 1], p->ev_fork, 0));
  return DPX_OK;
}

dpx_status join_lanes(dpx_plan* p, const Design& d, hipStream_t s) {
  for (int l = 1; l < d.lanes; ++l) {
    DPX_HIP(hipEventRecord(p->ev_join[l - 1], p->aux[l - 1]));
    DPX_HIP(hipStreamWaitEvent(s, p->ev_join[l - 1], 0));
  }
  return DPX_OK;
}

// Times every column-pass variant on the design's first wavelengths (forward column pass
// of layer 0 on a zeroed spectrum buffer) and keeps the fastest.  All variants produce the
// same bits, so the choice changes speed only.
// Autotuner results: the column variant and the radix plans of a (transform length, pad,
// band-limit flag, timed chunk) key.  Kept per plan creation, and across processes in the text
// file named by the environment variable DPX_TUNE_CACHE when it is set (one line per key:
// "dpx-tune M pad band wc row_plan col_plan col_variant"; lines for lengths, plans or variants
// the library does not have are ignored).
struct TuneChoice {
  int row_plan, col_plan, col_variant;
};
using TuneKey = std::array<int, 4>;

void tune_cache_load(std::map<TuneKey, TuneChoice>& cache) {
  const char* path = std::getenv("DPX_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    int M, pad, band, wc, rp, cp, cv;
    if (std::sscanf(line, "dpx-tune %d %d %d %d %d %d %d", &M, &pad, &band, &wc, &rp, &cp, &cv) != 7) continue;
    const int np = dpx::radix_plan_count(M);
    if (np == 0 || rp < 0 || rp >= np || cp < 0 || cp >= np || !dpx::col_variant_supported(M, pad, cv)) continue;
    cache[{M, pad, band, wc}] = {rp, cp, cv};
  }
  std::fclose(f);
}

void tune_cache_store(const TuneKey& k, const TuneChoice& c) {
  const char* path = std::getenv("DPX_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "dpx-tune %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], c.row_plan, c.col_plan,
               c.col_variant);
  std::fclose(f);
}

// Times the column-pass variants and radix plans, and the radix plans of the middle forward row
// pass, on one chunk of up to 256 of the design's wavelengths (the planes hold zeros; the
// passes' cost does not depend on the values), and keeps the fastest of each that the plan's
// options leave free.  The candidates are timed in three interleaved rounds (three launches
// each) and each keeps its fastest round, so a drift of the clock over the tuning does not
// favour the candidates timed first; differences between candidates are a few per cent.
dpx_status autotune_design(dpx_plan* p, Design& d, std::map<TuneKey, TuneChoice>& cache) {
  const int wc = std::min(std::min(d.W, d.wl_chunk), 256);
  const TuneKey key{d.M, d.pad, d.band ? 1 : 0, wc};
  const bool free_variant = p->opts.force_variant < 0;
  const bool free_plan = p->opts.force_plan < 0 && !p->grouped && !d.band && !d.htab && !d.lds;
  auto it = cache.find(key);
  if (it != cache.end()) {
    if (free_variant) d.col_variant = it->second.col_variant;
    if (free_plan) {
      d.row_plan = it->second.row_plan;
      d.col_plan = it->second.col_plan;
    }
    return DPX_OK;
  }
  DPX_HIP(hipMemset(d.spec, 0, static_cast<size_t>(wc) * d.N * d.M * 8));
  hipEvent_t e0, e1;
  DPX_HIP(hipEventCreate(&e0));
  DPX_HIP(hipEventCreate(&e1));
  const bool was_timing = p->timing;
  p->timing = false;
  auto time_it = [&](auto&& launch, float& ms) -> dpx_status {
    DPX_HIP(hipEventRecord(e0, nullptr));
    for (int r = 0; r < 3; ++r) DPX_TRY(launch());
    DPX_HIP(hipEventRecord(e1, nullptr));
    DPX_HIP(hipEventSynchronize(e1));
    DPX_HIP(hipEventElapsedTime(&ms, e0, e1));
    return DPX_OK;
  };
  const int nplans = free_plan ? dpx::radix_plan_count(d.M) : 1;
  TuneChoice pick{d.row_plan, d.col_plan, d.col_variant};
  // column pass: every (radix plan, variant) left free
  std::vector<std::array<int, 2>> cand;
  for (int cp = 0; cp < nplans; ++cp)
    for (int v = 0; v < dpx::kColVariants; ++v) {
      if (!free_variant && v != d.col_variant) continue;
      if (!dpx::col_variant_supported(d.M, d.pad, v)) continue;
      if (v == 4 && (!p->dft.count(d.M * 4 + d.pad) || cp > 0)) continue;  // the matrix form has no radix plan
      if (d.band && v > 1) continue;
      cand.push_back({free_plan ? cp : d.col_plan, v});
    }
  std::vector<float> best(cand.size(), 1e30f);
  for (int round = 0; round < 4; ++round)   // round 0 warms every candidate up
    for (size_t c = 0; c < cand.size(); ++c) {
      d.col_plan = cand[c][0];
      d.col_variant = cand[c][1];
      float ms = 0.f;
      DPX_TRY(time_it([&]() { return run_col(p, d, 0, 0, false, 0, wc, 0, d.N, 0, d.N, nullptr); }, ms));
      if (round > 0) best[c] = std::min(best[c], ms);
    }
  {
    const size_t c = static_cast<size_t>(std::min_element(best.begin(), best.end()) - best.begin());
    pick.col_plan = cand[c][0];
    pick.col_variant = cand[c][1];
  }
  d.col_variant = pick.col_variant;
  d.col_plan = pick.col_plan;
  // row passes: the middle forward pass (heights of zero, no checkpoints) on every radix plan
  if (free_plan && nplans > 1) {
    float* hz = nullptr;
    DPX_TRY(dev_alloc(&hz, static_cast<int64_t>(d.N) * d.N * 4, "autotuner heights"));
    dpx_status st = hipMemset(hz, 0, static_cast<size_t>(d.N) * d.N * 4) == hipSuccess
                        ? DPX_OK : fail(DPX_E_DEVICE, "autotuner height clearing failed");
    RowArgs a = row_args(p, d, 0, wc, 0);
    a.h = hz;
    a.store_ckpt = 0;
    a.layer = 1;
    std::vector<float> rbest(nplans, 1e30f);
    for (int round = 0; round < 4 && st == DPX_OK; ++round)
      for (int rp = 0; rp < nplans && st == DPX_OK; ++rp) {
        d.row_plan = rp;
        a.tw = p->twiddles.at(tw_key(d.M, rp));
        float ms = 0.f;
        st = time_it([&]() { return run_row(p, d, dpx::ROW_FWD_MID, a, 0, d.N, nullptr); }, ms);
        if (round > 0) rbest[rp] = std::min(rbest[rp], ms);
      }
    (void)hipDeviceSynchronize();
    hipFree(hz);
    DPX_TRY(st);
    pick.row_plan = static_cast<int>(std::min_element(rbest.begin(), rbest.end()) - rbest.begin());
  }
  d.row_plan = pick.row_plan;
  p->timing = was_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cache[key] = pick;
  tune_cache_store(key, pick);
  return DPX_OK;
}

// Runs fn(design, stream) for every design: on the caller's stream, or with several
// independent designs spread over the plan's streams (forked from and joined back to s).
template <typename F>
dpx_status for_each_design(dpx_plan* p, hipStream_t s, F&& fn) {
  if (p->dstreams <= 1) {
    for (size_t i = 0; i < p->designs.size(); ++i) DPX_TRY(fn(p->designs[i], static_cast<int>(i), s));
    return DPX_OK;
  }
  DPX_HIP(hipEventRecord(p->ev_fork, s));
  for (int k = 1; k < p->dstreams; ++k) DPX_HIP(hipStreamWaitEvent(p->aux[k - 1], p->ev_fork, 0));
  for (size_t i = 0; i < p->designs.size(); ++i) {
    const int k = p->design_stream[i];
    DPX_TRY(fn(p->designs[i], static_cast<int>(i), k == 0 ? s : p->aux[k - 1]));
  }
  for (int k = 1; k < p->dstreams; ++k) {
    DPX_HIP(hipEventRecord(p->ev_join[k - 1], p->aux[k - 1]));
    DPX_HIP(hipStreamWaitEvent(s, p->ev_join[k - 1], 0));
  }
  return DPX_OK;
}

// Runs the grouped launch lists of every partition, partition k on stream k (forked from and
// joined back to s).
dpx_status run_group_parts(dpx_plan* p, const std::vector<std::vector<GroupLaunch>>& parts,
                           const dpx::CallBuffers& call, float* out_f, hipStream_t s) {
  const int n = static_cast<int>(parts.size());
  if (n <= 1) return n == 1 ? run_groups(p, parts[0], call, out_f, s) : DPX_OK;
  DPX_HIP(hipEventRecord(p->ev_fork, s));
  for (int k = 1; k < n; ++k) DPX_HIP(hipStreamWaitEvent(p->aux[k - 1], p->ev_fork, 0));
  for (int k = 0; k < n; ++k) DPX_TRY(run_groups(p, parts[k], call, out_f, k == 0 ? s : p->aux[k - 1]));
  for (int k = 1; k < n; ++k) {
    DPX_HIP(hipEventRecord(p->ev_join[k - 1], p->aux[k - 1]));
    DPX_HIP(hipStreamWaitEvent(s, p->ev_join[k - 1], 0));
  }
  return DPX_OK;
}

constexpr size_t kMaxGraphs = 16;

// Runs `enqueue` on the caller's stream, or (opts.use_graph, timers off) replays a graph of
// it captured on the first call with the same key.
template <typename F>
dpx_status run_graph_or_eager(dpx_plan* p, const std::array<uintptr_t, 5>& key, hipStream_t s,
                              F&& enqueue) {
  if (!p->opts.use_graph || p->timing) return enqueue(s);
  DPX_HIP(hipEventRecord(p->ev_gin, s));
  DPX_HIP(hipStreamWaitEvent(p->gstream, p->ev_gin, 0));
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    if (p->graphs.size() >= kMaxGraphs) {
      auto old = p->graphs.find(p->graph_order.front());
      if (old != p->graphs.end()) {
        (void)hipGraphExecDestroy(old->second);
        p->graphs.erase(old);
      }
      p->graph_order.erase(p->graph_order.begin());
    }
    DPX_HIP(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeRelaxed));
    const dpx_status st = enqueue(p->gstream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gstream, &g);
    if (st != DPX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(DPX_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(DPX_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    it = p->graphs.emplace(key, ex).first;
    p->graph_order.push_back(key);
  }
  DPX_HIP(hipGraphLaunch(it->second, p->gstream));
  DPX_HIP(hipEventRecord(p->ev_gout, p->gstream));
  DPX_HIP(hipStreamWaitEvent(s, p->ev_gout, 0));
  return DPX_OK;
}

template <typename... T>
std::array<uintptr_t, 5> graph_key(uintptr_t kind, T... ptrs) {
  std::array<uintptr_t, 5> k{kind, reinterpret_cast<uintptr_t>(ptrs)...};
  return k;
}

}  // namespace

extern "C" {

void dpx_opts_default(dpx_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->checkpoint_mode = 0;
  o->wl_chunk = 0;
  o->use_graph = 0;
  o->autotune = 0;
  o->force_variant = -1;
  o->transfer_table = 0;
  o->small_path = 0;
  o->max_workspace_bytes = 0;
  o->force_plan = -1;
}

const char* dpx_last_error(void) { return g_last_error.c_str(); }

const char* dpx_version(void) { return "dpx 0.1 (gfx950)"; }

int32_t dpx_variant_count(void) { return dpx::kColVariants; }

const char* dpx_variant_name(int32_t v) {
  return (v >= 0 && v < dpx::kColVariants) ? dpx::kColVariantNames[v] : "";
}

dpx_status dpx_plan_variant(const dpx_plan* p, int32_t i, int32_t* variant) {
  if (!p || !variant) return fail(DPX_E_ARG, "plan and variant must not be NULL");
  if (i < 0 || i >= static_cast<int>(p->designs.size()))
    return fail(DPX_E_ARG, "design index %d out of range", i);
  *variant = p->designs[i].col_variant;
  return ok();
}

int32_t dpx_radix_plan_count(int32_t M) { return dpx::radix_plan_count(M); }

const char* dpx_radix_plan_name(int32_t M, int32_t plan) { return dpx::radix_plan_name(M, plan); }

dpx_status dpx_plan_radix(const dpx_plan* p, int32_t i, int32_t* row_plan, int32_t* col_plan) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  if (i < 0 || i >= static_cast<int>(p->designs.size())) return fail(DPX_E_ARG, "design index %d out of range", i);
  if (row_plan) *row_plan = p->designs[i].row_plan;
  if (col_plan) *col_plan = p->designs[i].col_plan;
  return ok();
}

dpx_status dpx_plan_schedule(const dpx_plan* p, int32_t* schedule) {
  if (!p || !schedule) return fail(DPX_E_ARG, "plan and schedule must not be NULL");
  *schedule = p->grouped ? 2 : 1;
  return ok();
}

dpx_status dpx_plan_query(const dpx_design* ds, int32_t nd, const dpx_opts* opts, int64_t* bytes) {
  dpx_opts o;
  dpx_opts_default(&o);
  if (opts) o = *opts;
  DPX_TRY(validate(ds, nd, opts ? &o : nullptr));
  if (!bytes) return fail(DPX_E_ARG, "workspace_bytes is NULL");
  int64_t tot = 0;
  std::map<int, int> ms;
  bool groupable_all = o.checkpoint_mode == 0;
  for (int i = 0; i < nd; ++i) {
    Design d;
    layout_design(ds[i], o, d);
    tot += d.bytes;
    ms[d.M] = 1;
    groupable_all = groupable_all && d.nchunks == 1 && d.lanes == 1 && d.col_variant <= 3 && d.z_in == 0.0 &&
                    !d.band;
  }
  if (o.schedule == 2 && !groupable_all)
    return fail(DPX_E_UNSUPPORTED,
                "the grouped schedule needs checkpoint_mode 0, every design in one wavelength chunk "
                "on one stream, and a transform column variant (0-3)");
  for (auto& kv : ms) tot += static_cast<int64_t>(kv.first) * 8;
  *bytes = tot;
  return ok();
}

namespace {

// Per-wavelength constants of Eq. 1 and Eq. 4 (double precision on the host) to the device
// table, and the transfer tables rebuilt from them when the plan keeps tables.  Synchronous.
dpx_status upload_wavelengths(Design& d) {
  std::vector<WlConst> tab(d.W);
  const double md = static_cast<double>(d.M) * d.dx;
  for (int w = 0; w < d.W; ++w) {
    const double lam = d.wl[w];
    tab[w].rt = (d.n_mat[w] - d.n_m) / lam;
    tab[w].ca = kTwoPi * d.kappa[w] / lam;
    const double r = md * d.n_m / lam;
    tab[w].q0 = r * r;
    tab[w].ct = kTwoPi * (d.n_mat[w] - d.n_m) / lam;
  }
  if (hipMemcpy(d.d_wl, tab.data(), d.W * sizeof(WlConst), hipMemcpyHostToDevice) != hipSuccess)
    return fail(DPX_E_DEVICE, "copy of the wavelength table failed");
  for (int k = 0; k < d.nzslots; ++k) {
    int l = 0;
    while (d.zslot[l] != k) ++l;
    const int64_t hs = d.M / 2 + 1;
    const hipError_t e = dpx::launch_transfer_table(d.M, d.d_wl, d.W, d.z[l] / (static_cast<double>(d.M) * d.dx),
                                                    d.htab + static_cast<int64_t>(k) * d.W * hs * hs, nullptr);
    if (e != hipSuccess) return fail(DPX_E_DEVICE, "transfer table launch failed: %s", hipGetErrorString(e));
  }
  if (d.nzslots > 0 && hipDeviceSynchronize() != hipSuccess)
    return fail(DPX_E_DEVICE, "transfer table build failed");
  return DPX_OK;
}

}  // namespace

dpx_status dpx_plan_create(const dpx_design* ds, int32_t nd, const dpx_opts* opts, dpx_plan** out) {
  if (!out) return fail(DPX_E_ARG, "out is NULL");
  *out = nullptr;
  dpx_opts o;
  dpx_opts_default(&o);
  if (opts) o = *opts;
  DPX_TRY(validate(ds, nd, &o));
  int64_t need = 0;
  DPX_TRY(dpx_plan_query(ds, nd, &o, &need));
  if (o.max_workspace_bytes > 0 && need > o.max_workspace_bytes)
    return fail(DPX_E_NOMEM, "plan needs %lld device bytes, limit is %lld", static_cast<long long>(need),
                static_cast<long long>(o.max_workspace_bytes));

  dpx_plan* p = new dpx_plan();
  p->opts = o;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(DPX_E_DEVICE, "no HIP device");
  }
  int64_t h_off = 0, u_off = 0, img_off = 0;
  p->designs.resize(nd);
  dpx_status st = DPX_OK;
  for (int i = 0; i < nd && st == DPX_OK; ++i) {
    const dpx_design& src = ds[i];
    Design& d = p->designs[i];
    layout_design(src, o, d);
    d.wl.assign(src.wl, src.wl + src.n_wl);
    d.n_mat.assign(src.n_mat, src.n_mat + src.n_wl);
    d.kappa.assign(src.n_wl, 0.0);
    if (src.kappa) d.kappa.assign(src.kappa, src.kappa + src.n_wl);
    d.z.assign(src.z, src.z + src.layers);
    d.dz.assign(src.layers, 0.0);
    d.sx.assign(src.layers, 0.0);
    d.sy.assign(src.layers, 0.0);
    d.h_off = h_off;
    d.u_off = u_off;
    d.img_off = img_off;
    h_off += static_cast<int64_t>(d.K) * d.N * d.N;
    u_off += static_cast<int64_t>(d.N) * d.N;
    img_off += static_cast<int64_t>(d.W) * d.T * d.T;
    const int64_t nn = static_cast<int64_t>(d.N) * d.N;
    const int ck_w = (o.checkpoint_mode == 1) ? d.lanes * d.wl_chunk : d.W;
    if ((st = dev_alloc(&d.d_wl, d.W * sizeof(WlConst), "wavelength table")) != DPX_OK) break;
    if ((st = dev_alloc(&d.spec, static_cast<int64_t>(d.lanes) * d.wl_chunk * d.N * d.M * 8, "spectra")) != DPX_OK) break;
    if ((st = dev_alloc(&d.ckpt, static_cast<int64_t>(d.K - d.ck_first) * ck_w * nn * 8, "checkpoints")) != DPX_OK) break;
    if ((st = dev_alloc(&d.ofov, static_cast<int64_t>(ck_w) * d.F * d.F * 8, "output field")) != DPX_OK) break;
    if ((st = dev_alloc(&d.dh_part, static_cast<int64_t>(d.nslots) * d.K * nn * 4, "gradient partials")) != DPX_OK) break;
    if ((st = dev_alloc(&d.per_wl, d.W * 8, "per-wavelength loss")) != DPX_OK) break;
    if ((st = dev_alloc(&d.htab, d.table_bytes, "transfer tables")) != DPX_OK) break;
    if ((st = dev_alloc(&d.d_zrev, static_cast<int64_t>(d.K) * 8, "gap table")) != DPX_OK) break;
    {
      std::vector<double> zr(d.K);
      for (int l = 0; l < d.K; ++l) zr[l] = d.z[l] / (static_cast<double>(d.M) * d.dx);
      if (hipMemcpy(d.d_zrev, zr.data(), d.K * 8, hipMemcpyHostToDevice) != hipSuccess) {
        st = fail(DPX_E_DEVICE, "copy of the gap table failed");
        break;
      }
    }
    p->bytes += d.bytes;
    if ((st = upload_wavelengths(d)) != DPX_OK) break;
    // the twiddle tables of every radix plan of the length (a few KB each): the autotuner and
    // a column pass falling back to plan 0 may use any of them
    for (int pl = 0; pl < dpx::radix_plan_count(d.M) && st == DPX_OK; ++pl) {
      if (p->twiddles.count(tw_key(d.M, pl))) continue;
      std::vector<float2> tw;
      dpx::build_twiddle_table(d.M, pl, tw);
      float2* dtw = nullptr;
      const int64_t tb = static_cast<int64_t>(tw.size()) * 8;
      if ((st = dev_alloc(&dtw, tb, "twiddles")) != DPX_OK) break;
      p->twiddles[tw_key(d.M, pl)] = dtw;
      if (hipMemcpy(dtw, tw.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
        st = fail(DPX_E_DEVICE, "copy of the twiddle table failed");
        break;
      }
      p->bytes += tb;
    }
    if (st != DPX_OK) break;
    if (o.force_plan >= 0) d.row_plan = d.col_plan = o.force_plan;
  }
  for (const auto& d : p->designs) {
    p->h_total += static_cast<int64_t>(d.K) * d.N * d.N;
    p->img_total += static_cast<int64_t>(d.W) * d.T * d.T;
  }
  if (st == DPX_OK && o.check_finite) st = dev_alloc(&p->d_nonfinite, 256, "non-finite counters");
  // grouped schedule: asked for, or automatic for several designs whose wavelengths are not
  // split over chunk lanes (the grouped lists of up to four design partitions then run side by
  // side, like single designs)
  const bool try_group = o.schedule == 2 || (o.schedule == 0 && nd > 1 && o.streams <= 1);
  if (st == DPX_OK && try_group) {
    p->grouped = groupable(p);
    if (p->grouped)
      for (auto& d : p->designs) d.lds = false;  // the grouped launches take every design
    if (!p->grouped && o.schedule == 2)
      st = fail(DPX_E_UNSUPPORTED,
                "the grouped schedule needs checkpoint_mode 0, every design in one wavelength chunk "
                "on one stream, and a transform column variant (0-3)");
  }
  if (st == DPX_OK) {
    int max_lanes = 1;
    for (const auto& d : p->designs) max_lanes = std::max(max_lanes, d.lanes);
    // several independent designs (each on one lane) run side by side on up to four streams,
    // assigned longest-first to the least loaded stream by their W K M N cost
    if (nd > 1 && max_lanes == 1 && o.streams != 1) {
      p->dstreams = std::min(nd, o.streams > 1 ? o.streams : 4);
      std::vector<int> order(nd);
      for (int i = 0; i < nd; ++i) order[i] = i;
      auto cost = [&](int i) {
        const Design& d = p->designs[i];
        return static_cast<double>(d.W) * d.K * d.M * d.N;
      };
      std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
      std::vector<double> load(p->dstreams, 0.0);
      p->design_stream.assign(nd, 0);
      for (int i : order) {
        const int k = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        p->design_stream[i] = k;
        load[k] += cost(i);
      }
      max_lanes = std::max(max_lanes, p->dstreams);
    }
    if (hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_offset, hipEventDisableTiming) != hipSuccess) {
      st = fail(DPX_E_DEVICE, "event creation failed");
    }
    for (int l = 1; l < max_lanes && st == DPX_OK; ++l) {
      hipStream_t q = nullptr;
      hipEvent_t e = nullptr;
      // default priority, non-blocking with respect to the legacy default stream
      if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        st = fail(DPX_E_DEVICE, "stream creation failed");
        break;
      }
      p->aux.push_back(q);
      p->ev_join.push_back(e);
    }
  }
  if (st == DPX_OK && (o.force_variant == 4 || o.autotune)) {
    for (const auto& d : p->designs) {
      const int key = d.M * 4 + d.pad;
      if (p->dft.count(key) || !dpx::col_variant_supported(d.M, d.pad, 4)) continue;
      std::vector<float2> tab;
      dpx::build_dft_table(d.M, d.pad, tab);
      float2* dt = nullptr;
      const int64_t tb = static_cast<int64_t>(tab.size()) * 8;
      if ((st = dev_alloc(&dt, tb, "DFT matrices")) != DPX_OK) break;
      p->dft[key] = dt;
      if (hipMemcpy(dt, tab.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
        st = fail(DPX_E_DEVICE, "copy of the DFT matrices failed");
        break;
      }
      p->bytes += tb;
    }
  }
  if (st == DPX_OK && o.use_graph) {
    if (hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_gin, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_gout, hipEventDisableTiming) != hipSuccess)
      st = fail(DPX_E_DEVICE, "graph stream creation failed");
  }
  if (st == DPX_OK && o.autotune && (o.force_variant < 0 || o.force_plan < 0)) {
    std::map<TuneKey, TuneChoice> cache;
    tune_cache_load(cache);
    for (auto& d : p->designs)
      if ((st = autotune_design(p, d, cache)) != DPX_OK) break;
  }
  if (st == DPX_OK && p->grouped) {
    // the autotuner may have picked the matrix-core column pass, which has no grouped form
    if (groupable(p)) st = build_groups(p);
    else p->grouped = false;
  }
  if (st != DPX_OK) {
    std::string msg = g_last_error;
    dpx_plan_destroy(p);
    g_last_error = msg;
    return st;
  }
  *out = p;
  return ok();
}

dpx_status dpx_plan_destroy(dpx_plan* p) {
  if (!p) return ok();
  (void)hipDeviceSynchronize();
  for (auto& t : p->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto& d : p->designs) free_design(d);
  for (auto& kv : p->twiddles) hipFree(kv.second);
  for (auto& kv : p->dft) hipFree(kv.second);
  if (p->d_tasks) hipFree(p->d_tasks);
  if (p->d_nonfinite) hipFree(p->d_nonfinite);
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->gstream) (void)hipStreamDestroy(p->gstream);
  if (p->ev_gin) (void)hipEventDestroy(p->ev_gin);
  if (p->ev_gout) (void)hipEventDestroy(p->ev_gout);
  for (auto q : p->aux) (void)hipStreamDestroy(q);
  for (auto e : p->ev_join) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_offset) (void)hipEventDestroy(p->ev_offset);
  delete p;
  return ok();
}

dpx_status dpx_plan_layout(const dpx_plan* p, int32_t i, dpx_layout* out) {
  if (!p || !out) return fail(DPX_E_ARG, "plan and out must not be NULL");
  if (i < 0 || i >= static_cast<int>(p->designs.size()))
    return fail(DPX_E_ARG, "design index %d out of range", i);
  const Design& d = p->designs[i];
  out->h_offset = d.h_off;
  out->h_count = static_cast<int64_t>(d.K) * d.N * d.N;
  out->u_offset = d.u_off;
  out->u_count = static_cast<int64_t>(d.N) * d.N;
  out->img_offset = d.img_off;
  out->img_count = static_cast<int64_t>(d.W) * d.T * d.T;
  out->transform_len = d.M;
  out->target_side = d.T;
  out->workspace_bytes = d.bytes;
  out->transfer_tables = d.nzslots;
  out->lds_path = d.lds ? 1 : 0;
  return ok();
}

dpx_status dpx_plan_set_wavelengths(dpx_plan* p, int32_t i, const double* wl, const double* n_mat,
                                    const double* kappa, int32_t n_wl) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  if (i < 0 || i >= static_cast<int>(p->designs.size()))
    return fail(DPX_E_ARG, "design index %d out of range", i);
  Design& d = p->designs[i];
  if (n_wl != d.W)
    return fail(DPX_E_ARG, "design %d: n_wl must stay %d (got %d): the workspace is sized for it", i, d.W, n_wl);
  DPX_TRY(check_wavelengths(i, wl, n_mat, kappa, n_wl));
  // every pass reads the table: let work already queued finish before it changes
  if (hipDeviceSynchronize() != hipSuccess) return fail(DPX_E_DEVICE, "device synchronisation failed");
  d.wl.assign(wl, wl + n_wl);
  d.n_mat.assign(n_mat, n_mat + n_wl);
  if (kappa)
    d.kappa.assign(kappa, kappa + n_wl);
  else
    d.kappa.assign(n_wl, 0.0);
  DPX_TRY(upload_wavelengths(d));
  // store-mode checkpoints of an earlier forward belong to the old wavelengths
  p->fwd_valid = false;
  return ok();
}

dpx_status dpx_plan_set_misalignment(dpx_plan* p, int32_t i, const double* dz, const double* shift_x,
                                     const double* shift_y, int32_t n_gaps) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  if (i < 0 || i >= static_cast<int>(p->designs.size()))
    return fail(DPX_E_ARG, "design index %d out of range", i);
  Design& d = p->designs[i];
  if (n_gaps != d.K) return fail(DPX_E_ARG, "design %d: n_gaps must be %d (got %d)", i, d.K, n_gaps);
  std::vector<double> nz(d.K, 0.0), nx(d.K, 0.0), ny(d.K, 0.0);
  bool any = false, lateral = false;
  for (int l = 0; l < d.K; ++l) {
    if (dz) nz[l] = dz[l];
    if (shift_x) nx[l] = shift_x[l];
    if (shift_y) ny[l] = shift_y[l];
    if (!(std::isfinite(nz[l]) && std::isfinite(nx[l]) && std::isfinite(ny[l])))
      return fail(DPX_E_ARG, "design %d: misalignment of gap %d is not finite", i, l);
    if (!(d.z[l] + nz[l] >= 0.0))
      return fail(DPX_E_ARG, "design %d: gap %d would be negative (z %g + dz %g)", i, l, d.z[l], nz[l]);
    any = any || nz[l] != 0.0 || nx[l] != 0.0 || ny[l] != 0.0;
    lateral = lateral || nx[l] != 0.0 || ny[l] != 0.0;
  }
  if (any && (p->grouped || d.lds || d.nzslots > 0))
    return fail(DPX_E_UNSUPPORTED,
                "design %d: a misalignment needs the per-design schedule with the transfer function "
                "evaluated in the column pass (no grouped schedule, LDS-resident path or tables)", i);
  if (lateral && d.col_variant == 4)
    return fail(DPX_E_UNSUPPORTED, "design %d: the matrix-core column variant has no lateral translation", i);
  if (lateral && d.band)
    return fail(DPX_E_UNSUPPORTED, "design %d: no lateral translation with the band-limited spectrum", i);
  // captured graphs hold the old kernel arguments
  if (!p->graphs.empty()) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(DPX_E_DEVICE, "device synchronisation failed");
    for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    p->graph_order.clear();
  }
  d.dz = nz;
  d.sx = nx;
  d.sy = ny;
  // store-mode checkpoints of an earlier forward belong to the old transfer functions
  p->fwd_valid = false;
  return ok();
}

dpx_status dpx_plan_sizes(const dpx_plan* p, int64_t* h_count, int64_t* u_count, int64_t* img_count) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  int64_t hc = 0, uc = 0, ic = 0;
  for (const auto& d : p->designs) {
    hc += static_cast<int64_t>(d.K) * d.N * d.N;
    uc += static_cast<int64_t>(d.N) * d.N;
    ic += static_cast<int64_t>(d.W) * d.T * d.T;
  }
  if (h_count) *h_count = hc;
  if (u_count) *u_count = uc;
  if (img_count) *img_count = ic;
  return ok();
}

dpx_status dpx_forward(dpx_plan* p, const float* h, const float* u_in, float* intensity, void* stream) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  DPX_TRY(check_ptr(h, 4, "h"));
  DPX_TRY(check_ptr(intensity, 4, "intensity"));
  if (u_in) DPX_TRY(check_ptr(u_in, 8, "u_in"));
  DPX_TRY(sticky_check());
  hipStream_t caller = static_cast<hipStream_t>(stream);
  p->fwd_valid = false;
  auto enqueue = [&](hipStream_t s0) -> dpx_status {
    if (p->grouped)
      return run_group_parts(p, p->g_fwd, {h, reinterpret_cast<const float2*>(u_in), nullptr}, intensity, s0);
    return for_each_design(p, s0, [&](const Design& d, int, hipStream_t s) -> dpx_status {
      if (d.lds) return run_lds(p, d, false, h, u_in, intensity, nullptr, s);
      DPX_TRY(fork_lanes(p, d, s));
      for (int c = 0; c < d.nchunks; ++c) {
        const int lane = c % d.lanes;
        const int w0 = c * d.wl_chunk;
        const int wc = std::min(d.wl_chunk, d.W - w0);
        hipStream_t ls = lane_stream(p, lane, s);
        if (lane == 1 && c == 1) DPX_HIP(hipStreamWaitEvent(ls, p->ev_offset, 0));
        DPX_TRY(forward_chunk(p, d, h, u_in, w0, wc, lane, ls,
                              (c == 0 && d.lanes > 1) ? p->ev_offset : nullptr));
        const float2* of = (p->opts.checkpoint_mode == 1)
                               ? d.ofov + static_cast<int64_t>(lane) * d.wl_chunk * d.F * d.F
                               : d.ofov + static_cast<int64_t>(w0) * d.F * d.F;
        hipError_t e = dpx::launch_bin_intensity(
            of, intensity + d.img_off + static_cast<int64_t>(w0) * d.T * d.T, wc, d.F, d.b, ls);
        if (e != hipSuccess) return fail(DPX_E_DEVICE, "intensity launch failed: %s", hipGetErrorString(e));
      }
      return join_lanes(p, d, s);
    });
  };
  DPX_TRY(run_graph_or_eager(p, graph_key(1, h, u_in, intensity, nullptr), caller, enqueue));
  p->fwd_valid = (p->opts.checkpoint_mode == 0);
  p->last_h = h;
  p->last_u = u_in;
  DPX_TRY(check_outputs(p, {{intensity, p->img_total, false, "intensity"}}, caller));
  return ok();
}

dpx_status dpx_loss(dpx_plan* p, const float* intensity, const float* target, double* loss, float* dl_di,
                    void* stream) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  DPX_TRY(check_ptr(intensity, 4, "intensity"));
  DPX_TRY(check_ptr(target, 4, "target"));
  DPX_TRY(check_ptr(loss, 8, "loss"));
  if (dl_di) DPX_TRY(check_ptr(dl_di, 4, "dl_di"));
  DPX_TRY(sticky_check());
  hipStream_t caller = static_cast<hipStream_t>(stream);
  auto enqueue = [&](hipStream_t s0) -> dpx_status {
    if (p->grouped) {
      for (const auto& L : p->g_loss) {
        hipError_t e = dpx::launch_loss_group(L.g, intensity, target, dl_di, s0);
        if (e != hipSuccess) return fail(DPX_E_DEVICE, "loss launch failed: %s", hipGetErrorString(e));
      }
      hipError_t e = dpx::launch_loss_sum_group(p->d_loss_tasks, static_cast<int>(p->designs.size()), loss, s0);
      if (e != hipSuccess) return fail(DPX_E_DEVICE, "loss launch failed: %s", hipGetErrorString(e));
      return DPX_OK;
    }
    return for_each_design(p, s0, [&](const Design& d, int i, hipStream_t s) -> dpx_status {
      hipError_t e = dpx::launch_loss(intensity + d.img_off, target + d.img_off,
                                      dl_di ? dl_di + d.img_off : nullptr, d.per_wl, d.W, d.T, s);
      if (e == hipSuccess) e = dpx::launch_loss_sum(d.per_wl, loss + i, d.W, s);
      if (e != hipSuccess) return fail(DPX_E_DEVICE, "loss launch failed: %s", hipGetErrorString(e));
      return DPX_OK;
    });
  };
  DPX_TRY(run_graph_or_eager(p, graph_key(2, intensity, target, loss, dl_di), caller, enqueue));
  DPX_TRY(check_outputs(p,
                        {{loss, static_cast<int64_t>(p->designs.size()), true, "loss"},
                         {dl_di, p->img_total, false, "dl_di"}},
                        caller));
  return ok();
}

dpx_status dpx_backward(dpx_plan* p, const float* h, const float* u_in, const float* dl_di, float* dl_dh,
                        void* stream) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  DPX_TRY(check_ptr(h, 4, "h"));
  DPX_TRY(check_ptr(dl_di, 4, "dl_di"));
  DPX_TRY(check_ptr(dl_dh, 4, "dl_dh"));
  if (u_in) DPX_TRY(check_ptr(u_in, 8, "u_in"));
  DPX_TRY(sticky_check());
  const bool store = (p->opts.checkpoint_mode == 0);
  if (store && !(p->fwd_valid && p->last_h == h && p->last_u == u_in))
    return fail(DPX_E_STATE,
                "store-mode backward needs a preceding dpx_forward on this plan with the same h and "
                "u_in");
  hipStream_t caller = static_cast<hipStream_t>(stream);
  auto enqueue = [&](hipStream_t s0) -> dpx_status {
    if (p->grouped)
      return run_group_parts(p, p->g_bwd, {h, reinterpret_cast<const float2*>(u_in), dl_di}, dl_dh, s0);
    return for_each_design(p, s0, [&](const Design& d, int, hipStream_t s) -> dpx_status {
      if (d.lds) {
        DPX_TRY(run_lds(p, d, true, h, u_in, nullptr, dl_di, s));
        hipError_t e = dpx::launch_dh_reduce(d.dh_part, dl_dh + d.h_off, d.nslots,
                                             static_cast<int64_t>(d.K) * d.N * d.N, s);
        if (e != hipSuccess) return fail(DPX_E_DEVICE, "gradient reduction launch failed: %s", hipGetErrorString(e));
        return DPX_OK;
      }
      DPX_TRY(fork_lanes(p, d, s));
      for (int c = 0; c < d.nchunks; ++c) {
        const int lane = c % d.lanes;
        const int w0 = c * d.wl_chunk;
        const int wc = std::min(d.wl_chunk, d.W - w0);
        hipStream_t ls = lane_stream(p, lane, s);
        if (lane == 1 && c == 1) DPX_HIP(hipStreamWaitEvent(ls, p->ev_offset, 0));
        hipEvent_t first_ev = (c == 0 && d.lanes > 1) ? p->ev_offset : nullptr;
        if (!store) {
          DPX_TRY(forward_chunk(p, d, h, u_in, w0, wc, lane, ls, first_ev));
          first_ev = nullptr;
        }
        if (c < d.lanes) {
          // a lane's first chunk writes its dL/dh slots (later chunks add to them); when that
          // chunk is the short last one, the slots it does not reach must still read as zero
          const int used = (wc + d.w_per_block - 1) / d.w_per_block;
          if (used < d.slots_per_lane) {
            const int64_t per = static_cast<int64_t>(d.K) * d.N * d.N;
            hipError_t e = dpx::launch_fill_zero(
                d.dh_part + (static_cast<int64_t>(lane) * d.slots_per_lane + used) * per,
                static_cast<int64_t>(d.slots_per_lane - used) * per, ls);
            if (e != hipSuccess) return fail(DPX_E_DEVICE, "slot clearing launch failed: %s", hipGetErrorString(e));
          }
        }
        DPX_TRY(adjoint_chunk(p, d, h, u_in, dl_di, w0, wc, lane, c >= d.lanes, ls, first_ev));
      }
      DPX_TRY(join_lanes(p, d, s));
      const int64_t per = static_cast<int64_t>(d.K) * d.N * d.N;
      hipError_t e = dpx::launch_dh_reduce(d.dh_part, dl_dh + d.h_off, d.nslots, per, s);
      if (e != hipSuccess) return fail(DPX_E_DEVICE, "gradient reduction launch failed: %s", hipGetErrorString(e));
      return DPX_OK;
    });
  };
  DPX_TRY(run_graph_or_eager(p, graph_key(3, h, u_in, dl_di, dl_dh), caller, enqueue));
  DPX_TRY(check_outputs(p, {{dl_dh, p->h_total, false, "dl_dh"}}, caller));
  return ok();
}

static_assert(DPX_STATIC_LOSS_MAX_WL == dpx::kStaticLossMaxWl, "header and library agree on the fixed array");

dpx_status dpx_loss_static(const float* intensity, const float* target, int32_t n_wl, int32_t T, double* loss,
                           float* dl_di, void* stream) {
  DPX_TRY(check_ptr(intensity, 4, "intensity"));
  DPX_TRY(check_ptr(target, 4, "target"));
  DPX_TRY(check_ptr(loss, 8, "loss"));
  if (dl_di) DPX_TRY(check_ptr(dl_di, 4, "dl_di"));
  if (n_wl < 1 || n_wl > DPX_STATIC_LOSS_MAX_WL)
    return fail(DPX_E_ARG, "n_wl must be in [1, %d] (got %d)", DPX_STATIC_LOSS_MAX_WL, n_wl);
  if (T < 1 || T > 46340) return fail(DPX_E_ARG, "T must be in [1, 46340] (got %d)", T);
  DPX_TRY(sticky_check());
  double* part = nullptr;
  hipError_t e = dpx::static_loss_scratch(&part);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "fixed loss array lookup failed: %s", hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every partial is written by the first kernel before the second reads it, so the array
  // needs no clearing
  e = dpx::launch_loss(intensity, target, dl_di, part, n_wl, T, s);
  if (e == hipSuccess) e = dpx::launch_loss_sum(part, loss, n_wl, s);
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "loss launch failed: %s", hipGetErrorString(e));
  return ok();
}

dpx_status dpx_psnr(dpx_plan* p, const float* intensity, const float* target, double* psnr, void* stream) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  DPX_TRY(check_ptr(intensity, 4, "intensity"));
  DPX_TRY(check_ptr(target, 4, "target"));
  DPX_TRY(check_ptr(psnr, 8, "psnr"));
  DPX_TRY(sticky_check());
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t w_off = 0;
  for (const auto& d : p->designs) {
    hipError_t e = dpx::launch_psnr(intensity + d.img_off, target + d.img_off, psnr + w_off, d.W, d.T, s);
    if (e != hipSuccess) return fail(DPX_E_DEVICE, "PSNR launch failed: %s", hipGetErrorString(e));
    w_off += d.W;
  }
  return ok();
}

dpx_status dpx_adam_step(float* theta, float* h, const float* dl_dh, float* m, float* v, int64_t n, int32_t step,
                         double lr, double b1, double b2, double eps, double h_max, void* stream) {
  if (n < 0) return fail(DPX_E_ARG, "n must be >= 0");
  if (n == 0) return ok();
  DPX_TRY(check_ptr(theta, 4, "theta"));
  DPX_TRY(check_ptr(h, 4, "h"));
  DPX_TRY(check_ptr(dl_dh, 4, "dl_dh"));
  DPX_TRY(check_ptr(m, 4, "m"));
  DPX_TRY(check_ptr(v, 4, "v"));
  if (step < 1) return fail(DPX_E_ARG, "step counts from 1 (got %d)", step);
  if (!(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps >= 0.0) || !(h_max > 0.0))
    return fail(DPX_E_ARG, "need lr > 0, 0 <= b1, b2 < 1, eps >= 0, h_max > 0");
  DPX_TRY(sticky_check());
  dpx::AdamArgs a{};
  a.lr = static_cast<float>(lr);
  a.b1 = static_cast<float>(b1);
  a.b2 = static_cast<float>(b2);
  a.eps = static_cast<float>(eps);
  a.h_max = static_cast<float>(h_max);
  a.omb1 = static_cast<float>(1.0 - b1);
  a.omb2 = static_cast<float>(1.0 - b2);
  a.c1 = static_cast<float>(1.0 / (1.0 - std::pow(b1, step)));
  a.c2 = static_cast<float>(1.0 / (1.0 - std::pow(b2, step)));
  hipError_t e = dpx::launch_adam_sigmoid(theta, h, dl_dh, m, v, n, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "Adam step launch failed: %s", hipGetErrorString(e));
  return ok();
}

dpx_status dpx_quantize_heights(const float* h, float* h_q, int64_t n, double h_max, int32_t bits, void* stream) {
  if (n < 0) return fail(DPX_E_ARG, "n must be >= 0");
  if (bits < 1 || bits > 24) return fail(DPX_E_ARG, "bits must be in [1, 24] (got %d)", bits);
  if (!(std::isfinite(h_max) && h_max > 0.0)) return fail(DPX_E_ARG, "h_max must be finite and > 0");
  if (n == 0) return ok();
  DPX_TRY(check_ptr(h, 4, "h"));
  DPX_TRY(check_ptr(h_q, 4, "h_q"));
  DPX_TRY(sticky_check());
  const double levels = static_cast<double>((1 << bits) - 1);
  hipError_t e = dpx::launch_quantize(h, h_q, n, static_cast<float>(levels / h_max), static_cast<float>(h_max / levels),
                                      static_cast<float>(levels), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DPX_E_DEVICE, "quantiser launch failed: %s", hipGetErrorString(e));
  return ok();
}

dpx_status dpx_timing_enable(dpx_plan* p, int32_t enable) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  for (auto& t : p->pending) {
    (void)hipEventSynchronize(t.stop);
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  p->pending.clear();
  for (auto& t : p->totals) t = PassTotals{};
  p->timing = enable != 0;
  return ok();
}

dpx_status dpx_timing_read(dpx_plan* p, int32_t pass, double* total_ms, int64_t* launches, int64_t* bytes,
                           double* flops) {
  if (!p) return fail(DPX_E_ARG, "plan is NULL");
  if (pass < 0 || pass >= DPX_PASS_COUNT) return fail(DPX_E_ARG, "pass %d out of range", pass);
  for (auto& t : p->pending) {
    DPX_HIP(hipEventSynchronize(t.stop));
    float ms = 0.f;
    DPX_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
    for (int k : {t.pass, t.instance}) {
      if (k < 0) continue;
      PassTotals& a = p->totals[k];
      a.ms += ms;
      a.launches += 1;
      a.bytes += t.bytes;
      a.flops += t.flops;
    }
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  p->pending.clear();
  const PassTotals& a = p->totals[pass];
  if (total_ms) *total_ms = a.ms;
  if (launches) *launches = a.launches;
  if (bytes) *bytes = a.bytes;
  if (flops) *flops = a.flops;
  return ok();
}

}  // extern "C"
