// Launchers of the propagation passes for one transform length M = DPX_M: row passes (every
// mode, single-design and grouped), column passes (every variant and transfer-function
// source, single-design and grouped, and the matrix-core form) and the transfer table.  The
// build compiles this file once per supported length, so the kernel templates of the
// different lengths are instantiated in parallel translation units.
#include <cmath>

#include "pass_kernels.hpp"

#ifndef DPX_M
#error "compile with -DDPX_M=<transform length>"
#endif

#define DPX_PASTE2(a, b) a##b
#define DPX_PASTE(a, b) DPX_PASTE2(a, b)
#define DPX_NAME(f) DPX_PASTE(f, DPX_M)

namespace dpx {
namespace {

constexpr int M = DPX_M;

unsigned group_grid(const GroupArgs& g) { return static_cast<unsigned>(g.block0[g.ntasks]); }

// runs f with the radix plan as a compile-time constant (plans beyond 0 exist for some lengths)
template <typename F>
hipError_t with_plan(int plan, F&& f) {
  if constexpr (radix_plans(M) > 1) {
    if (plan == 1) return f(std::integral_constant<int, 1>{});
    if (plan == 2) return f(std::integral_constant<int, 2>{});
  }
  if (plan == 0) return f(std::integral_constant<int, 0>{});
  return hipErrorInvalidValue;
}

template <int PAD, int V>
hipError_t row_mode(int mode, const RowArgs& a, dim3 grid, hipStream_t s) {
  if constexpr (M == 1600 && PAD == 2 && V == 0) {
    if (mode == ROW_FWD_MID) {
      row_kernel_w3<M, PAD, ROW_FWD_MID><<<grid, row_block_threads<M, ROW_FWD_MID>(), 0, s>>>(a);
      return hipGetLastError();
    }
  }
  switch (mode) {
#define DPX_ROW(MD) \
  case MD: row_kernel<M, PAD, MD, V><<<grid, row_block_threads<M, MD>(), 0, s>>>(a); break;
    DPX_ROW(ROW_FWD_FIRST)
    DPX_ROW(ROW_FWD_MID)
    DPX_ROW(ROW_FWD_LAST)
    DPX_ROW(ROW_ADJ_SEED)
    DPX_ROW(ROW_ADJ_MID)
    DPX_ROW(ROW_ADJ_LAST)
    DPX_ROW(ROW_ADJ_LAST_U)
#undef DPX_ROW
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PAD>
hipError_t row_group_mode(int mode, const GroupArgs& g, hipStream_t s) {
  switch (mode) {
#define DPX_ROW(MD) \
  case MD: row_group_kernel<M, PAD, MD><<<group_grid(g), row_block_threads<M, MD>(), 0, s>>>(g); break;
    DPX_ROW(ROW_FWD_FIRST)
    DPX_ROW(ROW_FWD_MID)
    DPX_ROW(ROW_FWD_LAST)
    DPX_ROW(ROW_ADJ_SEED)
    DPX_ROW(ROW_ADJ_MID)
    DPX_ROW(ROW_ADJ_LAST)
    DPX_ROW(ROW_ADJ_LAST_U)
#undef DPX_ROW
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// H source of a launch: the table when the arguments carry one, the per-element evaluation
// with the translation ramp for a translated gap, else the variant's evaluation
int h_mode(int variant, bool table, bool shifted = false, bool band = false) {
  return table ? kHTable : band ? kHBand : shifted ? kHShift : (variant >= 2 ? kHMirror : kHEval);
}

// every aperture row in and out (the row-range tests compile away)
bool full_rows(const ColArgs& a) { return a.in_lo == 0 && a.out_lo == 0 && a.in_hi == a.n && a.out_hi == a.n; }

template <int PAD, int TX, int HM, int V>
hipError_t col_launch(bool conj, const ColArgs& a, int w_count, hipStream_t s) {
  dim3 grid(M / TX, (w_count + a.col_wpb - 1) / a.col_wpb);
  const bool full = full_rows(a);
  if (conj) {
    if (full) col_kernel<M, PAD, true, TX, HM, true, V><<<grid, TX * Geo<M>::P, 0, s>>>(a);
    else col_kernel<M, PAD, true, TX, HM, false, V><<<grid, TX * Geo<M>::P, 0, s>>>(a);
  } else {
    if (full) col_kernel<M, PAD, false, TX, HM, true, V><<<grid, TX * Geo<M>::P, 0, s>>>(a);
    else col_kernel<M, PAD, false, TX, HM, false, V><<<grid, TX * Geo<M>::P, 0, s>>>(a);
  }
  return hipGetLastError();
}

// tile widths of the transform variants: 8 / 16 columns, or 4 / 8 when a transform spans
// wavefronts (blocks stay within 1024 threads)
constexpr int kTileNarrow = Geo<M>::WAVE_LOCAL ? 8 : 4;
constexpr int kTileWide = Geo<M>::WAVE_LOCAL ? 16 : 8;

// H sources of each radix plan: plan 0 has them all; the other plans only the evaluated and
// mirrored transfer functions of the untranslated, full-spectrum gap (the plan layer refuses
// the rest)
template <int PAD, int TX, int V>
hipError_t col_launch_h(int hm, bool conj, const ColArgs& a, int w_count, hipStream_t s) {
  if constexpr (V == 0) {
    if (hm == kHTable) return col_launch<PAD, TX, kHTable, V>(conj, a, w_count, s);
    if (hm == kHBand) return col_launch<PAD, TX, kHBand, V>(conj, a, w_count, s);
    if (hm == kHShift) return col_launch<PAD, TX, kHShift, V>(conj, a, w_count, s);
  } else {
    if (hm == kHTable || hm == kHBand || hm == kHShift) return hipErrorInvalidValue;
  }
  if constexpr (Geo<M>::WAVE_LOCAL) {
    if (hm == kHMirror) return col_launch<PAD, TX, kHMirror, V>(conj, a, w_count, s);
  } else {
    // the mirrored form exchanges H across the lanes of one wavefront
    if (hm == kHMirror) return hipErrorInvalidValue;
  }
  return col_launch<PAD, TX, kHEval, V>(conj, a, w_count, s);
}

template <int PAD>
hipError_t col_variant(int variant, int plan, bool conj, const ColArgs& args, int w_count, hipStream_t s) {
  const bool shifted = args.sx != 0.0 || args.sy != 0.0;
  const ColArgs& a = args;
  const int hm = h_mode(variant, a.htab != nullptr, shifted, a.band_limited != 0);
  return with_plan(plan, [&](auto vc) -> hipError_t {
    constexpr int V = decltype(vc)::value;
    if (col_tile_width(M, variant) == kTileNarrow) return col_launch_h<PAD, kTileNarrow, V>(hm, conj, a, w_count, s);
    return col_launch_h<PAD, kTileWide, V>(hm, conj, a, w_count, s);
  });
}

template <int PAD>
hipError_t colgemm_launch(bool conj, const ColArgs& a, int w_count, hipStream_t s) {
  if constexpr (M <= 512 && M % 16 == 0 && (M / PAD) % 16 == 0) {
    ColArgs one = a;
    one.col_wpb = 1;
    dim3 grid(M / kGemmTile, w_count);
    if (conj)
      colgemm_kernel<M, PAD, true><<<grid, gemm_threads(M), 0, s>>>(one, a.dft);
    else
      colgemm_kernel<M, PAD, false><<<grid, gemm_threads(M), 0, s>>>(one, a.dft);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int PAD, int TX, int HM>
hipError_t col_group_tx(bool conj, bool full, const GroupArgs& g, hipStream_t s) {
  if (conj) {
    if (full) col_group_kernel<M, PAD, true, TX, HM, true><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
    else col_group_kernel<M, PAD, true, TX, HM, false><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
  } else {
    if (full) col_group_kernel<M, PAD, false, TX, HM, true><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
    else col_group_kernel<M, PAD, false, TX, HM, false><<<group_grid(g), TX * Geo<M>::P, 0, s>>>(g);
  }
  return hipGetLastError();
}

template <int PAD, int TX>
hipError_t col_group_h(int hm, bool conj, bool full, const GroupArgs& g, hipStream_t s) {
  if (hm == kHTable) return col_group_tx<PAD, TX, kHTable>(conj, full, g, s);
  if constexpr (Geo<M>::WAVE_LOCAL) {
    if (hm == kHMirror) return col_group_tx<PAD, TX, kHMirror>(conj, full, g, s);
  } else {
    if (hm == kHMirror) return hipErrorInvalidValue;
  }
  return col_group_tx<PAD, TX, kHEval>(conj, full, g, s);
}

template <int PAD>
hipError_t col_group_variant(int variant, bool table, bool conj, bool full, const GroupArgs& g, hipStream_t s) {
  const int hm = h_mode(variant, table);
  if (col_tile_width(M, variant) == kTileNarrow) return col_group_h<PAD, kTileNarrow>(hm, conj, full, g, s);
  return col_group_h<PAD, kTileWide>(hm, conj, full, g, s);
}

}  // namespace

hipError_t DPX_NAME(launch_row_)(int pad, int mode, int plan, const RowArgs& a, int n_row_blocks, int n_w_blocks,
                                 hipStream_t s) {
  const dim3 grid(n_row_blocks, n_w_blocks);
  return with_plan(plan, [&](auto vc) -> hipError_t {
    constexpr int V = decltype(vc)::value;
    if (pad == 2) return row_mode<2, V>(mode, a, grid, s);
    if (pad == 1) return row_mode<1, V>(mode, a, grid, s);
    return hipErrorInvalidValue;
  });
}

hipError_t DPX_NAME(launch_row_group_)(int pad, int mode, const GroupArgs& g, hipStream_t s) {
  if (pad == 2) return row_group_mode<2>(mode, g, s);
  if (pad == 1) return row_group_mode<1>(mode, g, s);
  return hipErrorInvalidValue;
}

hipError_t DPX_NAME(launch_col_)(int pad, bool conj, int variant, int plan, const ColArgs& a, int w_count,
                                 hipStream_t s) {
  if (variant == 4) {
    if (a.sx != 0.0 || a.sy != 0.0) return hipErrorInvalidValue;  // matrix-core form: no translation
    if (pad == 2) return colgemm_launch<2>(conj, a, w_count, s);
    if (pad == 1) return colgemm_launch<1>(conj, a, w_count, s);
    return hipErrorInvalidValue;
  }
  if (pad == 2) return col_variant<2>(variant, plan, conj, a, w_count, s);
  if (pad == 1) return col_variant<1>(variant, plan, conj, a, w_count, s);
  return hipErrorInvalidValue;
}

void DPX_NAME(twiddle_table_)(int plan, std::vector<float2>& out) {
  out.clear();
  (void)with_plan(plan, [&](auto vc) -> hipError_t {
    twiddle_table_host<M, decltype(vc)::value>(out);
    return hipSuccess;
  });
}

hipError_t DPX_NAME(launch_col_group_)(int pad, bool conj, int variant, bool table, bool full, const GroupArgs& g,
                                       hipStream_t s) {
  if (pad == 2) return col_group_variant<2>(variant, table, conj, full, g, s);
  if (pad == 1) return col_group_variant<1>(variant, table, conj, full, g, s);
  return hipErrorInvalidValue;
}

bool DPX_NAME(lds_supported_)(int pad) {
  return pad == 2 ? LdsGeo<M, 2>::FITS && M <= 128 : pad == 1 ? LdsGeo<M, 1>::FITS && M <= 128 : false;
}

hipError_t DPX_NAME(launch_lds_)(int pad, bool adjoint, const LdsArgs& a, hipStream_t s) {
  if constexpr (M <= 128) {
    auto go = [&](auto padc) -> hipError_t {
      constexpr int PD = decltype(padc)::value;
      if constexpr (LdsGeo<M, PD>::FITS) {
        if (adjoint)
          lds_adjoint_kernel<M, PD><<<a.W, kLdsThreads, 0, s>>>(a);
        else
          lds_forward_kernel<M, PD><<<a.W, kLdsThreads, 0, s>>>(a);
        return hipGetLastError();
      } else {
        return hipErrorInvalidValue;
      }
    };
    if (pad == 2) return go(std::integral_constant<int, 2>{});
    if (pad == 1) return go(std::integral_constant<int, 1>{});
  }
  return hipErrorInvalidValue;
}

hipError_t DPX_NAME(launch_transfer_table_)(const WlConst* wl, int W, double zrev, float2* out, hipStream_t s) {
  const dim3 grid(M / 2 + 1, W);
  transfer_table_kernel<M><<<grid, 256, 0, s>>>(wl, zrev, out);
  return hipGetLastError();
}

}  // namespace dpx
