// Structural checks of the LDS layouts of every transform plan (csrc/fft.hpp), on the host:
// each exchange after a non-final stage stores the M entries of a transform at distinct slots
// inside the region its kernels reserve (row and column kernels), the column tile's staged rows
// fit the region, and the blocks of the 1024-point passes still fit two to a CU.  Prints one
// line per failed check and "ok" at the end when there is none.
#include <cstdio>
#include <vector>

#include "fft.hpp"

using namespace dpx;

static int failures = 0;
#define CHECK(cond, ...)               \
  do {                                 \
    if (!(cond)) {                     \
      std::printf(__VA_ARGS__);        \
      std::printf("\n");               \
      ++failures;                      \
    }                                  \
  } while (0)

constexpr int kLdsPerCu = 163840;

// slot of exchange entry i after stage ST, as the stage's writes and reads address it: the
// plan's block padding where it has one (and the kernel uses it), else the shift padding
template <int M, int V>
int slot(int st, int i, bool block_padding) {
  const int xa = (V == 0 && block_padding) ? XPad<M>::A[st] : 0;
  const int xb = (V == 0 && block_padding) ? XPad<M>::B[st] : 0;
  return xa > 0 ? i + (i / xa) * xb : lds_slot<M>(i);
}

template <int M, int V>
void check_plan() {
  constexpr int NST = Radix<M, V>::NST;
  for (int pass = 0; pass < 2; ++pass) {  // 0: row kernels, 1: column kernels
    const bool bp = pass == 1 || XPad<M>::ROWS;
    const int region = pass == 0 ? Geo<M>::ROW_REGION : Geo<M>::COL_REGION;
    for (int st = 0; st + 1 < NST; ++st) {
      std::vector<char> used(region, 0);
      for (int i = 0; i < M; ++i) {
        const int s = slot<M, V>(st, i, bp);
        CHECK(s >= 0 && s < region, "M=%d plan %d %s stage %d: entry %d at slot %d outside the %d-slot region", M, V,
              pass ? "column" : "row", st, i, s, region);
        if (s >= 0 && s < region) {
          CHECK(!used[s], "M=%d plan %d %s stage %d: slot %d holds two entries", M, V, pass ? "column" : "row", st, s);
          used[s] = 1;
        }
      }
    }
  }
  // staged rows of tile column c: SKEW (c / 2) + y for y < M / 2 (zero-padded planes), y < M
  constexpr int TX = 8;
  const int last = XPad<M>::SKEW * ((TX - 1) / 2) + M - 1;
  CHECK(last < Geo<M>::COL_REGION, "M=%d: staged rows reach slot %d of a %d-slot column region", M, last,
        Geo<M>::COL_REGION);
}

template <int M>
void check_length() {
  check_plan<M, 0>();
  if constexpr (radix_plans(M) > 1) {
    check_plan<M, 1>();
    check_plan<M, 2>();
  }
}

int main() {
  check_length<64>();
  check_length<96>();
  check_length<128>();
  check_length<192>();
  check_length<256>();
  check_length<384>();
  check_length<512>();
  check_length<1024>();
  check_length<1600>();
  // the 1024-point column and row blocks (8 columns / 8 rows with the twiddle table of the
  // built-in plan) fit two to a CU
  const int col_block = 8 * Geo<1024>::COL_REGION * 8 + twiddle_count<1024, 0>() * 8;
  const int row_block = (512 / Geo<1024>::P) * Geo<1024>::ROW_REGION * 8 + twiddle_count<1024, 0>() * 8;
  CHECK(2 * col_block <= kLdsPerCu, "1024-point column block: %d bytes of LDS, two do not fit a CU", col_block);
  CHECK(2 * row_block <= kLdsPerCu, "1024-point row block: %d bytes of LDS, two do not fit a CU", row_block);
  if (failures == 0) std::printf("ok\n");
  return failures == 0 ? 0 : 1;
}
