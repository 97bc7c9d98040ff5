// Device pieces of the patch deposit shared by its reduction kernels: the coarse-cell
// registry's sizes and the overlap of a patch with a region of a cell.
//
// A registry entry (int4) of a patch: x = chunk (patch slot), y = box origin
// gx | gy << 10 | gz << 20, z = extents ex | ey << 10 | ez << 20 (each below 1024).
#pragma once
#include "pm_nu_internal.hpp"

namespace pmnu {

constexpr int kPatchList = 32;      // patches per coarse cell
constexpr int kPatchRegMax = 27;    // coarse cells per patch

// Up to two pieces of the overlap of a periodic patch interval [p, p + e) with the cell
// interval [cs, cs + cb) on an axis of length n (e <= n): patch-local start, cell-local
// start and length of each.
struct Pieces {
  int cnt;
  int pl[2], cl[2], len[2];
};
__device__ __forceinline__ Pieces overlap(int p, int e, int cs, int cb, int n) {
  Pieces r;
  const int d2 = (p - cs + n) & (n - 1);        // cell-local index of the patch start
  const int w = n - d2;                         // patch-local index where it re-enters
  const bool first = d2 < cb;                   // [p, ...) starts inside the cell
  const bool second = d2 != 0 && w < e;         // the patch wraps back into the cell
  const int len_a = min(e, cb - d2), len_b = min(e - w, cb);
  // fixed slots (no indexed writes, which would go to scratch)
  r.cnt = static_cast<int>(first) + static_cast<int>(second);
  r.pl[0] = first ? 0 : w;
  r.cl[0] = first ? d2 : 0;
  r.len[0] = first ? len_a : len_b;
  r.pl[1] = w;
  r.cl[1] = 0;
  r.len[1] = len_b;
  return r;
}

}  // namespace pmnu
