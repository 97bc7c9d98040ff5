// Host-side FP64 arithmetic of the step that runs once per configuration or per a_now:
// the k-bin geometry and the time grid of the history integral eq. (P-final). Plain C++
// with no HIP dependency (built into the library, and on its own with host sanitizers).
#pragma once

#include <cstdint>
#include <vector>

#include "background.hpp"

namespace pmnu {

// B log-spaced bins over |n|^2 in [1, 3 N^2 / 4] (|k| from 2 pi / L to sqrt(3) pi N / L):
// integer edges E_b = ceil((3N^2/4)^(b/B)), E_0 = 1; mode n is in bin b when
// E_b <= |n|^2 < E_{b+1} (the top bin also takes |n|^2 = 3N^2/4); full-sphere mode counts
// over the integer triples of [-N/2, N/2)^3 and mean |k|; empty bins have count 0.
struct BinGeometry {
  std::vector<int64_t> edges;      // [B+1]
  std::vector<double> counts;      // [B]
  std::vector<double> kmean;       // [B] h/Mpc (0 for empty bins)
  std::vector<uint16_t> bin_of_n2; // [3N^2/4 + 1]
  std::vector<int> nonempty;       // bins with counts > 0, increasing
};
BinGeometry make_bin_geometry(int n, double box_size, int n_bins);

// Sub-nodes of one interval [a_lo, a_hi] of the quadrature (Q equal steps in ln a): their
// scale factors a[Q], the s difference to the next sub-node seg[Q], and 1/(a H) hinv[Q].
void interval_nodes(const Background& bg, double a_lo, double a_hi, int Q, double* a,
                    double* seg, double* hinv);

// The quadrature of eq. (P-final) over nodes nd[0..n] (nd[n] = a_now) for one box:
// ds[q] = s(a_now) - s(a_q) and w[q] = pref * (trapezoid weight in ln a) / (a_q H(a_q)) for
// the n Q + 1 sub-nodes. seg/hinv of the stored intervals (n - 1) Q come from `stored`
// (sub-nodes 0 .. (n-1)Q - 1) and those of the last interval from `last` (Q values), as
// interval_nodes gives them; H(a_now) from bg.
void assemble_time_grid(const Background& bg, const double* nd, int n, int Q, double pref,
                        const double* stored_seg, const double* stored_hinv,
                        const double* last_seg, const double* last_hinv, double* ds,
                        double* w);

}  // namespace pmnu
