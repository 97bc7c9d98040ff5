// Bin geometry and time grid of the step (host FP64); see host_math.hpp.
#include "host_math.hpp"

#include <cmath>

namespace pmnu {

BinGeometry make_bin_geometry(int n, double box_size, int n_bins) {
  BinGeometry g;
  const int B = n_bins;
  const int n2max = 3 * n * n / 4;
  const double r2 = 3.0 * n * n / 4.0;
  g.edges.assign(B + 1, 0);
  for (int b = 0; b <= B; ++b)
    g.edges[b] = static_cast<int64_t>(std::ceil(std::pow(r2, static_cast<double>(b) / B)));
  g.edges[0] = 1;
  std::vector<int64_t> mult(n2max + 1, 0);
  const int h = n / 2;
  for (int i = -h; i < h; ++i)
    for (int j = -h; j < h; ++j)
      for (int l = -h; l < h; ++l) ++mult[i * i + j * j + l * l];
  g.bin_of_n2.assign(n2max + 1, 0);
  g.counts.assign(B, 0.0);
  std::vector<double> ksum(B, 0.0);
  const double kf = 2.0 * kPi / box_size;
  int b = 0;
  for (int n2 = 1; n2 <= n2max; ++n2) {
    while (b < B - 1 && n2 >= g.edges[b + 1]) ++b;
    g.bin_of_n2[n2] = static_cast<uint16_t>(b);
    g.counts[b] += static_cast<double>(mult[n2]);
    ksum[b] += static_cast<double>(mult[n2]) * kf * std::sqrt(static_cast<double>(n2));
  }
  g.kmean.assign(B, 0.0);
  for (int k = 0; k < B; ++k) {
    if (g.counts[k] > 0) {
      g.kmean[k] = ksum[k] / g.counts[k];
      g.nonempty.push_back(k);
    }
  }
  return g;
}

void interval_nodes(const Background& bg, double a_lo, double a_hi, int Q, double* a,
                    double* seg, double* hinv) {
  const double u0 = std::log(a_lo), u1 = std::log(a_hi);
  const double h = (u1 - u0) / Q;
  for (int r = 0; r < Q; ++r) a[r] = (r == 0) ? a_lo : std::exp(u0 + r * h);
  for (int r = 0; r < Q; ++r) {
    seg[r] = ds_of(bg, a[r], r + 1 < Q ? a[r + 1] : a_hi);
    hinv[r] = 1.0 / (a[r] * hubble_of(bg, a[r]));
  }
}

void assemble_time_grid(const Background& bg, const double* nd, int n, int Q, double pref,
                        const double* stored_seg, const double* stored_hinv,
                        const double* last_seg, const double* last_hinv, double* ds,
                        double* w) {
  const int nq = n * Q + 1;
  const int q_last = (n - 1) * Q;   // first sub-node of the interval to a_now
  std::vector<double> tw(nq, 0.0);  // trapezoid weights in ln a
  for (int jj = 0; jj < n; ++jj) {
    const double h = (std::log(nd[jj + 1]) - std::log(nd[jj])) / Q;
    for (int r = 0; r < Q; ++r) {
      tw[jj * Q + r] += (r == 0) ? 0.5 * h : h;
      tw[jj * Q + r + 1] += (r == Q - 1) ? 0.5 * h : 0.0;
    }
  }
  ds[nq - 1] = 0.0;
  for (int q = nq - 2; q >= 0; --q)
    ds[q] = ds[q + 1] + (q < q_last ? stored_seg[q] : last_seg[q - q_last]);
  for (int q = 0; q < nq - 1; ++q)
    w[q] = pref * tw[q] * (q < q_last ? stored_hinv[q] : last_hinv[q - q_last]);
  w[nq - 1] = pref * tw[nq - 1] / (nd[n] * hubble_of(bg, nd[n]));
}

}  // namespace pmnu
