// Command-line driver of the library's host-only arithmetic (bin geometry, background,
// time grid of eq. (P-final)), built with host sanitizers by tests/test_host_sanitized.py
// and compared there with the oracle. Reads one request per line on stdin:
//   bins N L B
//   hubble rel omega_m h n_equal n_massless n_masses m_1 .. m_k  n_a a_1 .. a_n
//   grid   rel omega_m h n_equal n_massless n_masses m_1 .. m_k  Q n_nodes a_0 .. a_n
// and prints for each the arrays it asks for, one "name v v v ..." line per array.
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_1209_0461_amd/csrc/background.hpp"
#include "../../paper_1209_0461_amd/csrc/host_math.hpp"

using namespace pmnu;

template <typename T>
static void print(const char* name, const std::vector<T>& v) {
  std::printf("%s", name);
  for (const T& x : v) std::printf(" %.17g", static_cast<double>(x));
  std::printf("\n");
}

static Background read_background(std::istringstream& in, double* om_out) {
  int rel = 0, n_equal = 0, n_massless = 0, k = 0;
  double om = 0.0, h = 0.0;
  in >> rel >> om >> h >> n_equal >> n_massless >> k;
  std::vector<double> masses(k);
  for (double& m : masses) in >> m;
  *om_out = om;
  return make_background(rel != 0, om, h, masses, n_equal, n_massless);
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string what;
    in >> what;
    if (what == "bins") {
      int n = 0, B = 0;
      double L = 0.0;
      in >> n >> L >> B;
      const BinGeometry g = make_bin_geometry(n, L, B);
      print("edges", g.edges);
      print("counts", g.counts);
      print("kmean", g.kmean);
      print("table", g.bin_of_n2);
      print("nonempty", g.nonempty);
    } else if (what == "hubble") {
      double om = 0.0;
      const Background bg = read_background(in, &om);
      int na = 0;
      in >> na;
      std::vector<double> out(na);
      for (double& v : out) {
        double a = 0.0;
        in >> a;
        v = hubble_of(bg, a);
      }
      print("hubble", out);
    } else if (what == "grid") {
      double om = 0.0;
      const Background bg = read_background(in, &om);
      int Q = 0, nn = 0;
      in >> Q >> nn;
      std::vector<double> nd(nn);
      for (double& a : nd) in >> a;
      const int n = nn - 1;                 // intervals; nd[n] is the current step
      std::vector<double> a((n - 1) * Q + Q), seg(a.size()), hinv(a.size());
      for (int j = 0; j < n; ++j)
        interval_nodes(bg, nd[j], nd[j + 1], Q, &a[j * Q], &seg[j * Q], &hinv[j * Q]);
      const int nq = n * Q + 1;
      std::vector<double> ds(nq), w(nq);
      const double pref = 1.5 * om * kH0 * kH0;
      assemble_time_grid(bg, nd.data(), n, Q, pref, seg.data(), hinv.data(),
                         &seg[(n - 1) * Q], &hinv[(n - 1) * Q], ds.data(), w.data());
      a.push_back(nd[n]);
      print("a", a);
      print("ds", ds);
      print("w", w);
    } else if (!what.empty()) {
      std::fprintf(stderr, "unknown request %s\n", what.c_str());
      return 2;
    }
  }
  return 0;
}
