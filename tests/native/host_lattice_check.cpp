// The host lattice builder under AddressSanitizer and UndefinedBehavior-
// Sanitizer (built with g++ by tests/test_host_sanitizers.py).  Reads one
// descriptor per line on stdin,
//   kind d b c0 c1 c2 cs2 n_free f0 f1 f2 f3 [e (b*d ints) w (b doubles)]
// (the arrays only for the custom kind), builds it, and prints
//   ok B nlow max_offdiag w_0 .. w_{B-1} norm_0 .. norm_{nlow-1}
// where max_offdiag is the largest |sum_j w_j H_r(j) H_s(j)| / sqrt(n_r n_s)
// over r != s (weighted orthogonality of the Hermite rows), or
//   err <status> <message>
// for a refused descriptor.  A line that starts with "S" instead prints,
// for the descriptor after it, the slot order of the user-supplied step
// kernel (mrtlb::velocity_slots) with and without rays:
//   slots <rays> <nrays> <npairs> <c_1 .. c_nrays> : <slot population indices>
// A last pass builds descriptors with missing arrays and out-of-range
// sizes, which must be refused.
#include <cmath>
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_2512_16230_amd/csrc/host_lattice.h"

using mrtlb::HostLattice;

static void report_slots(const mrtlb_lattice_desc& desc) {
  HostLattice L;
  std::string err;
  if (mrtlb::build_lattice(desc, &L, &err) != MRTLB_OK) {
    std::printf("err %s\n", err.c_str());
    return;
  }
  for (int rays = 1; rays >= 0; --rays) {
    int nr = -1, np = -1;
    std::vector<int> mult;
    const std::vector<int> slot = mrtlb::velocity_slots(L, rays == 1, &nr, &np, &mult);
    std::printf("slots %d %d %d", rays, nr, np);
    for (int c : mult) std::printf(" %d", c);
    std::printf(" :");
    for (int j : slot) std::printf(" %d", j);
    std::printf("\n");
  }
}

static void report(const mrtlb_lattice_desc& desc) {
  HostLattice L;
  std::string err;
  const mrtlb_status st = mrtlb::build_lattice(desc, &L, &err);
  if (st != MRTLB_OK) {
    std::printf("err %d %s\n", (int)st, err.c_str());
    return;
  }
  double worst = 0;
  for (int r = 0; r < L.nlow; ++r)
    for (int s = r + 1; s < L.nlow; ++s) {
      double dot = 0;
      for (int j = 0; j < L.B; ++j) dot += L.w[j] * L.H[(size_t)r * L.B + j] * L.H[(size_t)s * L.B + j];
      worst = std::fmax(worst, std::fabs(dot) / std::sqrt(L.norms[r] * L.norms[s]));
    }
  std::printf("ok %d %d %.3e", L.B, L.nlow, worst);
  for (double v : L.w) std::printf(" %.17g", v);
  for (double v : L.norms) std::printf(" %.17g", v);
  std::printf("\n");
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    if (line.empty()) continue;
    const bool slots = line[0] == 'S';
    std::istringstream in(slots ? line.substr(1) : line);
    mrtlb_lattice_desc desc{};
    in >> desc.kind >> desc.d >> desc.b >> desc.c[0] >> desc.c[1] >> desc.c[2] >> desc.cs2 >> desc.n_free;
    for (int k = 0; k < 4; ++k) in >> desc.free_w[k];
    std::vector<int> e;
    std::vector<double> w;
    if (desc.kind == MRTLB_CUSTOM) {
      e.resize((size_t)desc.b * desc.d);
      w.resize(desc.b);
      for (int& v : e) in >> v;
      for (double& v : w) in >> v;
      desc.e = e.data();
      desc.w = w.data();
    }
    if (slots) report_slots(desc);
    else report(desc);
  }
  // refused descriptors: no arrays, sizes out of range, a bad kind
  mrtlb_lattice_desc bad{};
  bad.kind = MRTLB_CUSTOM;
  bad.d = 2;
  bad.b = 9;
  bad.c[0] = bad.c[1] = bad.c[2] = 1;
  bad.cs2 = 1.0 / 3.0;
  report(bad);                               // NULL e and w
  std::vector<int> e(4 * 60, 0);
  std::vector<double> w(60, 1.0 / 60);
  bad.e = e.data();
  bad.w = w.data();
  bad.b = 60;                                // beyond the largest supported b
  report(bad);
  bad.b = 9;
  bad.d = 4;                                 // no such dimension
  report(bad);
  bad.kind = 99;
  report(bad);
  return 0;
}
