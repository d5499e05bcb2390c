// Host-side lattice builder (FP64): weights, corrected Hermite rows, norms.
#pragma once

#include <string>
#include <vector>

#include "../../include/mrtlb.h"

namespace mrtlb {

// Row order of the low-order (order <= 3) Hermite rows, component form:
// 2D: 1, x, y, xx, yy, xy, xyy, yxx, xxx, yyy
// 3D: 1, x, y, z, xx, yy, zz, xy, xz, yz, xyy, xzz, yxx, yzz, zxx, zyy, xyz,
//     xxx, yyy, zzz
// Standard lattices (D2Q9, D3Q27) stop before the pure rows (nlow 8 / 17).
struct HostLattice {
  int kind = 0, D = 0, B = 0, nlow = 0;
  bool standard = false;
  double c[3] = {1, 1, 1};
  double cs2 = 0;
  std::vector<int> e;          // B x D
  std::vector<double> w;       // B
  double corr[3][3] = {};      // corr[a][b]: coefficient of c_a(c_b^2 - cs^2) removed from the pure row a
  std::vector<double> H;       // nlow x B
  std::vector<double> norms;   // nlow
};

// Fills *out from the descriptor; returns MRTLB_OK or an error with *err set.
mrtlb_status build_lattice(const mrtlb_lattice_desc& desc, HostLattice* out, std::string* err);

// Slot order of the populations for the user-supplied lattices' step
// kernel: with rays, first rays (slots 4r .. 4r + 3: +-e, then +-c e for an
// integer c >= 2, the smallest such c; bases taken shortest first), then
// the remaining pairs of opposite velocities (each velocity with its first
// unused opposite, in index order), then the velocities without one.
// Returns the population index of each slot; sets *nrays, *npairs and the
// multiplier c of each ray in *mult.
std::vector<int> velocity_slots(const HostLattice& L, bool rays, int* nrays, int* npairs, std::vector<int>* mult);

// Index helpers for the component row order above.
int row_j(int D, int a);             // order 1, axis a
int row_nn(int D, int a);            // order 2 normal (c_a^2 - cs^2)
int row_off(int D, int a, int b);    // order 2 off-diagonal, a < b
int row_abb(int D, int a, int b);    // order 3 mixed c_a (c_b^2 - cs^2), a != b
int row_xyz();                       // order 3, 3D only
int row_aaa(int D, int a);           // order 3 pure (corrected)

}  // namespace mrtlb
