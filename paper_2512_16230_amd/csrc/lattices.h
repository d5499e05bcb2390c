// Velocity sets of the supported lattices as compile-time tables, shared by
// the host lattice builder and the kernels (integer multiples e_j; the
// physical velocity is c_j = diag(c) e_j).  Column orders follow the paper:
//   rD2Q25  Sec. V, eq. (3-1): rest, then the D2Q9 ring scaled by 1, 2, 3
//   rD2Q13  Sec. V, eq. (Q13lattice)
//   rD3Q53  App. D: D3Q27 in the printed order, then 2x its 26 moving columns
//   rD3Q33  App. D: D3Q27, then (+-2,0,0), (0,+-2,0), (0,0,+-2)
//   rD2Q21  the first 21 columns of rD2Q25 (its (+-3,+-3) group removed)
//   D2Q21K  App. C: rest, D2Q9 ring, the eight knight moves, (+-3,0), (0,+-3)
//   rD3Q45  the first 45 columns of rD3Q53 (its (+-2,+-2,+-2) group removed)
//   rD2Q17-k  App. C, D2Q17 cases 1-5: the printed velocity matrices (rD2Q25
//           subgroups whose dropped groups carry zero weight)
#pragma once

namespace mrtlb {

enum LatticeKind {
  kRD2Q25 = 0, kRD2Q13 = 1, kRD3Q53 = 2, kRD3Q33 = 3, kRD2Q21 = 4, kD2Q21K = 5, kRD3Q45 = 6,
  kRD2Q17_1 = 7, kRD2Q17_2 = 8, kRD2Q17_3 = 9, kRD2Q17_4 = 10, kRD2Q17_5 = 11, kD2Q9 = 12, kD3Q27 = 13,
  kCustom = 14
};

struct LatRD2Q25 {
  static constexpr int kind = kRD2Q25, D = 2, B = 25, MAXE = 3;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0, 3, -3, -3, 3};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3, 3, 3, -3, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q13 {
  static constexpr int kind = kRD2Q13, D = 2, B = 13, MAXE = 2;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q21 {
  static constexpr int kind = kRD2Q21, D = 2, B = 21, MAXE = 3;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3};
  static constexpr int EZ[B] = {};
};

struct LatD2Q21K {
  static constexpr int kind = kD2Q21K, D = 2, B = 21, MAXE = 3;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 1, -1, -2, -2, -1, 1, 2, 3, 0, -3, 0};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 1, 2, 2, 1, -1, -2, -2, -1, 0, 3, 0, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q17_1 {
  static constexpr int kind = kRD2Q17_1, D = 2, B = 17, MAXE = 3;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, -2, -2, 2, 3, 0, -3, 0};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 2, 2, -2, -2, 0, 3, 0, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q17_2 {
  static constexpr int kind = kRD2Q17_2, D = 2, B = 17, MAXE = 3;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 3, 0, -3, 0, 3, -3, -3, 3};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 3, 0, -3, 3, 3, -3, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q17_3 {
  static constexpr int kind = kRD2Q17_3, D = 2, B = 17, MAXE = 3;
  static constexpr int EX[B] = {0, 1, -1, -1, 1, 2, 0, -2, 0, 3, 0, -3, 0, 3, -3, -3, 3};
  static constexpr int EY[B] = {0, 1, 1, -1, -1, 0, 2, 0, -2, 0, 3, 0, -3, 3, 3, -3, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q17_4 {
  static constexpr int kind = kRD2Q17_4, D = 2, B = 17, MAXE = 3;
  static constexpr int EX[B] = {0, 1, -1, -1, 1, 2, -2, -2, 2, 3, 0, -3, 0, 3, -3, -3, 3};
  static constexpr int EY[B] = {0, 1, 1, -1, -1, 2, 2, -2, -2, 0, 3, 0, -3, 3, 3, -3, -3};
  static constexpr int EZ[B] = {};
};

struct LatRD2Q17_5 {
  static constexpr int kind = kRD2Q17_5, D = 2, B = 17, MAXE = 2;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2};
  static constexpr int EZ[B] = {};
};

// Standard single-layer D2Q9 (the first layer of eq. 3-1): k = 1 model,
// no pure third-order rows, non-diagonal S2 block (eq. 4-27).
struct LatD2Q9 {
  static constexpr int kind = kD2Q9, D = 2, B = 9, MAXE = 1;
  static constexpr int EX[B] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int EY[B] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int EZ[B] = {};
};

#define MRTLB_D3Q27_X 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1
#define MRTLB_D3Q27_Y 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, -1, 1, 1, -1
#define MRTLB_D3Q27_Z 0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1

struct LatRD3Q53 {
  static constexpr int kind = kRD3Q53, D = 3, B = 53, MAXE = 2;
  static constexpr int EX[B] = {MRTLB_D3Q27_X, 2, -2, 0, 0, 0, 0, 2, -2, -2, 2, 2, -2, -2, 2, 0, 0, 0, 0, 2, -2, 2, -2, 2, -2, -2, 2};
  static constexpr int EY[B] = {MRTLB_D3Q27_Y, 0, 0, 2, -2, 0, 0, 2, -2, 2, -2, 0, 0, 0, 0, 2, -2, -2, 2, 2, -2, 2, -2, -2, 2, 2, -2};
  static constexpr int EZ[B] = {MRTLB_D3Q27_Z, 0, 0, 0, 0, 2, -2, 0, 0, 0, 0, 2, -2, 2, -2, 2, -2, 2, -2, 2, -2, -2, 2, 2, -2, 2, -2};
};

struct LatRD3Q45 {
  static constexpr int kind = kRD3Q45, D = 3, B = 45, MAXE = 2;
  static constexpr int EX[B] = {MRTLB_D3Q27_X, 2, -2, 0, 0, 0, 0, 2, -2, -2, 2, 2, -2, -2, 2, 0, 0, 0, 0};
  static constexpr int EY[B] = {MRTLB_D3Q27_Y, 0, 0, 2, -2, 0, 0, 2, -2, 2, -2, 0, 0, 0, 0, 2, -2, -2, 2};
  static constexpr int EZ[B] = {MRTLB_D3Q27_Z, 0, 0, 0, 0, 2, -2, 0, 0, 0, 0, 2, -2, 2, -2, 2, -2, 2, -2};
};

// Standard D3Q27: the first 27 columns of the rD3Q53 velocity matrix.
struct LatD3Q27 {
  static constexpr int kind = kD3Q27, D = 3, B = 27, MAXE = 1;
  static constexpr int EX[B] = {MRTLB_D3Q27_X};
  static constexpr int EY[B] = {MRTLB_D3Q27_Y};
  static constexpr int EZ[B] = {MRTLB_D3Q27_Z};
};

struct LatRD3Q33 {
  static constexpr int kind = kRD3Q33, D = 3, B = 33, MAXE = 2;
  static constexpr int EX[B] = {MRTLB_D3Q27_X, 2, -2, 0, 0, 0, 0};
  static constexpr int EY[B] = {MRTLB_D3Q27_Y, 0, 0, 2, -2, 0, 0};
  static constexpr int EZ[B] = {MRTLB_D3Q27_Z, 0, 0, 0, 0, 2, -2};
};

#undef MRTLB_D3Q27_X
#undef MRTLB_D3Q27_Y
#undef MRTLB_D3Q27_Z

// User-supplied velocity set: the velocities live in KParams at run time;
// this type only carries the dimension for the moment-space code.
template <int DIM>
struct LatCustom {
  static constexpr int kind = kCustom, D = DIM, B = 1, MAXE = 1;
  static constexpr int EX[1] = {0};
  static constexpr int EY[1] = {0};
  static constexpr int EZ[1] = {0};
};

// Standard lattices: single layer, k = 1 model.
template <class L>
constexpr bool is_standard() {
  return L::kind == kD2Q9 || L::kind == kD3Q27;
}

template <class L>
constexpr int ez(int j) {
  if constexpr (L::D == 3) return L::EZ[j];
  return 0;
}

constexpr int iabs(int v) { return v < 0 ? -v : v; }
constexpr int igcd(int a, int b) { return b == 0 ? a : igcd(b, a % b); }

// Per-lattice index tables, evaluated once per lattice at compile time (the
// kernels query them inside nested compile-time loops):
//  * opp[j]: the population with velocity -e_j;
//  * pairs: the p-th pair is (first[p], opp[first[p]]), taken in increasing
//    order of the first index with first < opposite;
//  * rays: pairs whose velocities are multiples of one direction (e, 2e, 3e
//    on the multispeed lattices) form a ray.  Pair p's first velocity is
//    sign[p] * scale[p] * base, base = dir[leader[p]] being the primitive
//    direction of the ray's first pair (its leader).
template <class L>
struct LatticeTables {
  static constexpr int NP = (L::B - 1) / 2;
  int opp[L::B] = {};
  int first[NP > 0 ? NP : 1] = {};
  int scale[NP > 0 ? NP : 1] = {};
  int leader[NP > 0 ? NP : 1] = {};
  int sign[NP > 0 ? NP : 1] = {};
  int dir[NP > 0 ? NP : 1][3] = {};
};

template <class L>
constexpr LatticeTables<L> make_tables() {
  LatticeTables<L> t;
  for (int j = 0; j < L::B; ++j) {
    t.opp[j] = -1;
    for (int k = 0; k < L::B && t.opp[j] < 0; ++k) {
      bool same = L::EX[k] == -L::EX[j] && L::EY[k] == -L::EY[j];
      if (L::D == 3) same = same && ez<L>(k) == -ez<L>(j);
      if (same) t.opp[j] = k;
    }
  }
  int count = 0;
  for (int j = 1; j < L::B; ++j)
    if (j < t.opp[j]) t.first[count++] = j;
  for (int p = 0; p < LatticeTables<L>::NP; ++p) {
    const int j = t.first[p];
    const int v[3] = {L::EX[j], L::EY[j], ez<L>(j)};
    t.scale[p] = igcd(igcd(iabs(v[0]), iabs(v[1])), iabs(v[2]));
    for (int a = 0; a < 3; ++a) t.dir[p][a] = a < L::D ? v[a] / t.scale[p] : 0;
  }
  for (int p = 0; p < LatticeTables<L>::NP; ++p) {
    t.leader[p] = p;
    t.sign[p] = 1;
    for (int q = 0; q <= p; ++q) {
      bool same = true, opp = true;
      for (int a = 0; a < L::D; ++a) {
        same = same && t.dir[q][a] == t.dir[p][a];
        opp = opp && t.dir[q][a] == -t.dir[p][a];
      }
      if (same || opp) {
        t.leader[p] = q;
        t.sign[p] = same ? 1 : -1;
        break;
      }
    }
  }
  return t;
}

template <class L>
inline constexpr LatticeTables<L> kTables = make_tables<L>();

// Index of the population with velocity -e_j.
template <class L>
constexpr int opposite(int j) { return kTables<L>.opp[j]; }

template <class L>
constexpr int pair_first(int p) { return kTables<L>.first[p]; }

template <class L>
constexpr int n_pairs() { return (L::B - 1) / 2; }

template <class L>
constexpr int ray_scale(int p) { return kTables<L>.scale[p]; }

template <class L>
constexpr int ray_leader(int p) { return kTables<L>.leader[p]; }

// +1 / -1: pair p's direction equals / opposes its ray leader's
template <class L>
constexpr int ray_sign(int p) { return kTables<L>.sign[p]; }

// component a of the ray direction (the leader's primitive velocity)
template <class L>
constexpr int ray_dir(int leader, int a) { return kTables<L>.dir[leader][a]; }

}  // namespace mrtlb
