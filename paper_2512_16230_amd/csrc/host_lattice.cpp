// Host-side lattice builder: weights from the paper's weight equations,
// Hermite rows of order <= 3 with the rectangular-lattice correction of the
// pure third-order rows, and their W-norms.  All FP64.
#include "host_lattice.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <utility>

#include "kernels.h"
#include "lattices.h"

namespace mrtlb {

namespace {

template <class L>
void copy_velocities(HostLattice* out) {
  out->D = L::D;
  out->B = L::B;
  out->e.assign(L::B * L::D, 0);
  for (int j = 0; j < L::B; ++j) {
    out->e[j * L::D + 0] = L::EX[j];
    out->e[j * L::D + 1] = L::EY[j];
    if (L::D == 3) out->e[j * L::D + 2] = ez<L>(j);
  }
}

// Layer (max |e_a|) and the set of non-zero axes as a bit mask.
void classify(const int* ej, int D, int* layer, int* mask) {
  *layer = 0;
  *mask = 0;
  for (int a = 0; a < D; ++a) {
    int v = std::abs(ej[a]);
    if (v > *layer) *layer = v;
    if (v) *mask |= 1 << a;
  }
}

// rD2Q25 weights, Sec. V eq. (WeightQ25); free = {w13, w17, w18, w21}.
void weights_rd2q25(const double* c, double cs2, const double* fr, HostLattice* out) {
  const double d1 = cs2 / (c[0] * c[0]), d2 = cs2 / (c[1] * c[1]);
  const double w13 = fr[0], w17 = fr[1], w18 = fr[2], w21 = fr[3];
  const double w5 = (d1 * d2 - 64 * w13 - 324 * w21) / 4;
  const double w9 = (d1 * (3 * d1 - 1) - 48 * w13 - 144 * w17 - 288 * w21) / 24;
  const double w10 = (d2 * (3 * d2 - 1) - 48 * w13 - 144 * w18 - 288 * w21) / 24;
  const double w1 = d1 / 2 - (2 * w5 + 4 * w9 + 8 * w13 + 9 * w17 + 18 * w21);
  const double w2 = d2 / 2 - (2 * w5 + 4 * w10 + 8 * w13 + 9 * w18 + 18 * w21);
  const double w0 = 1 - 2 * (w1 + w2 + w9 + w10 + w17 + w18) - 4 * (w5 + w13 + w21);
  // [layer][mask]: mask 1 = x axis, 2 = y axis, 3 = diagonal
  const double tab[4][4] = {{w0, 0, 0, 0}, {0, w1, w2, w5}, {0, w9, w10, w13}, {0, w17, w18, w21}};
  out->w.resize(out->B);
  for (int j = 0; j < out->B; ++j) {
    int layer, mask;
    classify(&out->e[j * 2], 2, &layer, &mask);
    out->w[j] = tab[layer][mask];
  }
}

// App. C knight-move D2Q21 weights, free w9: w5, w17, w18, w1, w2, w0 in
// that order from eq. (new11); w9 on all eight knight moves.
void weights_d2q21k(const double* c, double cs2, double w9, HostLattice* out) {
  const double d1 = cs2 / (c[0] * c[0]), d2 = cs2 / (c[1] * c[1]);
  const double w5 = d1 * d2 / 4 - 8 * w9;
  const double w17 = (d1 * (3 * d1 - 1) - 48 * w9) / 144;
  const double w18 = (d2 * (3 * d2 - 1) - 48 * w9) / 144;
  const double w1 = d1 / 2 - 2 * w5 - 10 * w9 - 9 * w17;
  const double w2 = d2 / 2 - 2 * w5 - 10 * w9 - 9 * w18;
  const double w0 = 1 - 2 * (w1 + w2 + 2 * w5 + 4 * w9 + w17 + w18);
  // [layer][mask]: the knight moves are the layer-2 velocities, (+-3, 0) and
  // (0, +-3) the layer-3 ones
  const double tab[4][4] = {{w0, 0, 0, 0}, {0, w1, w2, w5}, {0, 0, 0, w9}, {0, w17, w18, 0}};
  out->w.resize(out->B);
  for (int j = 0; j < out->B; ++j) {
    int layer, mask;
    classify(&out->e[j * 2], 2, &layer, &mask);
    out->w[j] = tab[layer][mask];
  }
}

// rD2Q13 closed-form weights printed with Sec. V eq. (Q13lattice).
// Standard single-layer lattices: one D1Q3 weight per axis, 1 - d_a at
// rest and d_a / 2 at +-1 (d_a = cs^2 / c_a^2), multiplied over the axes:
// unit mass, Delta2 = cs^2 I and Delta4_aabb = cs^4 (a != b).
void weights_standard(const double* c, double cs2, HostLattice* out) {
  out->w.assign(out->B, 1.0);
  for (int j = 0; j < out->B; ++j)
    for (int a = 0; a < out->D; ++a) {
      const double d = cs2 / (c[a] * c[a]);
      out->w[j] *= out->e[j * out->D + a] != 0 ? 0.5 * d : 1.0 - d;
    }
}

void weights_rd2q13(const double* c, double cs2, HostLattice* out) {
  const double d1 = cs2 / (c[0] * c[0]), d2 = cs2 / (c[1] * c[1]);
  const double w9 = d1 * (3 * d1 - 1) / 24, w10 = d2 * (3 * d2 - 1) / 24;
  const double w0 = (1 - d1) * (1 - d2) + 6 * (w9 + w10);
  const double w1 = d1 * (1 - d2) / 2 - 4 * w9, w2 = d2 * (1 - d1) / 2 - 4 * w10;
  const double w5 = d1 * d2 / 4;
  const double tab[3][4] = {{w0, 0, 0, 0}, {0, w1, w2, w5}, {0, w9, w10, 0}};
  out->w.resize(out->B);
  for (int j = 0; j < out->B; ++j) {
    int layer, mask;
    classify(&out->e[j * 2], 2, &layer, &mask);
    out->w[j] = tab[layer][mask];
  }
}

// rD3Q53 (free = {w33, w37, w41, w45}) and rD3Q33 (no free weights), App. D,
// with d0a = cs^2 / c_a^2 as required by eq. (new11).
void weights_3d(const double* c, double cs2, const double* fr, bool q53, HostLattice* out) {
  const double d1 = cs2 / (c[0] * c[0]), d2 = cs2 / (c[1] * c[1]), d3 = cs2 / (c[2] * c[2]);
  const double w33 = q53 ? fr[0] : 0, w37 = q53 ? fr[1] : 0, w41 = q53 ? fr[2] : 0, w45 = q53 ? fr[3] : 0;
  const double w19 = d1 * d2 * d3 / 8 - 64 * w45;
  const double w7 = d1 * d2 / 4 - 2 * w19 - 16 * w33 - 32 * w45;
  const double w11 = d1 * d3 / 4 - 2 * w19 - 16 * w37 - 32 * w45;
  const double w15 = d2 * d3 / 4 - 2 * w19 - 16 * w41 - 32 * w45;
  const double w27 = d1 * (3 * d1 - 1) / 24 - 2 * (w33 + w37) - 4 * w45;
  const double w28 = d2 * (3 * d2 - 1) / 24 - 2 * (w33 + w41) - 4 * w45;
  const double w29 = d3 * (3 * d3 - 1) / 24 - 2 * (w41 + w37) - 4 * w45;
  const double w1 = d1 / 2 - 2 * (w7 + w11) - 4 * w19 - 4 * w27 - 8 * (w33 + w37) - 16 * w45;
  const double w2 = d2 / 2 - 2 * (w7 + w15) - 4 * w19 - 4 * w28 - 8 * (w33 + w41) - 16 * w45;
  const double w3 = d3 / 2 - 2 * (w11 + w15) - 4 * w19 - 4 * w29 - 8 * (w41 + w37) - 16 * w45;
  const double w0 = 1 - 2 * (w1 + w2 + w3 + w27 + w28 + w29) - 4 * (w7 + w11 + w15 + w33 + w37 + w41) -
                    8 * (w19 + w45);
  // [layer][mask]: mask bits x=1, y=2, z=4
  double tab[3][8] = {};
  tab[0][0] = w0;
  tab[1][1] = w1; tab[1][2] = w2; tab[1][4] = w3; tab[1][3] = w7; tab[1][5] = w11; tab[1][6] = w15; tab[1][7] = w19;
  tab[2][1] = w27; tab[2][2] = w28; tab[2][4] = w29; tab[2][3] = w33; tab[2][5] = w37; tab[2][6] = w41; tab[2][7] = w45;
  out->w.resize(out->B);
  for (int j = 0; j < out->B; ++j) {
    int layer, mask;
    classify(&out->e[j * 3], 3, &layer, &mask);
    out->w[j] = tab[layer][mask];
  }
}

double wdot(const HostLattice& L, const std::vector<double>& p, const std::vector<double>& q) {
  double s = 0;
  for (int j = 0; j < L.B; ++j) s += L.w[j] * p[j] * q[j];
  return s;
}

}  // namespace

int row_j(int, int a) { return 1 + a; }
int row_nn(int D, int a) { return 1 + D + a; }
int row_off(int D, int a, int b) {
  // 2D: xy -> 5; 3D: xy -> 7, xz -> 8, yz -> 9
  if (D == 2) return 5;
  const int k = (a == 0) ? (b == 1 ? 0 : 1) : 2;
  return 7 + k;
}
int row_abb(int D, int a, int b) {
  // 2D: xyy 6, yxx 7.  3D: xyy 10, xzz 11, yxx 12, yzz 13, zxx 14, zyy 15
  if (D == 2) return a == 0 ? 6 : 7;
  int k = 0;
  for (int aa = 0; aa < 3; ++aa)
    for (int bb = 0; bb < 3; ++bb) {
      if (aa == bb) continue;
      if (aa == a && bb == b) return 10 + k;
      ++k;
    }
  return -1;
}
int row_xyz() { return 16; }
int row_aaa(int D, int a) { return D == 2 ? 8 + a : 17 + a; }

mrtlb_status build_lattice(const mrtlb_lattice_desc& desc, HostLattice* out, std::string* err) {
  char buf[256];
  HostLattice L;
  L.kind = desc.kind;
  switch (desc.kind) {
    case kRD2Q25: copy_velocities<LatRD2Q25>(&L); break;
    case kRD2Q13: copy_velocities<LatRD2Q13>(&L); break;
    case kRD3Q53: copy_velocities<LatRD3Q53>(&L); break;
    case kRD3Q33: copy_velocities<LatRD3Q33>(&L); break;
    case kRD2Q21: copy_velocities<LatRD2Q21>(&L); break;
    case kD2Q21K: copy_velocities<LatD2Q21K>(&L); break;
    case kRD3Q45: copy_velocities<LatRD3Q45>(&L); break;
    case kRD2Q17_1: copy_velocities<LatRD2Q17_1>(&L); break;
    case kRD2Q17_2: copy_velocities<LatRD2Q17_2>(&L); break;
    case kRD2Q17_3: copy_velocities<LatRD2Q17_3>(&L); break;
    case kRD2Q17_4: copy_velocities<LatRD2Q17_4>(&L); break;
    case kRD2Q17_5: copy_velocities<LatRD2Q17_5>(&L); break;
    case kD2Q9: copy_velocities<LatD2Q9>(&L); break;
    case kD3Q27: copy_velocities<LatD3Q27>(&L); break;
    case kCustom: {
      if (!(desc.d == 2 || desc.d == 3) || desc.b < 2 || desc.b > kMaxB || !desc.e || !desc.w) {
        snprintf(buf, sizeof buf, "a custom lattice needs d in {2, 3}, 2 <= b <= %d and both arrays", kMaxB);
        *err = buf;
        return MRTLB_EINVAL;
      }
      L.D = desc.d;
      L.B = desc.b;
      L.e.assign(desc.e, desc.e + (size_t)desc.b * desc.d);
      for (int v : L.e)
        if (v < -8 || v > 8) {
          *err = "custom velocities must be integer multiples with |e| <= 8";
          return MRTLB_EINVAL;
        }
      L.w.assign(desc.w, desc.w + desc.b);
      double sum = 0;
      for (double v : L.w) sum += v;
      if (!(std::fabs(sum - 1.0) <= 1e-12)) {
        *err = "custom weights must sum to 1";
        return MRTLB_EINVAL;
      }
      break;
    }
    default:
      snprintf(buf, sizeof buf, "unknown lattice kind %d", desc.kind);
      *err = buf;
      return MRTLB_EINVAL;
  }
  const int D = L.D, B = L.B;
  const int need_free =
      (desc.kind == kRD2Q25 || desc.kind == kRD3Q53 || (desc.kind >= kRD2Q17_1 && desc.kind <= kRD2Q17_5)) ? 4
      : (desc.kind == kRD2Q21 || desc.kind == kRD3Q45) ? 3
      : desc.kind == kD2Q21K ? 1 : 0;
  if (desc.n_free != need_free) {
    snprintf(buf, sizeof buf, "lattice kind %d takes %d free weights, got %d", desc.kind, need_free, desc.n_free);
    *err = buf;
    return MRTLB_EINVAL;
  }
  if (!(desc.cs2 > 0) || !std::isfinite(desc.cs2)) {
    *err = "cs2 must be positive and finite";
    return MRTLB_EINVAL;
  }
  for (int a = 0; a < D; ++a) {
    if (!(desc.c[a] > 0) || !std::isfinite(desc.c[a])) {
      *err = "c_a must be positive and finite";
      return MRTLB_EINVAL;
    }
    L.c[a] = desc.c[a];
  }
  L.cs2 = desc.cs2;
  switch (desc.kind) {
    case kRD2Q25: weights_rd2q25(L.c, L.cs2, desc.free_w, &L); break;
    case kRD2Q13: weights_rd2q13(L.c, L.cs2, &L); break;
    case kRD3Q53: weights_3d(L.c, L.cs2, desc.free_w, true, &L); break;
    case kRD3Q33: weights_3d(L.c, L.cs2, nullptr, false, &L); break;
    case kRD2Q21: {
      // Sec. V item (i): the rD2Q25 weights with w21 = 0
      const double fr[4] = {desc.free_w[0], desc.free_w[1], desc.free_w[2], 0.0};
      weights_rd2q25(L.c, L.cs2, fr, &L);
      break;
    }
    case kD2Q21K: weights_d2q21k(L.c, L.cs2, desc.free_w[0], &L); break;
    case kRD2Q17_1: case kRD2Q17_2: case kRD2Q17_3: case kRD2Q17_4: case kRD2Q17_5: {
      // the rD2Q25 weights (free = {w13, w17, w18, w21}); the groups the case
      // drops must come out zero
      HostLattice full;
      copy_velocities<LatRD2Q25>(&full);
      weights_rd2q25(L.c, L.cs2, desc.free_w, &full);
      L.w.assign(B, 0.0);
      for (int k = 0; k < full.B; ++k) {
        int hit = -1;
        for (int j = 0; j < B; ++j)
          if (L.e[j * 2] == full.e[k * 2] && L.e[j * 2 + 1] == full.e[k * 2 + 1]) hit = j;
        if (hit >= 0) {
          L.w[hit] = full.w[k];
        } else if (std::fabs(full.w[k]) > 1e-12) {
          snprintf(buf, sizeof buf,
                   "the weight of dropped velocity (%d, %d) is %.3g, not 0: cs2 and the free weights do not give "
                   "this D2Q17 case", full.e[k * 2], full.e[k * 2 + 1], full.w[k]);
          *err = buf;
          return MRTLB_EINVAL;
        }
      }
      break;
    }
    case kRD3Q45: {
      // the rD3Q53 weights with w45 = 0
      const double fr[4] = {desc.free_w[0], desc.free_w[1], desc.free_w[2], 0.0};
      weights_3d(L.c, L.cs2, fr, true, &L);
      break;
    }
    case kD2Q9: case kD3Q27: weights_standard(L.c, L.cs2, &L); break;
    case kCustom: break;   // given
  }
  for (int j = 0; j < B; ++j) {
    if (!(L.w[j] > 0)) {
      snprintf(buf, sizeof buf, "weight w[%d] = %.6g is not positive for these c, cs2 and free weights", j, L.w[j]);
      *err = buf;
      return MRTLB_ENUMERIC;
    }
  }

  // Physical velocities.
  std::vector<double> cv(B * D);
  for (int j = 0; j < B; ++j)
    for (int a = 0; a < D; ++a) cv[j * D + a] = L.c[a] * L.e[j * D + a];
  auto cc = [&](int j, int a) { return cv[j * D + a]; };
  const double cs2 = L.cs2;

  // Standard lattices: c_a^3 = c_a^2 c_a on one layer, so the pure rows
  // would repeat the first-order rows; they are left out (rows are built
  // in the full order and the first nlow kept).
  L.standard = desc.kind == kD2Q9 || desc.kind == kD3Q27;
  const int nfull = D == 2 ? 10 : 20;
  L.nlow = L.standard ? nfull - D : nfull;
  std::vector<std::vector<double>> rows(nfull, std::vector<double>(B, 0.0));
  for (int j = 0; j < B; ++j) {
    rows[0][j] = 1.0;
    for (int a = 0; a < D; ++a) {
      rows[row_j(D, a)][j] = cc(j, a);
      rows[row_nn(D, a)][j] = cc(j, a) * cc(j, a) - cs2;
      for (int b = a + 1; b < D; ++b) rows[row_off(D, a, b)][j] = cc(j, a) * cc(j, b);
      for (int b = 0; b < D; ++b)
        if (b != a) rows[row_abb(D, a, b)][j] = cc(j, a) * (cc(j, b) * cc(j, b) - cs2);
      rows[row_aaa(D, a)][j] = cc(j, a) * (cc(j, a) * cc(j, a) - 3 * cs2);
    }
    if (D == 3) rows[row_xyz()][j] = cc(j, 0) * cc(j, 1) * cc(j, 2);
  }
  // Correction: remove from each pure row its W-projection on the span of
  // the mixed rows c_a (c_b^2 - cs^2), b != a.  The Gram system is at most
  // 2 x 2 and solved directly.
  for (int a = 0; a < D && !L.standard; ++a) {
    int bs[2], nb = 0;
    for (int b = 0; b < D; ++b)
      if (b != a) bs[nb++] = b;
    const std::vector<double>& p = rows[row_aaa(D, a)];
    double G[2][2], r[2], x[2];
    for (int i = 0; i < nb; ++i) {
      r[i] = wdot(L, p, rows[row_abb(D, a, bs[i])]);
      for (int k = 0; k < nb; ++k) G[i][k] = wdot(L, rows[row_abb(D, a, bs[i])], rows[row_abb(D, a, bs[k])]);
    }
    if (nb == 1) {
      if (!(std::fabs(G[0][0]) > 0)) { *err = "singular correction system"; return MRTLB_ENUMERIC; }
      x[0] = r[0] / G[0][0];
    } else {
      const double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
      if (!(std::fabs(det) > 1e-300)) { *err = "singular correction system"; return MRTLB_ENUMERIC; }
      x[0] = (r[0] * G[1][1] - r[1] * G[0][1]) / det;
      x[1] = (r[1] * G[0][0] - r[0] * G[1][0]) / det;
    }
    std::vector<double>& pr = rows[row_aaa(D, a)];
    for (int i = 0; i < nb; ++i) {
      L.corr[a][bs[i]] = x[i];
      const std::vector<double>& m = rows[row_abb(D, a, bs[i])];
      for (int j = 0; j < B; ++j) pr[j] -= x[i] * m[j];
    }
  }
  L.H.assign(L.nlow * B, 0.0);
  L.norms.assign(L.nlow, 0.0);
  for (int r = 0; r < L.nlow; ++r) {
    for (int j = 0; j < B; ++j) L.H[r * B + j] = rows[r][j];
    L.norms[r] = wdot(L, rows[r], rows[r]);
    if (!(L.norms[r] > 0)) { *err = "zero Hermite norm"; return MRTLB_ENUMERIC; }
  }
  // The reduced collision needs W-orthogonal rows of order <= 3 (the
  // paper's lattices meet this by construction; a custom set must).
  for (int r = 0; r < L.nlow; ++r)
    for (int q = r + 1; q < L.nlow; ++q) {
      const double g = wdot(L, rows[r], rows[q]);
      if (!(std::fabs(g) <= 1e-10 * std::sqrt(L.norms[r] * L.norms[q]))) {
        snprintf(buf, sizeof buf, "Hermite rows %d and %d are not W-orthogonal (relative inner product %.3g)", r, q,
                 g / std::sqrt(L.norms[r] * L.norms[q]));
        *err = buf;
        return MRTLB_ENUMERIC;
      }
    }
  *out = std::move(L);
  return MRTLB_OK;
}

// Slot order for the user-supplied lattices' step kernel (host_lattice.h).
std::vector<int> velocity_slots(const HostLattice& L, bool rays, int* nrays, int* npairs, std::vector<int>* mult) {
  const int D = L.D;
  auto comp = [&](int j, int a) { return L.e[j * D + a]; };
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> singles;
  std::vector<char> used(L.B, 0);
  auto opposite = [&](int i, int j) {
    bool any = false;
    for (int a = 0; a < D; ++a) {
      if (comp(i, a) != -comp(j, a)) return false;
      any |= comp(i, a) != 0;
    }
    return any;
  };
  for (int i = 0; i < L.B; ++i) {
    if (used[i]) continue;
    used[i] = 1;
    int partner = -1;
    for (int j = i + 1; j < L.B && partner < 0; ++j)
      if (!used[j] && opposite(i, j)) partner = j;
    if (partner >= 0) {
      used[partner] = 1;
      pairs.emplace_back(i, partner);
    } else {
      singles.push_back(i);
    }
  }
  // c such that e_j = c e_i (0 if none)
  auto multiple = [&](int i, int j) {
    int c = 0;
    for (int a = 0; a < D; ++a) {
      if (comp(i, a) == 0) {
        if (comp(j, a) != 0) return 0;
        continue;
      }
      if (comp(j, a) % comp(i, a) != 0) return 0;
      const int q = comp(j, a) / comp(i, a);
      if (q < 2 || (c != 0 && q != c)) return 0;
      c = q;
    }
    return c;
  };
  auto norm1 = [&](int j) {
    int n = 0;
    for (int a = 0; a < D; ++a) n += std::abs(comp(j, a));
    return n;
  };
  std::vector<size_t> order(pairs.size());
  for (size_t p = 0; p < pairs.size(); ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return norm1(pairs[x].first) < norm1(pairs[y].first); });
  std::vector<char> taken(pairs.size(), 0);
  std::vector<int> slots, rest;
  mult->clear();
  for (size_t oi = 0; oi < (rays ? order.size() : 0); ++oi) {
    const size_t p = order[oi];
    if (taken[p]) continue;
    const int base = pairs[p].first;
    int best = -1, bestc = 0;
    bool flip = false;
    for (size_t q = 0; q < pairs.size(); ++q) {
      if (q == p || taken[q]) continue;
      for (int side = 0; side < 2; ++side) {
        const int c = multiple(base, side ? pairs[q].second : pairs[q].first);
        if (c >= 2 && (best < 0 || c < bestc)) {
          best = (int)q;
          bestc = c;
          flip = side == 1;
        }
      }
    }
    if (best < 0) continue;
    taken[p] = taken[best] = 1;
    const auto& qp = pairs[best];
    slots.insert(slots.end(), {base, pairs[p].second, flip ? qp.second : qp.first, flip ? qp.first : qp.second});
    mult->push_back(bestc);
  }
  *nrays = (int)mult->size();
  int np = 0;
  for (size_t p = 0; p < pairs.size(); ++p)
    if (!taken[p]) {
      slots.push_back(pairs[p].first);
      slots.push_back(pairs[p].second);
      ++np;
    }
  *npairs = np;
  slots.insert(slots.end(), singles.begin(), singles.end());
  return slots;
}

}  // namespace mrtlb
