// MI355X (gfx950) kernels and C ABI of the Hermite-matrix MRT lattice
// Boltzmann method (arXiv 2512.16230): fused pull collide-and-stream,
// initialisation, moment read-out, checkpoint and FP64 conserved sums.
//
// Layout in HBM: populations structure-of-arrays, f[j][z][y][x] (x fastest),
// two buffers (pull propagation, double-buffered).  The buffer holds the
// post-collision populations of the previous step, so f_bar_j(x, t) =
// buf_j(x - e_j): a step gathers along -e_j, collides in registers and
// writes every population at its own node (coalesced stores).
//
// Collision (per node, registers only).  With the component Hermite rows of
// order <= 3 (H0 = 1, H1 = c, H2 = cc - cs^2, H3 mixed / xyz / corrected
// pure) and every row above third order relaxing at the single rate s_h,
// the update of eq. (2-3) with Lambda = H^-1 S H is
//     f* = (1 - s_h) f + W sum_{r<=3} H_r (m*_r - (1 - s_h) m_r) / n_r
// (the reduced form of eq. H-MRT-LB-1).  The forward moments are taken as
// raw monomial sums over symmetric velocity pairs (even monomials from
// f_p + f_q, odd ones from f_p - f_q) and the back-transform as a monomial
// polynomial evaluated per pair, so each population costs a few FMAs and no
// b x b matrix is formed.  The normal second-order rows relax their trace at
// s_bulk and their deviator at s_shear.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/mrtlb.h"
#include "host_lattice.h"
#include "kernels.h"
#include "lattices.h"

namespace mrtlb {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <class L>
constexpr int evel(int j, int a) {
  return a == 0 ? L::EX[j] : (a == 1 ? L::EY[j] : ez<L>(j));
}

constexpr int off_index(int a, int b) { return a == 0 ? (b == 1 ? 0 : 1) : 2; }

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <int ST>
struct StoreT;
template <>
struct StoreT<kFP64> { using T = double; using Real = double; };
template <>
struct StoreT<kFP32> { using T = float; using Real = float; };
template <>
struct StoreT<kFP32Dev> { using T = float; using Real = float; };
template <>
struct StoreT<kFP16Dev> { using T = _Float16; using Real = float; };
template <>
struct StoreT<kBF16Dev> { using T = uint16_t; using Real = float; };

template <int ST, class Real>
__device__ __forceinline__ Real load_pop(const typename StoreT<ST>::T* p, uint32_t i, const KParams<Real>& P, int j) {
  if constexpr (ST == kFP16Dev) {
    return (Real)(float)p[i] * P.wsc[j];
  } else if constexpr (ST == kBF16Dev) {
    return (Real)bf16_to_f32(p[i]) * P.wsc[j];
  } else {
    return (Real)p[i];
  }
}

template <int ST, class Real>
__device__ __forceinline__ void store_pop(typename StoreT<ST>::T* p, uint32_t i, Real v, const KParams<Real>& P, int j) {
  if constexpr (ST == kFP16Dev) {
    p[i] = (_Float16)(float)(v * P.iwsc[j]);
  } else if constexpr (ST == kBF16Dev) {
    p[i] = f32_to_bf16_rne((float)(v * P.iwsc[j]));
  } else {
    p[i] = (typename StoreT<ST>::T)v;
  }
}

// ---------------------------------------------------------------------------
// node geometry: wrapped neighbour offsets for -MAXE..MAXE along each axis
// ---------------------------------------------------------------------------

template <class L>
struct NodeGeom {
  static constexpr int M = L::MAXE;
  uint32_t xo[2 * M + 1];   // wrap(ix - s)
  uint32_t yo[2 * M + 1];   // wrap(iy - s) * nx
  uint32_t zo[2 * M + 1];   // wrap(iz - s) * nx * ny
  uint32_t self;

  __device__ __forceinline__ void init(int ix, int iy, int iz, int nx, int ny, int nz) {
#pragma unroll
    for (int s = -M; s <= M; ++s) {
      xo[s + M] = (uint32_t)wrap(ix - s, nx);
      yo[s + M] = (uint32_t)wrap(iy - s, ny) * (uint32_t)nx;
      if constexpr (L::D == 3) zo[s + M] = (uint32_t)wrap(iz - s, nz) * (uint32_t)nx * (uint32_t)ny;
    }
    self = xo[M] + yo[M] + (L::D == 3 ? zo[M] : 0u);
  }
  // element index of the source of population j (pull: x - e_j)
  template <int J>
  __device__ __forceinline__ uint32_t src() const {
    uint32_t i = xo[L::EX[J] + M] + yo[L::EY[J] + M];
    if constexpr (L::D == 3) i += zo[ez<L>(J) + M];
    return i;
  }
  // element index of x + s_a along axis a (s = +-1)
  __device__ __forceinline__ uint32_t shifted(int a, int s) const {
    uint32_t xi = xo[M], yi = yo[M], zi = (L::D == 3 ? zo[M] : 0u);
    if (a == 0) xi = xo[M - s];
    if (a == 1) yi = yo[M - s];
    if constexpr (L::D == 3) {
      if (a == 2) zi = zo[M - s];
    }
    return xi + yi + zi;
  }
};

// ---------------------------------------------------------------------------
// moments of a node
// ---------------------------------------------------------------------------

template <class Real>
struct Moments {
  Real R0;
  Real m1[3], m2n[3], m2o[3], m3m[3][3], m3p[3], mxyz;
};

// Hermite moments (component rows, physical units) of x[0..B-1].
template <class L, class Real>
__device__ __forceinline__ void forward(const Real (&x)[L::B], const KParams<Real>& P, Moments<Real>& M) {
  constexpr int D = L::D;
  Real R0 = x[0];
  Real R1[3] = {0, 0, 0}, R2n[3] = {0, 0, 0}, R2o[3] = {0, 0, 0}, R3p[3] = {0, 0, 0};
  Real R3m[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  Real Rxyz = 0;
  static_for<0, n_pairs<L>()>([&](auto kk) {
    constexpr int p = pair_first<L>(decltype(kk)::value);
    constexpr int q = opposite<L>(p);
    const Real s = x[p] + x[q];
    const Real d = x[p] - x[q];
    R0 += s;
    static_for<0, D>([&](auto aa) {
      constexpr int a = decltype(aa)::value;
      constexpr int ea = evel<L>(p, a);
      if constexpr (ea != 0) {
        R1[a] += Real(ea) * d;
        R2n[a] += Real(ea * ea) * s;
        R3p[a] += Real(ea * ea * ea) * d;
        static_for<0, D>([&](auto bb) {
          constexpr int b = decltype(bb)::value;
          constexpr int eb = evel<L>(p, b);
          if constexpr (b != a && eb != 0) R3m[a][b] += Real(ea * eb * eb) * d;
          if constexpr (b > a && eb != 0) R2o[off_index(a, b)] += Real(ea * eb) * s;
        });
      }
    });
    if constexpr (D == 3) {
      constexpr int exyz = evel<L>(p, 0) * evel<L>(p, 1) * evel<L>(p, 2);
      if constexpr (exyz != 0) Rxyz += Real(exyz) * d;
    }
  });
  M.R0 = R0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    M.m1[a] = P.c1[a] * R1[a];
    M.m2n[a] = P.c2[a] * R2n[a] - P.cs2 * R0;
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a + 1; b < D; ++b) M.m2o[off_index(a, b)] = P.cab[off_index(a, b)] * R2o[off_index(a, b)];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real pure = P.c3[a] * R3p[a] - 3 * P.cs2 * M.m1[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      M.m3m[a][b] = P.cabb[a][b] * R3m[a][b] - P.cs2 * M.m1[a];
      pure -= P.corr[a][b] * M.m3m[a][b];
    }
    M.m3p[a] = pure;
  }
  if constexpr (D == 3) M.mxyz = P.cxyz * Rxyz;
}

// Per-row coefficients delta_r = (target_r) / n_r turned into monomial
// coefficients in lattice units, then evaluated per velocity pair:
//   x_j <- kx * x_j + w_j * sum_P beta_P e_j^P
template <class L, class Real>
__device__ __forceinline__ void backward(Real (&x)[L::B], const KParams<Real>& P, Real kx, Real d0, const Real* d1,
                                         const Real* d2n, const Real* d2o, const Real (*d3m)[3], const Real* d3p,
                                         Real dxyz) {
  constexpr int D = L::D;
  Real b0 = d0;
  Real b1[3], b2n[3], b2o[3], b3m[3][3], b3p[3];
#pragma unroll
  for (int a = 0; a < D; ++a) b0 -= P.cs2 * d2n[a];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real t = d1[a] + P.k3[a] * d3p[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      t -= P.cs2 * d3m[a][b];
      b3m[a][b] = P.cabb[a][b] * (d3m[a][b] - P.corr[a][b] * d3p[a]);
    }
    b1[a] = P.c1[a] * t;
    b2n[a] = P.c2[a] * d2n[a];
    b3p[a] = P.c3[a] * d3p[a];
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a + 1; b < D; ++b) b2o[off_index(a, b)] = P.cab[off_index(a, b)] * d2o[off_index(a, b)];
  Real bxyz = 0;
  if constexpr (D == 3) bxyz = P.cxyz * dxyz;
  x[0] = kx * x[0] + P.w[0] * b0;
  static_for<0, n_pairs<L>()>([&](auto kk) {
    constexpr int p = pair_first<L>(decltype(kk)::value);
    constexpr int q = opposite<L>(p);
    Real even = b0, odd = 0;
    static_for<0, D>([&](auto aa) {
      constexpr int a = decltype(aa)::value;
      constexpr int ea = evel<L>(p, a);
      if constexpr (ea != 0) {
        even += Real(ea * ea) * b2n[a];
        odd += Real(ea) * b1[a] + Real(ea * ea * ea) * b3p[a];
        static_for<0, D>([&](auto bb) {
          constexpr int b = decltype(bb)::value;
          constexpr int eb = evel<L>(p, b);
          if constexpr (b != a && eb != 0) odd += Real(ea * eb * eb) * b3m[a][b];
          if constexpr (b > a && eb != 0) even += Real(ea * eb) * b2o[off_index(a, b)];
        });
      }
    });
    if constexpr (D == 3) {
      constexpr int exyz = evel<L>(p, 0) * evel<L>(p, 1) * evel<L>(p, 2);
      if constexpr (exyz != 0) odd += Real(exyz) * bxyz;
    }
    const Real wp = P.w[p];
    x[p] = kx * x[p] + wp * (even + odd);
    x[q] = kx * x[q] + wp * (even - odd);
  });
}

// Equilibrium Hermite moments (orders 1..3) from the conserved variables.
template <class L, class Real, int MODEL>
struct Equilibrium {
  Real e1[3], e2n[3], e2o[3], e3m[3][3], e3p[3], exyz;

  // NSE: j = rho_m u (momentum incl. the half force), u = j / rho_m.
  // NCDE: phi, u = advection velocity.
  __device__ __forceinline__ void build(const KParams<Real>& P, Real rho_or_phi, const Real* j, const Real* u) {
    constexpr int D = L::D;
    if constexpr (MODEL == kNcde) {
      const Real phi = rho_or_phi;
      const Real Phi = P.phi_coef * (phi + P.D2 * phi * phi * phi * Real(1.0 / 3.0));
#pragma unroll
      for (int a = 0; a < D; ++a) {
        e1[a] = phi * u[a];
        e2n[a] = P.cs2 * (Phi - phi) + e1[a] * u[a];
        e3p[a] = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) e3m[a][b] = 0;
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) e2o[off_index(a, b)] = e1[a] * u[b];
      exyz = 0;
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        e1[a] = j[a];
        e2n[a] = j[a] * u[a];
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) e2o[off_index(a, b)] = j[a] * u[b];
      if (P.m30) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          Real pure = e2n[a] * u[a];
#pragma unroll
          for (int b = 0; b < D; ++b) {
            if (b == a) continue;
            e3m[a][b] = e2n[b] * u[a];  // rho u_a u_b^2
            pure -= P.corr[a][b] * e3m[a][b];
          }
          e3p[a] = pure;
        }
        if constexpr (D == 3) exyz = j[0] * u[1] * u[2];
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          e3p[a] = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) e3m[a][b] = 0;
        }
        exyz = 0;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// the fused collide-and-stream step
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t xcd_remap(uint32_t lin, uint32_t total) {
  // Workgroups are dealt to the XCDs round-robin; give every XCD a
  // contiguous range of tiles so that neighbouring tiles (which share
  // partially-read cache lines and halo rows) meet in the same L2.
  const uint32_t q = total / kNumXcd;
  if (lin >= q * kNumXcd) return lin;
  return (lin % kNumXcd) * q + lin / kNumXcd;
}

template <class Real>
__device__ __forceinline__ int find_job(const Job<Real>* jobs, int njobs, uint32_t lin) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= lin) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class L, class Real>
__device__ __forceinline__ bool tile_node(const Job<Real>& J, uint32_t local, int& ix, int& iy, int& iz) {
  const int bxs = J.bx_shift;
  const int rows = kBlock >> bxs;
  const uint32_t tx = local % (uint32_t)J.gx;
  const uint32_t rg = local / (uint32_t)J.gx;
  const int ny = J.P.ny;
  const uint32_t rgy = (uint32_t)((ny + rows - 1) / rows);
  const int tid = threadIdx.x;
  ix = (int)(tx << bxs) + (tid & ((1 << bxs) - 1));
  iy = (int)(rg % rgy) * rows + (tid >> bxs);
  iz = (int)(rg / rgy);
  return ix < J.P.nx && iy < ny;
}

template <class L, int ST, int MODEL, bool FORCE>
__global__ __launch_bounds__(kBlock) void k_step(const Job<typename StoreT<ST>::Real>* __restrict__ jobs, int njobs,
                                                uint32_t total_blocks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B, D = L::D;
  const uint32_t lin = xcd_remap(blockIdx.x, total_blocks);
  const int jb = njobs > 1 ? find_job(jobs, njobs, lin) : 0;
  const Job<Real>& J = jobs[jb];
  const KParams<Real>& P = J.P;
  int ix, iy, iz;
  if (!tile_node<L>(J, lin - J.block_begin, ix, iy, iz)) return;
  NodeGeom<L> g;
  g.init(ix, iy, iz, P.nx, P.ny, P.nz);
  const uint32_t N = P.N;
  const T* __restrict__ fin = static_cast<const T*>(J.fin);
  T* __restrict__ fout = static_cast<T*>(J.fout);

  // a1: gather along -e_j
  Real x[B];
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    x[j] = load_pop<ST>(fin + (size_t)j * N, g.template src<j>(), P, j);
  });

  // a3: forward Hermite moments
  Moments<Real> M;
  forward<L>(x, P, M);

  // a2: conserved variables, a5: sources
  Real F[3] = {0, 0, 0}, src1[3] = {0, 0, 0}, T2n[3] = {0, 0, 0}, T2o[3] = {0, 0, 0};
  Real u[3], jm[3];
  const Real R = M.R0 + P.rho_ref;
  if constexpr (MODEL == kNcde) {
    const Real phi_prev = J.phi_prev[g.self];
    Real adv = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      u[a] = P.adv[a];
      const Real grad = (J.phi_prev[g.shifted(a, 1)] - J.phi_prev[g.shifted(a, -1)]) / (2 * P.c1[a]);
      adv += u[a] * grad;
    }
    const Real scal = (R - phi_prev) + adv;
#pragma unroll
    for (int a = 0; a < D; ++a) src1[a] = u[a] * scal;
    J.phi_out[g.self] = R;
  } else {
    if constexpr (FORCE) {
#pragma unroll
      for (int a = 0; a < D; ++a) F[a] = J.force[(size_t)a * N + g.self];
    }
    const Real rho_m = P.inc ? P.rho0 : R;
    const Real inv = Real(1) / rho_m;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      jm[a] = M.m1[a] + Real(0.5) * F[a];
      u[a] = jm[a] * inv;
      src1[a] = F[a];
    }
    if constexpr (FORCE) {
#pragma unroll
      for (int a = 0; a < D; ++a) T2n[a] = 2 * u[a] * F[a];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) T2o[off_index(a, b)] = u[a] * F[b] + u[b] * F[a];
    }
  }

  // a4: equilibrium moments
  Equilibrium<L, Real, MODEL> E;
  E.build(P, R, jm, u);

  // a6: relaxation; targets t_r = m*_r - (1 - s_h) m_r, scaled by 1/n_r
  const Real kx = Real(1) - P.sh;
  Real d1[3], d2n[3], d2o[3], d3m[3][3], d3p[3], dxyz = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const Real ms = M.m1[a] - P.s1 * (M.m1[a] - E.e1[a]) + (Real(1) - Real(0.5) * P.s1) * src1[a];
    d1[a] = (ms - kx * M.m1[a]) * P.in1[a];
  }
  {
    Real neq[3], tn = 0, tT = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      neq[a] = M.m2n[a] - E.e2n[a];
      tn += neq[a];
      tT += T2n[a];
    }
    tn *= Real(1.0 / D);
    tT *= Real(1.0 / D);
    const Real kb = Real(1) - P.sb, ks = Real(1) - P.ss;
    const Real gb = Real(1) - Real(0.5) * P.sb, gs = Real(1) - Real(0.5) * P.ss;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const Real ms = E.e2n[a] + kb * tn + ks * (neq[a] - tn) + gb * tT + gs * (T2n[a] - tT);
      d2n[a] = (ms - kx * M.m2n[a]) * P.in2n[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) {
        const int o = off_index(a, b);
        const Real ms = E.e2o[o] + ks * (M.m2o[o] - E.e2o[o]) + gs * T2o[o];
        d2o[o] = (ms - kx * M.m2o[o]) * P.in2o[o];
      }
  }
  {
    const Real k3 = Real(1) - P.s3;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      d3p[a] = (E.e3p[a] + k3 * (M.m3p[a] - E.e3p[a]) - kx * M.m3p[a]) * P.in3p[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        d3m[a][b] = (E.e3m[a][b] + k3 * (M.m3m[a][b] - E.e3m[a][b]) - kx * M.m3m[a][b]) * P.in3m[a][b];
      }
    }
    if constexpr (D == 3) dxyz = (E.exyz + k3 * (M.mxyz - E.exyz) - kx * M.mxyz) * P.inxyz;
  }
  // order 0 is conserved: m*_0 = m_0
  const Real d0 = P.sh * M.R0 * P.in0;

  // a7: back to populations
  backward<L>(x, P, kx, d0, d1, d2n, d2o, d3m, d3p, dxyz);

  // a8: store at the own node
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    store_pop<ST>(fout + (size_t)j * N, g.self, x[j], P, j);
  });
}

// ---------------------------------------------------------------------------
// initialisation: f_bar(x,0) = f_eq - F/2, written at x - e_j (inverse of the
// pull gather).  Computed in FP64 regardless of the storage.
// ---------------------------------------------------------------------------

template <class L, int ST, int MODEL>
__global__ __launch_bounds__(kBlock) void k_init(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                const KParams<double>* __restrict__ PD, const double* __restrict__ rho,
                                                const double* __restrict__ uin, const double* __restrict__ fin,
                                                uint32_t total_blocks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B, D = L::D;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!tile_node<L>(J, blockIdx.x, ix, iy, iz)) return;
  NodeGeom<L> g;
  g.init(ix, iy, iz, P.nx, P.ny, P.nz);
  const uint32_t N = P.N;
  const double R = rho[g.self];
  double u[3] = {0, 0, 0}, jm[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  if constexpr (MODEL == kNcde) {
    for (int a = 0; a < D; ++a) u[a] = P.adv[a];
    static_cast<Real*>(J.phi_out)[g.self] = (Real)R;
    const_cast<Real*>(J.phi_prev)[g.self] = (Real)R;
  } else {
    const double rho_m = P.inc ? P.rho0 : R;
    for (int a = 0; a < D; ++a) {
      u[a] = uin[(size_t)a * N + g.self];
      jm[a] = rho_m * u[a];
      if (fin) F[a] = fin[(size_t)a * N + g.self];
    }
  }
  Equilibrium<L, double, MODEL> E;
  E.build(P, R, jm, u);
  double d1[3], d2n[3], d2o[3], d3m[3][3], d3p[3], dxyz = 0;
  for (int a = 0; a < D; ++a) {
    d1[a] = (E.e1[a] - 0.5 * F[a]) * P.in1[a];
    d2n[a] = E.e2n[a] * P.in2n[a];
    d3p[a] = E.e3p[a] * P.in3p[a];
    for (int b = 0; b < D; ++b)
      if (b != a) d3m[a][b] = E.e3m[a][b] * P.in3m[a][b];
    for (int b = a + 1; b < D; ++b) d2o[off_index(a, b)] = E.e2o[off_index(a, b)] * P.in2o[off_index(a, b)];
  }
  if constexpr (D == 3) dxyz = E.exyz * P.inxyz;
  double x[B];
  for (int j = 0; j < B; ++j) x[j] = 0;
  const double d0 = R * P.in0 - P.rho_ref;
  backward<L>(x, P, 0.0, d0, d1, d2n, d2o, d3m, d3p, dxyz);
  T* __restrict__ out = static_cast<T*>(J.fout);
  const KParams<Real>& PR = J.P;
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    // buf_j(x - e_j) = f_bar_j(x): the source index of the pull gather
    store_pop<ST>(out + (size_t)j * N, g.template src<j>(), (Real)x[j], PR, j);
  });
}

// ---------------------------------------------------------------------------
// read-out: gather f_bar(x, t) and compute moments or copy populations
// ---------------------------------------------------------------------------

template <class L, int ST, int MODEL, int WHAT>  // WHAT 0: moments, 1: populations
__global__ __launch_bounds__(kBlock) void k_gather(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                  const KParams<double>* __restrict__ PD, double* __restrict__ out0,
                                                  double* __restrict__ out1) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B, D = L::D;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!tile_node<L>(J, blockIdx.x, ix, iy, iz)) return;
  NodeGeom<L> g;
  g.init(ix, iy, iz, P.nx, P.ny, P.nz);
  const uint32_t N = P.N;
  const T* __restrict__ fin = static_cast<const T*>(J.fin);
  double x[B];
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    x[j] = (double)load_pop<ST>(fin + (size_t)j * N, g.template src<j>(), J.P, j);
  });
  if constexpr (WHAT == 1) {
    for (int j = 0; j < B; ++j) out0[(size_t)j * N + g.self] = x[j] + P.w[j] * P.rho_ref;
  } else {
    double R = 0, m1[3] = {0, 0, 0};
    static_for<0, B>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      R += x[j];
      static_for<0, D>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        if constexpr (evel<L>(j, a) != 0) m1[a] += double(evel<L>(j, a)) * x[j];
      });
    });
    R += P.rho_ref;
    out0[g.self] = R;
    if (out1) {
      if constexpr (MODEL == kNcde) {
        for (int a = 0; a < D; ++a) out1[(size_t)a * N + g.self] = P.adv[a];
      } else {
        const double rho_m = P.inc ? P.rho0 : R;
        for (int a = 0; a < D; ++a) {
          double jm = P.c1[a] * m1[a];
          if (J.force) jm += 0.5 * (double)J.force[(size_t)a * N + g.self];
          out1[(size_t)a * N + g.self] = jm / rho_m;
        }
      }
    }
  }
}

// Restore: buf_j(x - e_j) = f_bar_j(x) - w_j rho_ref.
template <class L, int ST>
__global__ __launch_bounds__(kBlock) void k_scatter(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                   const KParams<double>* __restrict__ PD, const double* __restrict__ in) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!tile_node<L>(J, blockIdx.x, ix, iy, iz)) return;
  NodeGeom<L> g;
  g.init(ix, iy, iz, P.nx, P.ny, P.nz);
  const uint32_t N = P.N;
  T* __restrict__ out = static_cast<T*>(J.fout);
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    const double v = in[(size_t)j * N + g.self] - P.w[j] * P.rho_ref;
    store_pop<ST>(out + (size_t)j * N, g.template src<j>(), (Real)v, J.P, j);
  });
}

// ---------------------------------------------------------------------------
// FP64 plane sums (conserved quantities): partial[plane][chunk] over chunks
// of kBlock * kChunkIters elements, wavefront shuffles then a fixed LDS tree.
// ---------------------------------------------------------------------------

constexpr int kChunkIters = 16;

template <int ST>
__global__ __launch_bounds__(kBlock) void k_plane_sums(const void* __restrict__ base, uint32_t N, int nplanes_pop,
                                                      const typename StoreT<ST>::Real* __restrict__ force, int nforce,
                                                      const KParams<typename StoreT<ST>::Real>* __restrict__ PR,
                                                      double* __restrict__ partial, uint32_t nchunks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  const uint32_t chunk = blockIdx.x;
  const int plane = blockIdx.y;
  const uint32_t begin = chunk * (uint32_t)(kBlock * kChunkIters);
  double acc = 0;
  for (int it = 0; it < kChunkIters; ++it) {
    const uint32_t i = begin + (uint32_t)it * kBlock + threadIdx.x;
    if (i < N) {
      if (plane < nplanes_pop) {
        const T* p = static_cast<const T*>(base) + (size_t)plane * N;
        acc += (double)load_pop<ST>(p, i, *PR, plane);
      } else {
        acc += (double)force[(size_t)(plane - nplanes_pop) * N + i];
      }
    }
  }
  // wavefront reduction (64 lanes), fixed butterfly order
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < kBlock / 64; ++k) s += red[k];
    partial[(size_t)plane * nchunks + chunk] = s;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

thread_local std::string g_last_error;

static mrtlb_status fail(mrtlb_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(MRTLB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

}  // namespace mrtlb

using namespace mrtlb;

struct mrtlb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t used = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct mrtlb_lattice {
  HostLattice L;
};

struct mrtlb_solve {
  mrtlb_ctx* ctx = nullptr;
  HostLattice L;
  mrtlb_model_desc model{};
  int storage = 0;
  int has_force = 0;
  int nx = 1, ny = 1, nz = 1;
  uint32_t N = 0;
  size_t bytes = 0;
  void* f[2] = {nullptr, nullptr};
  void* force = nullptr;        // Real, d x N
  void* phi[2] = {nullptr, nullptr};
  void* jobs = nullptr;         // two Job<Real> (parity 0, 1)
  void* pd = nullptr;           // KParams<double>
  int cur = 0;
  int64_t steps = 0;
  KParams<double> Pd{};
  KParams<float> Pf{};
  int bx_shift = 8, gx = 1, nrowgroups = 1;
  uint32_t nblocks = 0;
};

namespace mrtlb {

static bool is_double(int storage) { return storage == kFP64; }
static size_t elem_bytes(int storage) {
  switch (storage) {
    case kFP64: return 8;
    case kFP32: case kFP32Dev: return 4;
    default: return 2;
  }
}
static int lattice_maxe(int kind) { return kind == kRD2Q25 ? 3 : 2; }

template <class Real>
static void fill_params(const mrtlb_solve& s, KParams<Real>& P) {
  const HostLattice& L = s.L;
  const int D = L.D;
  std::memset(&P, 0, sizeof P);
  P.nx = s.nx; P.ny = s.ny; P.nz = s.nz; P.N = s.N;
  P.inc = s.model.model == MRTLB_NSE_INC;
  P.m30 = s.model.m30 != 0;
  P.cs2 = (Real)L.cs2;
  for (int a = 0; a < 3; ++a) {
    const double c = a < D ? L.c[a] : 1.0;
    P.c1[a] = (Real)c; P.c2[a] = (Real)(c * c); P.c3[a] = (Real)(c * c * c);
  }
  P.cab[0] = (Real)(L.c[0] * L.c[1]);
  if (D == 3) { P.cab[1] = (Real)(L.c[0] * L.c[2]); P.cab[2] = (Real)(L.c[1] * L.c[2]); }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) P.cabb[a][b] = (Real)(L.c[a] * L.c[b] * L.c[b]);
  P.cxyz = D == 3 ? (Real)(L.c[0] * L.c[1] * L.c[2]) : (Real)0;
  const double scale = 128.0;
  for (int j = 0; j < L.B; ++j) {
    P.w[j] = (Real)L.w[j];
    P.wsc[j] = (Real)(L.w[j] / scale);
    P.iwsc[j] = (Real)(scale / L.w[j]);
  }
  for (int a = 0; a < D; ++a) {
    double ksum = 0;
    for (int b = 0; b < D; ++b) {
      P.corr[a][b] = (Real)L.corr[a][b];
      ksum += L.corr[a][b];
    }
    P.k3[a] = (Real)(-3 * L.cs2 + L.cs2 * ksum);
  }
  P.in0 = (Real)(1.0 / L.norms[0]);
  for (int a = 0; a < D; ++a) {
    P.in1[a] = (Real)(1.0 / L.norms[row_j(D, a)]);
    P.in2n[a] = (Real)(1.0 / L.norms[row_nn(D, a)]);
    P.in3p[a] = (Real)(1.0 / L.norms[row_aaa(D, a)]);
    for (int b = 0; b < D; ++b) {
      if (b != a) P.in3m[a][b] = (Real)(1.0 / L.norms[row_abb(D, a, b)]);
      if (b > a) P.in2o[off_index(a, b)] = (Real)(1.0 / L.norms[row_off(D, a, b)]);
    }
  }
  if (D == 3) P.inxyz = (Real)(1.0 / L.norms[row_xyz()]);
  const mrtlb_model_desc& m = s.model;
  P.s1 = (Real)m.s1; P.ss = (Real)m.s_shear; P.sb = (Real)m.s_bulk; P.s3 = (Real)m.s3; P.sh = (Real)m.s_high;
  const bool dev = s.storage == kFP32Dev || s.storage == kFP16Dev || s.storage == kBF16Dev;
  P.rho_ref = (Real)(dev && m.model != MRTLB_NCDE ? m.rho0 : 0.0);
  P.rho0 = (Real)m.rho0;
  if (m.model == MRTLB_NCDE) {
    const double K = L.cs2 * (1.0 / m.s1 - 0.5);
    P.phi_coef = (Real)(m.D0 / K);
    P.D2 = (Real)m.D2;
  }
  for (int a = 0; a < 3; ++a) P.adv[a] = (Real)(a < D ? m.adv_u[a] : 0.0);
}

template <class Real>
static Job<Real> make_job(const mrtlb_solve& s, int parity, const KParams<Real>& P) {
  Job<Real> J;
  std::memset(&J, 0, sizeof J);
  J.P = P;
  J.fin = s.f[parity];
  J.fout = s.f[parity ^ 1];
  J.force = static_cast<const Real*>(s.force);
  J.phi_prev = static_cast<const Real*>(s.phi[parity]);
  J.phi_out = static_cast<Real*>(s.phi[parity ^ 1]);
  J.block_begin = 0;
  J.nblocks = s.nblocks;
  J.gx = s.gx;
  J.bx_shift = s.bx_shift;
  J.nrowgroups = s.nrowgroups;
  return J;
}

// --- kernel dispatch -------------------------------------------------------

template <class F>
static bool with_lattice(int kind, F&& f) {
  switch (kind) {
    case kRD2Q25: f(LatRD2Q25{}); return true;
    case kRD2Q13: f(LatRD2Q13{}); return true;
    case kRD3Q53: f(LatRD3Q53{}); return true;
    case kRD3Q33: f(LatRD3Q33{}); return true;
  }
  return false;
}

template <class F>
static bool with_storage(int st, F&& f) {
  switch (st) {
    case kFP64: f(std::integral_constant<int, kFP64>{}); return true;
    case kFP32: f(std::integral_constant<int, kFP32>{}); return true;
    case kFP32Dev: f(std::integral_constant<int, kFP32Dev>{}); return true;
    case kFP16Dev: f(std::integral_constant<int, kFP16Dev>{}); return true;
    case kBF16Dev: f(std::integral_constant<int, kBF16Dev>{}); return true;
  }
  return false;
}

// NCDE kernels exist for the 2D lattices only (the paper's NCDE lattice is
// rD2Q13; rD2Q25 is accepted as well).
template <class L>
constexpr bool ncde_ok() { return L::D == 2; }

static hipError_t launch_step(int kind, int st, int model, bool force, const void* jobs, int njobs,
                              uint32_t total_blocks, hipStream_t stream) {
  hipError_t err = hipErrorInvalidValue;
  with_lattice(kind, [&](auto lat) {
    using L = decltype(lat);
    with_storage(st, [&](auto stc) {
      constexpr int ST = decltype(stc)::value;
      using Real = typename StoreT<ST>::Real;
      const auto* J = static_cast<const Job<Real>*>(jobs);
      if (model == MRTLB_NCDE) {
        if constexpr (ncde_ok<L>()) {
          hipLaunchKernelGGL((k_step<L, ST, kNcde, false>), dim3(total_blocks), dim3(kBlock), 0, stream, J, njobs,
                             total_blocks);
          err = hipGetLastError();
        }
      } else if (force) {
        hipLaunchKernelGGL((k_step<L, ST, kNseComp, true>), dim3(total_blocks), dim3(kBlock), 0, stream, J, njobs,
                           total_blocks);
        err = hipGetLastError();
      } else {
        hipLaunchKernelGGL((k_step<L, ST, kNseComp, false>), dim3(total_blocks), dim3(kBlock), 0, stream, J, njobs,
                           total_blocks);
        err = hipGetLastError();
      }
    });
  });
  return err;
}

}  // namespace mrtlb

// ===========================================================================
// C ABI
// ===========================================================================

// Entry points keep the C linkage of their declarations in mrtlb.h.

const char* mrtlb_last_error(void) { return g_last_error.c_str(); }

int mrtlb_version(void) { return (1 << 16) | 0; }

mrtlb_status mrtlb_ctx_create(int device, void* stream, size_t budget, mrtlb_ctx** out) {
  if (!out) return fail(MRTLB_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MRTLB_EINVAL, "device ordinal out of range");
  HIP_TRY(hipSetDevice(device));
  size_t freeb = 0, total = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &total));
  auto* c = new (std::nothrow) mrtlb_ctx;
  if (!c) return fail(MRTLB_ENOMEM, "host allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return fail(MRTLB_EDEVICE, "hipEventCreate failed");
  }
  *out = c;
  return MRTLB_OK;
}

void mrtlb_ctx_destroy(mrtlb_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

mrtlb_status mrtlb_ctx_memory(const mrtlb_ctx* c, size_t* used, size_t* budget) {
  if (!c) return fail(MRTLB_EINVAL, "ctx is NULL");
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  return MRTLB_OK;
}

mrtlb_status mrtlb_ctx_synchronize(mrtlb_ctx* c) {
  if (!c) return fail(MRTLB_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MRTLB_OK;
}

mrtlb_status mrtlb_lattice_create(const mrtlb_lattice_desc* desc, mrtlb_lattice** out) {
  if (!desc || !out) return fail(MRTLB_EINVAL, "NULL argument");
  *out = nullptr;
  auto* l = new (std::nothrow) mrtlb_lattice;
  if (!l) return fail(MRTLB_ENOMEM, "host allocation failed");
  std::string err;
  mrtlb_status st = build_lattice(*desc, &l->L, &err);
  if (st != MRTLB_OK) {
    delete l;
    return fail(st, err);
  }
  *out = l;
  return MRTLB_OK;
}

void mrtlb_lattice_destroy(mrtlb_lattice* l) { delete l; }

mrtlb_status mrtlb_lattice_query(const mrtlb_lattice* l, int* b, int* d, int* e, double* w, int* nlow, double* H,
                                 double* norms) {
  if (!l) return fail(MRTLB_EINVAL, "lattice is NULL");
  const HostLattice& L = l->L;
  if (b) *b = L.B;
  if (d) *d = L.D;
  if (nlow) *nlow = L.nlow;
  if (e) std::copy(L.e.begin(), L.e.end(), e);
  if (w) std::copy(L.w.begin(), L.w.end(), w);
  if (H) std::copy(L.H.begin(), L.H.end(), H);
  if (norms) std::copy(L.norms.begin(), L.norms.end(), norms);
  return MRTLB_OK;
}

static mrtlb_status check_model(const mrtlb_model_desc& m, int D, int kind) {
  if (m.model != MRTLB_NSE_INC && m.model != MRTLB_NSE_COMP && m.model != MRTLB_NCDE)
    return fail(MRTLB_EINVAL, "unknown model");
  const double r[6] = {m.s0, m.s1, m.s_shear, m.s_bulk, m.s3, m.s_high};
  for (double v : r)
    if (!(v > 0 && v < 2)) return fail(MRTLB_EINVAL, "relaxation rates must lie in (0, 2)");
  if (m.model == MRTLB_NSE_INC && !(m.rho0 > 0)) return fail(MRTLB_EINVAL, "rho0 must be positive");
  if (m.model == MRTLB_NCDE && D != 2) return fail(MRTLB_EINVAL, "the NCDE model is built for 2D lattices");
  (void)kind;
  return MRTLB_OK;
}

mrtlb_status mrtlb_solve_footprint(const mrtlb_lattice* lat, const int64_t n[3], int storage, int model,
                                   int has_force, size_t* bytes) {
  if (!lat || !n || !bytes) return fail(MRTLB_EINVAL, "NULL argument");
  if (storage < kFP64 || storage > kBF16Dev) return fail(MRTLB_EINVAL, "unknown storage");
  const int D = lat->L.D;
  const int64_t nz = D == 3 ? n[2] : 1;
  if (n[0] < 1 || n[1] < 1 || nz < 1) return fail(MRTLB_EINVAL, "grid sizes must be >= 1");
  const int64_t N = n[0] * n[1] * nz;
  const size_t real = is_double(storage) ? 8 : 4;
  size_t b = 2 * (size_t)lat->L.B * (size_t)N * elem_bytes(storage);
  if (has_force) b += (size_t)D * (size_t)N * real;
  if (model == MRTLB_NCDE) b += 2 * (size_t)N * real;
  b += 2 * sizeof(Job<double>) + sizeof(KParams<double>);
  *bytes = b;
  return MRTLB_OK;
}

static void release(mrtlb_solve* s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  for (void* p : {s->f[0], s->f[1], s->force, s->phi[0], s->phi[1], s->jobs, s->pd})
    if (p) (void)hipFree(p);
}

static mrtlb_status upload_jobs(mrtlb_solve* s) {
  if (is_double(s->storage)) {
    Job<double> j[2] = {make_job(*s, 0, s->Pd), make_job(*s, 1, s->Pd)};
    HIP_TRY(hipMemcpyAsync(s->jobs, j, sizeof j, hipMemcpyHostToDevice, s->ctx->stream));
    HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  } else {
    Job<float> j[2] = {make_job(*s, 0, s->Pf), make_job(*s, 1, s->Pf)};
    HIP_TRY(hipMemcpyAsync(s->jobs, j, sizeof j, hipMemcpyHostToDevice, s->ctx->stream));
    HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  }
  return MRTLB_OK;
}

mrtlb_status mrtlb_solve_create(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                const int64_t n[3], int storage, int has_force, mrtlb_solve** out) {
  if (!ctx || !lat || !model || !n || !out) return fail(MRTLB_EINVAL, "NULL argument");
  *out = nullptr;
  const int D = lat->L.D;
  mrtlb_status st = check_model(*model, D, lat->L.kind);
  if (st != MRTLB_OK) return st;
  if (has_force && model->model == MRTLB_NCDE) return fail(MRTLB_EINVAL, "the NCDE model takes no force field");
  size_t bytes = 0;
  st = mrtlb_solve_footprint(lat, n, storage, model->model, has_force, &bytes);
  if (st != MRTLB_OK) return st;
  const int64_t nz = D == 3 ? n[2] : 1;
  const int maxe = lattice_maxe(lat->L.kind);
  if (n[0] < maxe || n[1] < maxe || (D == 3 && nz < maxe))
    return fail(MRTLB_EINVAL, "every grid size must be at least the largest lattice offset");
  if (n[0] * n[1] * nz >= ((int64_t)1 << 31)) return fail(MRTLB_EINVAL, "node count must be below 2^31");
  if (n[0] > (1 << 24) || n[1] > (1 << 24)) return fail(MRTLB_EINVAL, "grid size too large");
  if (ctx->used + bytes > ctx->budget)
    return fail(MRTLB_ENOMEM, "footprint " + std::to_string(bytes) + " B exceeds the remaining HBM budget");
  auto* s = new (std::nothrow) mrtlb_solve;
  if (!s) return fail(MRTLB_ENOMEM, "host allocation failed");
  s->ctx = ctx;
  s->L = lat->L;
  s->model = *model;
  s->storage = storage;
  s->has_force = has_force ? 1 : 0;
  s->nx = (int)n[0]; s->ny = (int)n[1]; s->nz = (int)nz;
  s->N = (uint32_t)(n[0] * n[1] * nz);
  s->bytes = bytes;
  // tile: x-width 64/128/256, 256 threads per workgroup
  s->bx_shift = s->nx > 128 ? 8 : (s->nx > 64 ? 7 : 6);
  const int rows = kBlock >> s->bx_shift;
  s->gx = (s->nx + (1 << s->bx_shift) - 1) >> s->bx_shift;
  s->nrowgroups = ((s->ny + rows - 1) / rows) * s->nz;
  s->nblocks = (uint32_t)s->gx * (uint32_t)s->nrowgroups;
  (void)hipSetDevice(ctx->device);
  const size_t pop = (size_t)s->L.B * s->N * elem_bytes(storage);
  const size_t real = is_double(storage) ? 8 : 4;
  auto alloc = [&](void** p, size_t sz) { return hipMalloc(p, sz) == hipSuccess; };
  bool ok = alloc(&s->f[0], pop) && alloc(&s->f[1], pop) &&
            alloc(&s->jobs, 2 * std::max(sizeof(Job<double>), sizeof(Job<float>))) &&
            alloc(&s->pd, sizeof(KParams<double>));
  if (ok && has_force) ok = alloc(&s->force, (size_t)D * s->N * real);
  if (ok && model->model == MRTLB_NCDE) ok = alloc(&s->phi[0], s->N * real) && alloc(&s->phi[1], s->N * real);
  if (!ok) {
    release(s);
    delete s;
    (void)hipGetLastError();
    return fail(MRTLB_ENOMEM, "device allocation failed");
  }
  fill_params(*s, s->Pd);
  fill_params(*s, s->Pf);
  if (hipMemcpy(s->pd, &s->Pd, sizeof s->Pd, hipMemcpyHostToDevice) != hipSuccess || upload_jobs(s) != MRTLB_OK) {
    release(s);
    delete s;
    return fail(MRTLB_EDEVICE, "parameter upload failed");
  }
  ctx->used += bytes;
  *out = s;
  return MRTLB_OK;
}

void mrtlb_solve_destroy(mrtlb_solve* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->ctx->stream);
  release(s);
  s->ctx->used -= s->bytes;
  delete s;
}

int64_t mrtlb_solve_steps(const mrtlb_solve* s) { return s ? s->steps : -1; }

// Staging: device FP64 copies of host fields.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

mrtlb_status mrtlb_init_fields(mrtlb_solve* s, const double* rho, const double* u, const double* force) {
  if (!s || !rho) return fail(MRTLB_EINVAL, "NULL argument");
  const int D = s->L.D;
  const bool ncde = s->model.model == MRTLB_NCDE;
  if (!ncde && !u) return fail(MRTLB_EINVAL, "u is required for the NSE models");
  if ((force != nullptr) != (s->has_force != 0)) return fail(MRTLB_EINVAL, "force must be given iff the solve has a force field");
  for (uint32_t i = 0; i < s->N; ++i)
    if (!std::isfinite(rho[i])) return fail(MRTLB_ENUMERIC, "non-finite initial density/phi");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  DevBuf dr, du, df;
  HIP_TRY(hipMalloc(&dr.p, (size_t)s->N * 8));
  HIP_TRY(hipMemcpyAsync(dr.p, rho, (size_t)s->N * 8, hipMemcpyHostToDevice, st));
  if (!ncde) {
    HIP_TRY(hipMalloc(&du.p, (size_t)D * s->N * 8));
    HIP_TRY(hipMemcpyAsync(du.p, u, (size_t)D * s->N * 8, hipMemcpyHostToDevice, st));
  }
  if (force) {
    HIP_TRY(hipMalloc(&df.p, (size_t)D * s->N * 8));
    HIP_TRY(hipMemcpyAsync(df.p, force, (size_t)D * s->N * 8, hipMemcpyHostToDevice, st));
    // the stepping kernels read the force in the compute precision
    if (is_double(s->storage)) {
      HIP_TRY(hipMemcpyAsync(s->force, df.p, (size_t)D * s->N * 8, hipMemcpyDeviceToDevice, st));
    } else {
      std::vector<float> tmp((size_t)D * s->N);
      for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)force[i];
      HIP_TRY(hipMemcpyAsync(s->force, tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
  }
  s->cur = 0;
  s->steps = 0;
  // the init kernel writes f into buffer cur^1 and phi into both history
  // slots; run it with the parity-1 job so that fout = f[0]
  mrtlb_status rs = upload_jobs(s);
  if (rs != MRTLB_OK) return rs;
  const size_t jsz = is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  const void* job1 = static_cast<char*>(s->jobs) + jsz;
  hipError_t err = hipErrorInvalidValue;
  const int model = s->model.model;
  with_lattice(s->L.kind, [&](auto lat) {
    using L = decltype(lat);
    with_storage(s->storage, [&](auto stc) {
      constexpr int ST = decltype(stc)::value;
      using Real = typename StoreT<ST>::Real;
      const auto* J = static_cast<const Job<Real>*>(job1);
      const auto* PD = static_cast<const KParams<double>*>(s->pd);
      if (model == MRTLB_NCDE) {
        if constexpr (ncde_ok<L>()) {
          hipLaunchKernelGGL((k_init<L, ST, kNcde>), dim3(s->nblocks), dim3(kBlock), 0, st, J, PD,
                             (const double*)dr.p, (const double*)nullptr, (const double*)nullptr, s->nblocks);
          err = hipGetLastError();
        }
      } else {
        hipLaunchKernelGGL((k_init<L, ST, kNseComp>), dim3(s->nblocks), dim3(kBlock), 0, st, J, PD,
                           (const double*)dr.p, (const double*)du.p, (const double*)df.p, s->nblocks);
        err = hipGetLastError();
      }
    });
  });
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("init launch: ") + hipGetErrorString(err));
  HIP_TRY(hipStreamSynchronize(st));
  return MRTLB_OK;
}

mrtlb_status mrtlb_step(mrtlb_solve* s, int64_t nsteps) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (nsteps < 0) return fail(MRTLB_EINVAL, "nsteps must be >= 0");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const size_t jsz = is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  for (int64_t k = 0; k < nsteps; ++k) {
    const void* job = static_cast<char*>(s->jobs) + jsz * s->cur;
    hipError_t e = launch_step(s->L.kind, s->storage, s->model.model, s->has_force != 0, job, 1, s->nblocks,
                               s->ctx->stream);
    if (e != hipSuccess) return fail(MRTLB_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    s->cur ^= 1;
    s->steps += 1;
  }
  return MRTLB_OK;
}

mrtlb_status mrtlb_step_timed(mrtlb_solve* s, int64_t nsteps, double* ms) {
  if (!s || !ms) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipEventRecord(s->ctx->ev0, s->ctx->stream));
  mrtlb_status st = mrtlb_step(s, nsteps);
  if (st != MRTLB_OK) return st;
  HIP_TRY(hipEventRecord(s->ctx->ev1, s->ctx->stream));
  HIP_TRY(hipEventSynchronize(s->ctx->ev1));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, s->ctx->ev0, s->ctx->ev1));
  *ms = t;
  return MRTLB_OK;
}

template <class Real>
static mrtlb_status batch_group(mrtlb_solve* const* g, int n, int64_t nsteps, void* dev_jobs) {
  // jobs for both parities of every member, laid out [parity][member]
  std::vector<Job<Real>> jobs(2 * (size_t)n);
  uint32_t begin = 0;
  for (int i = 0; i < n; ++i) {
    const mrtlb_solve& s = *g[i];
    const KParams<Real>& P = *reinterpret_cast<const KParams<Real>*>(is_double(s.storage) ? (const void*)&s.Pd
                                                                                          : (const void*)&s.Pf);
    for (int par = 0; par < 2; ++par) {
      Job<Real> J = make_job(s, s.cur ^ par, P);
      J.block_begin = begin;
      jobs[(size_t)par * n + i] = J;
    }
    begin += s.nblocks;
  }
  hipStream_t st = g[0]->ctx->stream;
  HIP_TRY(hipMemcpyAsync(dev_jobs, jobs.data(), jobs.size() * sizeof(Job<Real>), hipMemcpyHostToDevice, st));
  for (int64_t k = 0; k < nsteps; ++k) {
    const void* jp = static_cast<const char*>(dev_jobs) + (size_t)(k & 1) * n * sizeof(Job<Real>);
    hipError_t e = launch_step(g[0]->L.kind, g[0]->storage, g[0]->model.model, g[0]->has_force != 0, jp, n, begin, st);
    if (e != hipSuccess) return fail(MRTLB_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
  }
  // the staging buffer must outlive the launches
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i) {
    g[i]->cur ^= (int)(nsteps & 1);
    g[i]->steps += nsteps;
  }
  return MRTLB_OK;
}

mrtlb_status mrtlb_batch_step(mrtlb_solve* const* solves, int n, int64_t nsteps) {
  if (!solves || n < 0 || nsteps < 0) return fail(MRTLB_EINVAL, "bad argument");
  if (n == 0 || nsteps == 0) return MRTLB_OK;
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return fail(MRTLB_EINVAL, "NULL solve in batch");
    if (solves[i]->ctx != solves[0]->ctx) return fail(MRTLB_EINVAL, "solves of a batch must share a context");
    for (int k = 0; k < i; ++k)
      if (solves[k] == solves[i]) return fail(MRTLB_EINVAL, "a solve appears twice in the batch");
  }
  HIP_TRY(hipSetDevice(solves[0]->ctx->device));
  // group by (lattice kind, storage, model, force); order of first appearance
  std::vector<int> done(n, 0);
  for (int i = 0; i < n; ++i) {
    if (done[i]) continue;
    std::vector<mrtlb_solve*> grp;
    const mrtlb_solve* a = solves[i];
    for (int k = i; k < n; ++k) {
      const mrtlb_solve* b = solves[k];
      if (!done[k] && b->L.kind == a->L.kind && b->storage == a->storage && b->model.model == a->model.model &&
          b->has_force == a->has_force && (b->model.model == MRTLB_NCDE) == (a->model.model == MRTLB_NCDE)) {
        grp.push_back(solves[k]);
        done[k] = 1;
      }
    }
    // one launch covers at most 2^31 workgroups; the job table lives in a
    // temporary device buffer
    const size_t jsz = is_double(a->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
    DevBuf jb;
    HIP_TRY(hipMalloc(&jb.p, 2 * grp.size() * jsz));
    mrtlb_status st = is_double(a->storage) ? batch_group<double>(grp.data(), (int)grp.size(), nsteps, jb.p)
                                            : batch_group<float>(grp.data(), (int)grp.size(), nsteps, jb.p);
    if (st != MRTLB_OK) return st;
  }
  return MRTLB_OK;
}

static mrtlb_status gather_launch(mrtlb_solve* s, int what, double* d0, double* d1) {
  const size_t jsz = is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  const void* job = static_cast<char*>(s->jobs) + jsz * s->cur;
  hipError_t err = hipErrorInvalidValue;
  const int model = s->model.model;
  hipStream_t st = s->ctx->stream;
  with_lattice(s->L.kind, [&](auto lat) {
    using L = decltype(lat);
    with_storage(s->storage, [&](auto stc) {
      constexpr int ST = decltype(stc)::value;
      using Real = typename StoreT<ST>::Real;
      const auto* J = static_cast<const Job<Real>*>(job);
      const auto* PD = static_cast<const KParams<double>*>(s->pd);
      if (what == 1) {
        hipLaunchKernelGGL((k_gather<L, ST, kNseComp, 1>), dim3(s->nblocks), dim3(kBlock), 0, st, J, PD, d0, d1);
      } else if (model == MRTLB_NCDE) {
        hipLaunchKernelGGL((k_gather<L, ST, kNcde, 0>), dim3(s->nblocks), dim3(kBlock), 0, st, J, PD, d0, d1);
      } else {
        hipLaunchKernelGGL((k_gather<L, ST, kNseComp, 0>), dim3(s->nblocks), dim3(kBlock), 0, st, J, PD, d0, d1);
      }
      err = hipGetLastError();
    });
  });
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("gather launch: ") + hipGetErrorString(err));
  return MRTLB_OK;
}

mrtlb_status mrtlb_read_moments(mrtlb_solve* s, double* rho, double* u) {
  if (!s || !rho) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int D = s->L.D;
  DevBuf dr, du;
  HIP_TRY(hipMalloc(&dr.p, (size_t)s->N * 8));
  if (u) HIP_TRY(hipMalloc(&du.p, (size_t)D * s->N * 8));
  mrtlb_status st = gather_launch(s, 0, (double*)dr.p, (double*)du.p);
  if (st != MRTLB_OK) return st;
  HIP_TRY(hipMemcpyAsync(rho, dr.p, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, du.p, (size_t)D * s->N * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  return MRTLB_OK;
}

mrtlb_status mrtlb_read_populations(mrtlb_solve* s, double* f) {
  if (!s || !f) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  DevBuf d;
  const size_t n = (size_t)s->L.B * s->N;
  HIP_TRY(hipMalloc(&d.p, n * 8));
  mrtlb_status st = gather_launch(s, 1, (double*)d.p, nullptr);
  if (st != MRTLB_OK) return st;
  HIP_TRY(hipMemcpyAsync(f, d.p, n * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  return MRTLB_OK;
}

mrtlb_status mrtlb_write_populations(mrtlb_solve* s, const double* f) {
  if (!s || !f) return fail(MRTLB_EINVAL, "NULL argument");
  const size_t n = (size_t)s->L.B * s->N;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) return fail(MRTLB_ENUMERIC, "non-finite population");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  DevBuf d;
  HIP_TRY(hipMalloc(&d.p, n * 8));
  HIP_TRY(hipMemcpyAsync(d.p, f, n * 8, hipMemcpyHostToDevice, st));
  // write into the current buffer: the parity-(cur^1) job has fout = f[cur]
  const size_t jsz = is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  const void* job = static_cast<char*>(s->jobs) + jsz * (s->cur ^ 1);
  hipError_t err = hipErrorInvalidValue;
  with_lattice(s->L.kind, [&](auto lat) {
    using L = decltype(lat);
    with_storage(s->storage, [&](auto stc) {
      constexpr int ST = decltype(stc)::value;
      using Real = typename StoreT<ST>::Real;
      hipLaunchKernelGGL((k_scatter<L, ST>), dim3(s->nblocks), dim3(kBlock), 0, st,
                         static_cast<const Job<Real>*>(job), static_cast<const KParams<double>*>(s->pd),
                         (const double*)d.p);
      err = hipGetLastError();
    });
  });
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("scatter launch: ") + hipGetErrorString(err));
  HIP_TRY(hipStreamSynchronize(st));
  return MRTLB_OK;
}

mrtlb_status mrtlb_conserved(mrtlb_solve* s, double* mass, double* momentum) {
  if (!s || !mass) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int B = s->L.B, D = s->L.D;
  const int nf = s->force ? D : 0;
  const int planes = B + nf;
  const uint32_t chunk = kBlock * kChunkIters;
  const uint32_t nchunks = (s->N + chunk - 1) / chunk;
  DevBuf part;
  HIP_TRY(hipMalloc(&part.p, (size_t)planes * nchunks * 8));
  hipStream_t st = s->ctx->stream;
  const size_t jsz = is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  const char* jobp = static_cast<const char*>(s->jobs) + jsz * s->cur;
  hipError_t err = hipErrorInvalidValue;
  with_storage(s->storage, [&](auto stc) {
    constexpr int ST = decltype(stc)::value;
    using Real = typename StoreT<ST>::Real;
    // KParams is the first member of the job in device memory
    const auto* PR = reinterpret_cast<const KParams<Real>*>(jobp);
    hipLaunchKernelGGL((k_plane_sums<ST>), dim3(nchunks, planes), dim3(kBlock), 0, st, s->f[s->cur], s->N, B,
                       static_cast<const Real*>(s->force), nf, PR, (double*)part.p, nchunks);
    err = hipGetLastError();
  });
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("sum launch: ") + hipGetErrorString(err));
  std::vector<double> h((size_t)planes * nchunks);
  HIP_TRY(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<double> plane(planes, 0.0);
  for (int p = 0; p < planes; ++p)
    for (uint32_t c = 0; c < nchunks; ++c) plane[p] += h[(size_t)p * nchunks + c];
  double m = 0, mom[3] = {0, 0, 0};
  const double ref = (s->storage == kFP32Dev || s->storage == kFP16Dev || s->storage == kBF16Dev) &&
                             s->model.model != MRTLB_NCDE
                         ? s->model.rho0
                         : 0.0;
  for (int j = 0; j < B; ++j) {
    m += plane[j];
    for (int a = 0; a < D; ++a) mom[a] += s->L.c[a] * s->L.e[j * D + a] * plane[j];
  }
  m += ref * (double)s->N;
  for (int a = 0; a < nf; ++a) mom[a] += 0.5 * plane[B + a];
  bool finite = std::isfinite(m);
  for (int a = 0; a < D; ++a) finite = finite && std::isfinite(mom[a]);
  *mass = m;
  if (momentum)
    for (int a = 0; a < D; ++a) momentum[a] = mom[a];
  if (!finite) return fail(MRTLB_ENUMERIC, "non-finite value in the solve's state");
  return MRTLB_OK;
}

