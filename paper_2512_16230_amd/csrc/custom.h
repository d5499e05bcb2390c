// Kernels for a user-supplied velocity set (kind MRTLB_CUSTOM), included by
// custom_2d.hip and custom_3d.hip.  The structured kernels are compiled per
// velocity set; here the set is read at run time: the integer multiples e_j
// from KParams, and for the step a slot table of weights, scales,
// monomials and offsets (built by the ABI layer) through the constant
// address space.  The step holds the b gathered populations in
// registers (loops unrolled to a class of 16, 32 or 64 slots and guarded by
// the run-time b), so every population is read once and written once.  The
// moment-space part of the step (conserved variables, sources, equilibrium,
// relaxation) is the same code as for the compiled lattices; the NSE models
// only.  Measured alternatives on MI355X (rD2Q25's set, 4096^2, FP32
// deviations): a two-pass step that read every population again for the
// update, 10.2k MLUPS; the gathered values kept in LDS ([b][thread], 54 KB
// per workgroup, two workgroups per CU), 7.7k.
#pragma once

#include "device.h"

namespace mrtlb {

namespace {

// Element of f_bar_j at node (ix, iy, iz): the pull source x - e_j in the
// row-blocked layout (per grid row its b population rows of pitch nxp).
template <class Real>
__device__ __forceinline__ uint32_t csrc(const KParams<Real>& P, int j, int ix, int iy, int iz) {
  const uint32_t xs = (uint32_t)wrap(ix - (int)P.ce[j][0], P.nx);
  const uint32_t ys = (uint32_t)wrap(iy - (int)P.ce[j][1], P.ny);
  const uint32_t zs = (uint32_t)wrap(iz - (int)P.ce[j][2], P.nz);
  return ((zs * (uint32_t)P.ny + ys) * (uint32_t)P.cb + (uint32_t)j) * (uint32_t)P.nxp + xs;
}

// sum_r H_r delta_r / n_r at velocity e (lattice units), from the monomial
// coefficients of back_coeffs.
template <int D, class Real>
__device__ __forceinline__ Real poly_at(const BackCoeffs<Real>& C, const int (&e)[3]) {
  Real v = C.b0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const Real ea = (Real)e[a];
    v += ea * C.b1[a] + ea * ea * C.b2n[a] + ea * ea * ea * C.b3p[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      const Real eb = (Real)e[b];
      v += ea * eb * eb * C.b3m[a][b];
      if (b > a) v += ea * eb * C.b2o[off_index(a, b)];
    }
  }
  if constexpr (D == 3) v += (Real)(e[0] * e[1] * e[2]) * C.bxyz;
  return v;
}

template <class Real>
__device__ __forceinline__ void velocity(const KParams<Real>& P, int j, int (&e)[3]) {
  e[0] = P.ce[j][0];
  e[1] = P.ce[j][1];
  e[2] = P.ce[j][2];
}

}  // namespace

// One fused step, one node per thread over the padded rows, the b gathered
// populations held in register slots (BC >= b slots, loops unrolled to BC
// and guarded by the run-time counts).  The slot table (kernels.h: pairs
// of opposite velocities first, then the velocities without one; weights,
// scales, monomials, population indices and source-row offsets) is read
// through the constant address space: uniform scalar loads whose values
// enter the FMAs as scalar operands.  A pair sums its even monomials over
// f_a + f_b and its odd ones over f_a - f_b, and the back-transform
// evaluates the even and odd parts E, O once for both (E + O at e_a, E - O
// at e_b = -e_a); a ray of two pairs (+-e, +-c e) shares e's monomials,
// scaled by c, c^2, c^3 for orders 1, 2, 3.  When the row pitch is a multiple of 64 no wavefront
// crosses a grid row, so the source rows are computed once per wavefront
// on the scalar unit and the lane offset is x - e_x (wrapped per lane only
// in wavefronts that hold a periodic x-edge).
template <class Real>
using ConstReal = __attribute__((address_space(4))) const Real;
using ConstU32 = __attribute__((address_space(4))) const uint32_t;

template <int DIM, int ST, bool FORCE, int BC, bool RAYS>
__global__ __launch_bounds__(kBlock) void k_step_custom(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                       int njobs, uint32_t total_blocks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  using L = LatCustom<DIM>;
  constexpr int K = kCMono<DIM>;     // monomials k = 1 .. K - 1
  constexpr int KS = kCSlot<DIM>;
  constexpr int TB = (int)sizeof(T);
  const uint32_t lin = xcd_remap(blockIdx.x, total_blocks);
  const int jb = njobs > 1 ? find_job(jobs, njobs, lin) : 0;
  const Job<Real>& J = jobs[jb];
  const KParams<Real>& P = J.P;
  int ix, iy, iz;
  if (!tile_node<1>(J, lin - J.block_begin, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const int b = P.cb, nr = RAYS ? P.cnr : 0, np = P.cnp;
  const int pe = 4 * nr + 2 * np;    // first slot without an opposite
  const auto* tab = (const ConstReal<Real>*)J.mtab;
  const auto* tie = (const ConstU32*)((const char*)J.mtab + (size_t)b * KS * sizeof(Real));
  const uint32_t ny = (uint32_t)P.ny, nxp = (uint32_t)P.nxp, ub = (uint32_t)b;
  const bool interior = __all(ix >= P.cmx && ix + P.cmx < P.nx) != 0;

  // a1: gather (u: wave-uniform element offset in soffset, l: per lane).
  // MODE 0: rows vary within the wavefront, all per lane; 1: one row per
  // wavefront, y and z wrapped on the scalar unit; 2: one row per wavefront
  // and no y or z wrap needed, the source row at the table's offset from
  // the own row.
  T raw[BC];
  const uint32_t own = ((uint32_t)iz * ny + (uint32_t)iy) * ub * nxp;
  auto gather = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
    const auto rin = make_rsrc(J.fin, P.pop_bytes);
    const int wy = MODE > 0 ? __builtin_amdgcn_readfirstlane(iy) : iy;
    const int wz = MODE > 0 ? __builtin_amdgcn_readfirstlane(iz) : iz;
    const uint32_t wown = MODE > 0 ? (uint32_t)__builtin_amdgcn_readfirstlane(own) : own;
#pragma unroll
    for (int s = 0; s < BC; ++s) {
      if (s < b) {
        const auto* w = tie + s * kCInts;
        const int ex = (int)w[1];
        uint32_t xs = (uint32_t)(ix - ex);
        if (!interior) xs = (uint32_t)wrap(ix - ex, P.nx);
        uint32_t u, l;
        if constexpr (MODE == 2) {
          u = wown + w[4];
          l = xs;
        } else {
          const int ey = (int)w[2], ez = DIM == 3 ? (int)w[3] : 0;
          const uint32_t ys = (uint32_t)wrap(wy - ey, P.ny);
          const uint32_t zs = DIM == 3 ? (uint32_t)wrap(wz - ez, P.nz) : 0u;
          const uint32_t row = ((zs * ny + ys) * ub + w[0]) * nxp;
          u = MODE == 1 ? row : 0u;
          l = MODE == 1 ? xs : row + xs;
        }
        raw[s] = __builtin_bit_cast(T, buf_load<TB>(rin, l * (uint32_t)TB, u * (uint32_t)TB));
      } else {
        raw[s] = T(0);
      }
    }
  };
  const bool unirow = P.nxp % 64 == 0;
  if (unirow) {
    const int wy = __builtin_amdgcn_readfirstlane(iy), wz = __builtin_amdgcn_readfirstlane(iz);
    const bool yz_inside = wy >= P.cmy && wy + P.cmy < P.ny && (DIM == 2 || (wz >= P.cmz && wz + P.cmz < P.nz));
    if (yz_inside) gather(std::integral_constant<int, 2>{});
    else gather(std::integral_constant<int, 1>{});
  } else {
    gather(std::integral_constant<int, 0>{});
  }

  // the physical deviation held by slot s
  auto val = [&](int s) -> Real {
    if constexpr (scaled_storage<ST>()) return (Real)pin(units<ST>(raw[s]) * (float)tab[s * KS + 1]);
    else return (Real)raw[s];
  };

  // a3: raw moment sums, Rk[k] = sum_j monomial_k(e_j) f_j.  A ray
  // (slots 4r .. 4r + 3: +-e, then +-c e) adds to monomial k of e the sum
  // (f_a + f_b) of the first pair plus c^order times that of the second
  // (order 2), or the difference (f_a - f_b) likewise (orders 1 and 3).
  const Real z = Real(-0.0);
  Real R0 = z, Rk[K];
#pragma unroll
  for (int k = 1; k < K; ++k) Rk[k] = z;
#pragma unroll
  for (int r = 0; r < (RAYS ? BC / 4 : 0); ++r) {
    if (r < nr) {
      const int s0 = 4 * r;
      const Real fa = val(s0), fb = val(s0 + 1), ga = val(s0 + 2), gb = val(s0 + 3);
      const auto* c = tab + (s0 + 2) * KS + 2 + K;   // c, c^2, c^3
      const Real s1 = fa + fb, d1 = fa - fb, s2 = ga + gb, d2 = ga - gb;
      const Real S = s1 + c[1] * s2, D1 = d1 + c[0] * d2, D3 = d1 + c[2] * d2;
      const auto* m = tab + s0 * KS + 2;
      R0 += s1;
      R0 += s2;
#pragma unroll
      for (int k = 1; k < K; ++k) Rk[k] += m[k] * (cm_order(DIM, k) == 2 ? S : cm_order(DIM, k) == 1 ? D1 : D3);
    }
  }
#pragma unroll
  for (int s = 0; s < BC; s += 2) {
    if (s >= 4 * nr && s < pe) {
      const Real fa = val(s), fb = val(s + 1);
      const Real sm = fa + fb, df = fa - fb;
      const auto* m = tab + s * KS + 2;
      R0 += sm;
#pragma unroll
      for (int k = 1; k < K; ++k) Rk[k] += m[k] * (cm_even(DIM, k) ? sm : df);
    }
  }
#pragma unroll
  for (int s = 0; s < BC; ++s) {
    if (s >= pe && s < b) {
      const Real f = val(s);
      const auto* m = tab + s * KS + 2;
      R0 += f;
#pragma unroll
      for (int k = 1; k < K; ++k) Rk[k] += m[k] * f;
    }
  }
  Real R1[3] = {z, z, z}, R2n[3] = {z, z, z}, R2o[3] = {z, z, z}, R3p[3] = {z, z, z};
  Real R3m[3][3] = {{z, z, z}, {z, z, z}, {z, z, z}};
  Real Rxyz = z;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    R1[a] = Rk[cm_1(DIM, a)];
    R2n[a] = Rk[cm_2n(DIM, a)];
    R3p[a] = Rk[cm_3p(DIM, a)];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (c == a) continue;
      R3m[a][c] = Rk[cm_3m(DIM, a, c)];
      if (c > a) R2o[off_index(a, c)] = Rk[cm_2o(DIM, a, c)];
    }
  }
  if constexpr (DIM == 3) Rxyz = Rk[cm_xyz()];
  Moments<Real> M;
  finish_moments<DIM, false>(P, R0, R1, R2n, R2o, R3p, R3m, Rxyz, M);

  // a2, a4-a6
  Targets<Real> tg;
  relax_node<L, ST, kNseComp, FORCE>(M, J, g, ix, tg);

  // a7 + a8: f* = kx f + w (sum_r H_r delta_r / n_r), stored at the own node
  BackCoeffs<Real> C;
  back_coeffs<DIM, false>(P, tg.d0, tg.d1, tg.d2n, tg.d2o, tg.d3m, tg.d3p, tg.dxyz, C);
  Real cf[K];
  cf[0] = C.b0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    cf[cm_1(DIM, a)] = C.b1[a];
    cf[cm_2n(DIM, a)] = C.b2n[a];
    cf[cm_3p(DIM, a)] = C.b3p[a];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (c == a) continue;
      cf[cm_3m(DIM, a, c)] = C.b3m[a][c];
      if (c > a) cf[cm_2o(DIM, a, c)] = C.b2o[off_index(a, c)];
    }
  }
  if constexpr (DIM == 3) cf[cm_xyz()] = C.bxyz;
  const auto rout = make_rsrc(J.fout, P.pop_bytes);
  const uint32_t own_u = unirow ? (uint32_t)__builtin_amdgcn_readfirstlane(own) : 0u;
  const uint32_t own_l = unirow ? (uint32_t)ix : own + (uint32_t)ix;
  float smax = 0.0f;
  auto put = [&](int s, Real out) {
    T q;
    if constexpr (scaled_storage<ST>()) {
      const float o = pin((float)out * (float)tab[s * KS + 2]);
      if constexpr (ST == kI16Dev) smax = fmaxf(smax, fabsf(o));
      q = to_stored<ST>(o);
    } else {
      q = (T)out;
    }
    buf_store<TB>(rout, __builtin_bit_cast(typename RawChunk<TB>::T, q), own_l * (uint32_t)TB,
                  (own_u + tie[s * kCInts] * nxp) * (uint32_t)TB);
  };
#pragma unroll
  for (int r = 0; r < (RAYS ? BC / 4 : 0); ++r) {
    if (r < nr) {
      // the polynomial's order-2, order-1 and order-3 parts at e; at c e
      // they scale by c^2, c, c^3
      const int s0 = 4 * r;
      const auto* m = tab + s0 * KS + 2;
      const auto* c = tab + (s0 + 2) * KS + 2 + K;
      Real E2 = z, O1 = z, O3 = z;
#pragma unroll
      for (int k = 1; k < K; ++k) {
        if (cm_order(DIM, k) == 2) E2 += m[k] * cf[k];
        else if (cm_order(DIM, k) == 1) O1 += m[k] * cf[k];
        else O3 += m[k] * cf[k];
      }
      const Real E = cf[0] + E2, O = O1 + O3;
      put(s0, tg.kx * val(s0) + tab[s0 * KS] * (E + O));
      put(s0 + 1, tg.kx * val(s0 + 1) + tab[(s0 + 1) * KS] * (E - O));
      const Real Ec = cf[0] + c[1] * E2, Oc = c[0] * O1 + c[2] * O3;
      put(s0 + 2, tg.kx * val(s0 + 2) + tab[(s0 + 2) * KS] * (Ec + Oc));
      put(s0 + 3, tg.kx * val(s0 + 3) + tab[(s0 + 3) * KS] * (Ec - Oc));
    }
  }
#pragma unroll
  for (int s = 0; s < BC; s += 2) {
    if (s >= 4 * nr && s < pe) {
      const auto* m = tab + s * KS + 2;
      Real E = cf[0], O = z;
#pragma unroll
      for (int k = 1; k < K; ++k) {
        if (cm_even(DIM, k)) E += m[k] * cf[k];
        else O += m[k] * cf[k];
      }
      put(s, tg.kx * val(s) + tab[s * KS] * (E + O));
      put(s + 1, tg.kx * val(s + 1) + tab[(s + 1) * KS] * (E - O));
    }
  }
#pragma unroll
  for (int s = 0; s < BC; ++s) {
    if (s >= pe && s < b) {
      const auto* m = tab + s * KS + 2;
      Real poly = cf[0];
#pragma unroll
      for (int k = 1; k < K; ++k) poly += m[k] * cf[k];
      put(s, tg.kx * val(s) + tab[s * KS] * poly);
    }
  }
  raise_saturation<ST>(J, smax);
}

// f_bar(x, 0) = f_eq - F/2 in FP64, written at the pull source x - e_j.
template <int DIM, int ST>
__global__ __launch_bounds__(kBlock) void k_init_custom(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                       const KParams<double>* __restrict__ PD,
                                                       const double* __restrict__ rho, const double* __restrict__ uin,
                                                       const double* __restrict__ fin) {
  using Real = typename StoreT<ST>::Real;
  using L = LatCustom<DIM>;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  const double R = rho[self];
  double u[3] = {0, 0, 0}, jm[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  const double rho_m = P.inc ? P.rho0 : R;
  for (int a = 0; a < DIM; ++a) {
    u[a] = uin[(size_t)a * N + self];
    jm[a] = rho_m * u[a];
    if (fin) F[a] = fin[(size_t)a * N + self];
  }
  // mass source at this node (field or uniform) and its correction cS S
  const double msh = J.force ? P.cS * (P.sfield ? (double)J.force[(size_t)DIM * N + self] : P.msrc) : 0.0;
  Equilibrium<L, double, kNseComp> E;
  E.build(P, R, jm, u);
  double d1[3] = {0, 0, 0}, d2n[3] = {0, 0, 0}, d2o[3] = {0, 0, 0}, d3m[3][3] = {}, d3p[3] = {0, 0, 0}, dxyz = 0;
  for (int a = 0; a < DIM; ++a) {
    d1[a] = (E.e1[a] - P.fh * F[a]) * P.in1[a];
    // mass source: subtracting raw moments (cS S, ...) adds cs^2 cS S to the
    // Hermite second order
    d2n[a] = (E.e2n[a] + msh * P.cs2) * P.in2n[a];
    d3p[a] = E.e3p[a] * P.in3p[a];
    for (int c = 0; c < DIM; ++c)
      if (c != a) d3m[a][c] = E.e3m[a][c] * P.in3m[a][c];
    for (int c = a + 1; c < DIM; ++c) d2o[off_index(a, c)] = E.e2o[off_index(a, c)] * P.in2o[off_index(a, c)];
  }
  if constexpr (DIM == 3) dxyz = E.exyz * P.inxyz;
  const double d0 = (R - msh) * P.in0 - P.rho_ref;
  BackCoeffs<double> C;
  back_coeffs<DIM, false>(P, d0, d1, d2n, d2o, d3m, d3p, dxyz, C);
  const KParams<Real>& PR = J.P;
  float smax = 0.0f;
  for (int j = 0; j < P.cb; ++j) {
    int e[3];
    velocity(P, j, e);
    const double x = P.w[j] * poly_at<DIM>(C, e);
    smax = fmaxf(smax, sat_of<ST>((Real)x, PR, j));
    store_pop<ST>(J.fout, csrc(P, j, ix, iy, iz), (Real)x, PR, j);
  }
  raise_saturation<ST>(J, smax);
}

// Read-out: moments (WHAT 0) or populations (WHAT 1) in FP64.
template <int DIM, int ST, int WHAT>
__global__ __launch_bounds__(kBlock) void k_gather_custom(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                         const KParams<double>* __restrict__ PD,
                                                         double* __restrict__ out0, double* __restrict__ out1) {
  using L = LatCustom<DIM>;
  const auto& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  double R = 0, m1[3] = {0, 0, 0};
  for (int j = 0; j < P.cb; ++j) {
    const double v = (double)load_pop<ST>(J.fin, csrc(P, j, ix, iy, iz), J.P, j);
    if constexpr (WHAT == 1) {
      out0[(size_t)j * N + self] = v + P.w[j] * P.rho_ref;
    } else {
      R += v;
      for (int a = 0; a < DIM; ++a) m1[a] += (double)P.ce[j][a] * v;
    }
  }
  if constexpr (WHAT == 0) {
    R += P.rho_ref;
    if (J.force) R += P.cS * (P.sfield ? (double)J.force[(size_t)DIM * N + self] : P.msrc);
    out0[self] = R;
    if (out1) {
      const double rho_m = P.inc ? P.rho0 : R;
      for (int a = 0; a < DIM; ++a) {
        double jmom = P.c1[a] * m1[a];
        if (J.force) jmom += P.fh * (double)J.force[(size_t)a * N + self];
        out1[(size_t)a * N + self] = jmom / rho_m;
      }
    }
  }
}

// Restore populations (b x N, FP64, node order) into the pull layout.
template <int DIM, int ST>
__global__ __launch_bounds__(kBlock) void k_scatter_custom(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                          const KParams<double>* __restrict__ PD,
                                                          const double* __restrict__ in) {
  using Real = typename StoreT<ST>::Real;
  using L = LatCustom<DIM>;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  float smax = 0.0f;
  for (int j = 0; j < P.cb; ++j) {
    const double v = in[(size_t)j * P.N + self] - P.w[j] * P.rho_ref;
    smax = fmaxf(smax, sat_of<ST>((Real)v, J.P, j));
    store_pop<ST>(J.fout, csrc(P, j, ix, iy, iz), (Real)v, J.P, j);
  }
  raise_saturation<ST>(J, smax);
}

template <int DIM>
hipError_t launch_custom_dim(const LaunchReq& r) {
  hipError_t err = hipErrorInvalidValue;
  const dim3 grid(r.blocks), block(kBlock);
  if (r.model == kNcde || r.model == kCde) return err;   // the NSE models only
  with_storage(r.storage, [&](auto stc) {
    constexpr int ST = decltype(stc)::value;
    using Real = typename StoreT<ST>::Real;
    const auto* J = static_cast<const Job<Real>*>(r.jobs);
    const auto* PD = static_cast<const KParams<double>*>(r.pd);
    switch (r.op) {
      case kOpStep: {
        if (r.vec != 1) return;
        // register slots for the populations: the smallest class that holds b
        const uint32_t tb = r.xcd_order ? r.blocks : 0u;
        // the ray form is built for the unscaled storages (measured slower
        // for the 16-bit ones, whose conversions raise its register count)
        auto step = [&](auto bc) {
          constexpr int BC = decltype(bc)::value;
          auto go = [&](auto rays) {
            constexpr bool RAYS = decltype(rays)::value;
            if (r.force)
              hipLaunchKernelGGL((k_step_custom<DIM, ST, true, BC, RAYS>), grid, block, 0, r.stream, J, r.njobs, tb);
            else
              hipLaunchKernelGGL((k_step_custom<DIM, ST, false, BC, RAYS>), grid, block, 0, r.stream, J, r.njobs, tb);
          };
          if (!r.custom_rays) go(std::false_type{});
          else if constexpr (!scaled_storage<ST>()) go(std::true_type{});
        };
        if (r.custom_b <= 16) step(std::integral_constant<int, 16>{});
        else if (r.custom_b <= 32) step(std::integral_constant<int, 32>{});
        else step(std::integral_constant<int, 64>{});
        break;
      }
      case kOpInit:
        hipLaunchKernelGGL((k_init_custom<DIM, ST>), grid, block, 0, r.stream, J, PD, r.in0, r.in1, r.in2);
        break;
      case kOpMoments:
        hipLaunchKernelGGL((k_gather_custom<DIM, ST, 0>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        break;
      case kOpPopulations:
        hipLaunchKernelGGL((k_gather_custom<DIM, ST, 1>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        break;
      case kOpScatter:
        hipLaunchKernelGGL((k_scatter_custom<DIM, ST>), grid, block, 0, r.stream, J, PD, r.in0);
        break;
      default:
        return;
    }
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_custom_2d(const LaunchReq& r);
hipError_t launch_custom_3d(const LaunchReq& r);

}  // namespace mrtlb
