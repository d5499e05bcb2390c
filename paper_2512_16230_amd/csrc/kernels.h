// Device-side data structures shared by the kernels and the ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrtlb {

constexpr int kMaxB = 53;
constexpr int kBlock = 256;         // threads per workgroup of every node kernel
constexpr int kNumXcd = 8;          // MI355X: 8 XCDs, workgroups dealt round-robin

constexpr int kChunkIters = 16;      // elements per thread of one plane-sum chunk
constexpr double kI16Range = 2.0;    // default int16 range: |f - w rho_ref| <= 2 w

// Index of the off-diagonal pair (a, b), a < b: xy -> 0, xz -> 1, yz -> 2.
constexpr int off_index(int a, int b) { return a == 0 ? (b == 1 ? 0 : 1) : 2; }

// Slot table of a user-supplied lattice.  The step kernel holds the b
// populations in slots: first P.cnr rays (slots 4r .. 4r + 3: the pair of
// opposite velocities +-e, then the pair +-c e for an integer c >= 2), then
// P.cnp further pairs of opposite velocities (two slots each), then the
// velocities without an opposite (the rest velocity among them).  Per
// slot, kCSlot<D> reals: the weight w_j, the storage scales wsc_j and
// iwsc_j, the monomials of e_j that the moments of order <= 3 sum,
// numbered k = 1 .. kCMono<D> - 1 in the order e_a, e_a^2, e_a e_b (a < b),
// e_a^3, e_a e_b^2 (a != b), e_x e_y e_z (at index 2 + k), and c, c^2, c^3
// (the ray multiplier, set in the third slot of a ray); after the b rows of
// reals, b rows of kCInts 32-bit words: j, e_x, e_y, e_z, and the element
// offset of population j's source row from the own row's first element,
// ((-e_z ny - e_y) b + j) nxp modulo 2^32 (rows whose y and z neighbours
// need no wrap).  The forward transform adds monomial k times f_j to raw
// moment k; the back-transform evaluates sum_k monomial k times its
// coefficient.  A pair sums its even monomials (order 2) over f_a + f_b and
// its odd ones over f_a - f_b; a ray also folds its second pair into the
// first pair's monomials with the factors c, c^2, c^3 of orders 1, 2, 3.
template <int D>
constexpr int kCMono = D == 2 ? 10 : 20;
template <int D>
constexpr int kCSlot = kCMono<D> + 5;
constexpr int kCInts = 8;
constexpr bool cm_even(int D, int k) { return k >= 1 + D && k < 1 + 2 * D + D * (D - 1) / 2; }
// order of monomial k (1, 2 or 3)
constexpr int cm_order(int D, int k) { return k < 1 + D ? 1 : (cm_even(D, k) ? 2 : 3); }
constexpr int cm_1(int D, int a) { return 1 + a; }
constexpr int cm_2n(int D, int a) { return 1 + D + a; }
constexpr int cm_2o(int D, int a, int b) { return 1 + 2 * D + off_index(a, b); }
constexpr int cm_3p(int D, int a) { return 1 + 2 * D + D * (D - 1) / 2 + a; }
constexpr int cm_3m(int D, int a, int b) { return 1 + 3 * D + D * (D - 1) / 2 + a * (D - 1) + (b < a ? b : b - 1); }
constexpr int cm_xyz() { return 19; }

// kFP32DevF64: FP32 deviations in HBM, FP64 arithmetic in the kernels.
enum Storage { kFP64 = 0, kFP32 = 1, kFP32Dev = 2, kFP16Dev = 3, kBF16Dev = 4, kI16Dev = 5, kFP32DevF64 = 6 };
// kNseGrad: the NSE kernels with the gradient form of M2G_bar (lagged
// differences of the previous step's rho and rho u, stored per node).
enum ModelKind { kNseInc = 0, kNseComp = 1, kNcde = 2, kCde = 3, kNseGrad = 4 };

// Per-solve constants of the collision, in the compute precision.  Row
// constants refer to the component-form Hermite rows of order <= 3.
template <class Real>
struct KParams {
  int nx, ny, nz;
  int nxp;                  // population row pitch in elements (nx padded to 128 bytes)
  uint32_t N;               // nodes
  uint32_t pop_bytes;       // bytes of one population buffer (< 4 GiB)
  int inc;                  // NSE: incompressible (rho_m = rho0) or compressible (rho_m = rho)
  int m30;                  // NSE: third-order equilibrium moments rho uuu
  Real cs2;
  Real c1[3], c2[3], c3[3]; // c_a, c_a^2, c_a^3
  Real cab[3];              // c_x c_y, c_x c_z, c_y c_z
  Real cabb[3][3];          // c_a c_b^2
  Real cxyz;
  Real w[kMaxB];            // weights
  // 16-bit deviation storage.  A stored element s_j reads as the number
  // u_j (FP16/BF16: its value; int16: the integer) and means the deviation
  // f_j - w_j rho_ref = u_j * wsc[j]; it is written from an output number o_j
  // (FP16/BF16: o_j = u_j; int16: o_j = u_j / 32767 in [-1, 1]) with
  // o_j = (f_j - w_j rho_ref) * iwsc[j].  Opposite populations share wsc and
  // iwsc.  The step kernel's back-transform writes output numbers directly:
  // o_j = kin * kx * u_j + wo[j] * (...) with wo[j] = w_j * iwsc[j] and kin
  // = output numbers per read number (1, or 1/32767 for int16).  For the
  // other storages wsc = iwsc = kin = 1 and wo = w.
  Real wsc[kMaxB];
  Real iwsc[kMaxB];
  Real wo[kMaxB];
  Real kin;
  Real corr[3][3];          // correction coefficients of the pure third-order rows
  Real k3[3];               // -3 cs^2 + cs^2 sum_b corr[a][b]
  Real in0, in1[3], in2n[3], in2o[3], in3m[3][3], in3p[3], inxyz;  // 1 / norms
  Real s1, ss, sb, s3, sh;  // rates (s0 never acts: order-0 moment is conserved)
  // Standard lattices: the normal second-order block, I - S2 and I - S2/2
  // on the component rows c_a^2 - cs^2 (eq. 4-27); unused elsewhere.
  Real k2[3][3], g2[3][3];
  Real rho_ref;             // deviation reference: stored = f_bar - w rho_ref
  Real rho0;
  Real phi_coef, D2;        // NCDE: Phi = phi_coef (phi + D2 phi^3 / 3)
  Real adv[3];              // NCDE advection velocity
  Real gbt[3], gdd[3];      // general NCDE: A1 b_bar, diag(A2)
  // NCDE source S = sq + sk phi.  phi = (sum f + sqh) * sci; the zeroth
  // moment gains sa S(phi^n) + sp S(phi^{n-1}); the initial f_bar is
  // f_eq - sinit w S(phi0).  Full correction: sqh = sq/2, sci = 1/(1 - sk/2),
  // (sa, sp) = (1, 0), sinit = 1/2; three-level: sqh = 0, sci = 1,
  // (sa, sp) = (3/2, -1/2), sinit = 0.  No source: all terms vanish.
  Real sq, sk, sqh, sci, sa, sp, sinit;
  // NSE mass source S (forced kernel only): the uniform msrc, or per node
  // the plane d of the force buffer when sfield is set.  The zeroth moment
  // gains S, the second-order source gains -uu S.  NSE body force F and mass
  // source divided between G (share g, corrected with lambda2 and lambda1)
  // and F (eq. M-NSEs-2), h = 1 for the shifted f_bar and 0 for the
  // three-level scheme's unshifted f: rho = sum f + cS S with
  // cS = (g lambda1 + (1-g) h)/2, and rho u = sum c f + fh F with
  // fh = (g lambda2 + (1-g) h)/2 (eqs. 2-4-0, 2-4-2); the first moment gains
  // g1 F with g1 = 1 - s1 fh (NCDE: the factor 1 - s1/2 of M1G), plus
  // hf (F - F_prev) on the step after a force change (three-level scheme,
  // hf = (1-g)/2; the zeroth moment likewise hf (S - S_prev)); the normal
  // second-order rows gain kx2_a S with kx2_a = cs^2 (S2 I)_a (cS - 1/2),
  // the S20 share of M2G (eq. M-NSEs-4-0) and of the source distribution's
  // -cs^2 S_F I.
  Real msrc;
  int sfield;
  Real cS, fh, g1, hf;
  Real kx2[3];
  // velocity set at run time (read by the user-supplied-lattice kernels)
  int cb;                    // b
  int cmx, cmy, cmz;         // largest |e_x|, |e_y|, |e_z| over the set
  int cnr, cnp;              // rays and further pairs of opposite velocities (slot table)
  int8_t ce[kMaxB][3];       // integer velocity multiples e_j
  // MFMA transform (3D lattices, int16 storage): the forward product gives
  // the raw monomial sums as msig * (acc - mbias[P]) (see mfma.h)
  Real mbias[20];
  Real msig;
  // Drift correction: added to every node's zeroth and first Hermite moments
  // before the collision of one step (zero otherwise); the collision keeps
  // them, so the step moves the totals by N * dm0 and N * dm1.
  Real dm0, dm1[3];
};

// One solve's share of a (possibly batched) step launch.
template <class Real>
struct Job {
  KParams<Real> P;
  const void* fin;          // populations at t (post-collision, pre-propagation)
  void* fout;               // populations at t + 1
  const Real* force;        // d x N, or nullptr (CDE: the velocity field)
  const Real* fprev;        // NSE three-level: the force before the last change, else nullptr
  const Real* phi_prev;     // NCDE: phi^{n-1}; NSE gradient form: rho^{n-1} (rho_bar), then rho u^{n-1} (compressible)
  Real* phi_out;            // NCDE: phi^n; NSE gradient form: the same fields at step n
  int* sat;                 // int16 storage: set to 1 when a value saturates
  const void* mtab;         // MFMA transform: operand tables (16 KB); user-supplied lattice: the
                            // per-velocity table (b x kCMono<D> reals); or nullptr
  uint32_t block_begin;     // first linear workgroup of this job
  uint32_t nblocks;
  int vec;                  // nodes per thread along x
};

}  // namespace mrtlb
