// C ABI of the Hermite-matrix MRT lattice Boltzmann library: contexts,
// lattices, solves, and the host side of every entry point.  Kernels live in
// device.h and are instantiated per lattice in inst_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <cstdint>
#include <vector>

#include "../../include/mrtlb.h"
#include "host_lattice.h"
#include "kernels.h"
#include "lattices.h"
#include "launch.h"
#include "mfma_layout.h"

namespace mrtlb {

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

// side streams of one context for overlapping lattice groups (the box runs
// 4 hardware queues per process: the context stream and 3 side streams)
constexpr int kSideStreams = 3;

struct mrtlb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t used = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // job tables of batched launches: a device buffer and its pinned host
  // staging copy, grown on demand and reused (no allocation per call)
  void* job_dev = nullptr;
  void* job_host = nullptr;
  size_t job_cap = 0;
  // device address of this GPU's scratch array (mrtlb_conserved_noalloc)
  void* scratch = nullptr;
  // side streams of mrtlb_batch_step (created on first use, default
  // priority): each runs one lattice group; events join them to `stream`
  hipStream_t side[kSideStreams] = {};
  hipEvent_t side_done[kSideStreams] = {};
  hipEvent_t staged = nullptr;
  int lds_per_cu = 0;           // LDS bytes of one compute unit (occupancy cap of the 2D steps)
  int lds_per_block = 0;        // largest LDS allocation of one workgroup
  int cus = 0;                  // compute units (occupancy cap: workgroups per resident round)
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
  int nxp = 1;                  // population row pitch (elements)
  uint32_t N = 0;
  size_t bytes = 0;
  void* f[2] = {nullptr, nullptr};
  void* force = nullptr;        // Real, (d + 1) x N: the NSE force, then the mass-source field (CDE: d x N velocity)
  void* fprev = nullptr;        // Real, d x N: the NSE three-level scheme's F(t - dt) (allocated on the
                                // first force change)
  bool hist_pending = false;    // the next step adds the three-level difference term (fprev valid)
  int sfield = 0;               // NSE: the mass source is the field in plane d of the force buffer
  void* phi[2] = {nullptr, nullptr};
  void* jobs = nullptr;         // three Job<Real> slots (parity 0, 1, drift-corrected step), then the
                                // int16 saturation flag (an int) at jobs + kFlagOffset
  void* pd = nullptr;           // KParams<double>
  int cur = 0;
  int64_t steps = 0;
  KParams<double> Pd{};
  KParams<float> Pf{};
  int vec = 1;
  bool xcd_order = true;        // step kernel tile order (pick_xcd_order)
  uint32_t nblocks = 0;         // workgroups of one step launch
  uint32_t nblocks_node = 0;    // workgroups of the one-thread-per-node kernels
  // drift correction: FP64 check every drift_every steps against the sums
  // recorded at the reference point; a pending correction rides on the next
  // step (job slot 2)
  int64_t drift_every = 0;
  int64_t since_check = 0;
  bool have_ref = false;
  double ref_mass = 0, ref_mom[3] = {0, 0, 0};
  bool pending = false;
  double dm0 = 0, dm1[3] = {0, 0, 0};
  void* part = nullptr;         // FP64 partial sums of the plane-sum kernel
  size_t part_bytes = 0;
  bool external = false;        // f[0], f[1] belong to the caller
  int transform = 0;            // Hermite transforms of the step: 0 VALU, 1 MFMA
  void* mtab = nullptr;         // MFMA operand tables (kMfmaTabBytes), or a user-supplied set's slot table
  bool crays = false;           // user-supplied set: the step's slot table holds rays (custom_rays)
  uint32_t step_lds = 0;        // LDS each step workgroup reserves (pick_step_lds)
};

// Whether a user-supplied set's step uses rays (defined with the slot
// table below).
static bool custom_rays(const HostLattice& L, int storage);

namespace mrtlb {

// FP64 arithmetic (KParams<double>, Job<double>, FP64 node fields).
static bool is_double(int storage) { return storage == kFP64 || storage == kFP32DevF64; }
// The job slots of a solve and, after them, its saturation flag.
constexpr size_t kFlagOffset = 3 * (sizeof(Job<double>) > sizeof(Job<float>) ? sizeof(Job<double>) : sizeof(Job<float>));
constexpr size_t kJobsBytes = kFlagOffset + 256;
static size_t elem_bytes(int storage) {
  switch (storage) {
    case kFP64: return 8;
    case kFP32: case kFP32Dev: case kFP32DevF64: return 4;
    default: return 2;
  }
}
// Largest |e_a| of the velocity set.
static int lattice_maxe(const HostLattice& L) {
  int m = 0;
  for (int v : L.e) m = std::max(m, v < 0 ? -v : v);
  return m;
}

// Population row pitch: nx rounded up to 32 nodes.  Rows start on a 32-element
// boundary and the step kernel's wavefronts cover whole 32-node runs of a row
// (128 B for FP32), so a wavefront access never straddles an extra cache line
// whatever nx is.
static int64_t row_pitch(int64_t nx, int storage) {
  (void)storage;
  return (nx + 31) / 32 * 32;
}

// Nodes per thread of the step kernel: two consecutive x-nodes on the 2D
// lattices when rows hold at least 512 nodes, i.e. 8-byte (FP32), 16-byte
// (FP64) or 4-byte (16-bit) vector accesses per population, and one node
// otherwise.  With one node per lane the periodic wrap is a per-lane index,
// so short rows (where every wavefront holds row-edge lanes) run no
// divergent gather; the 3D lattices (b = 33, 53) stay at one node, where two
// would double a register file that already limits occupancy.  Measured:
// rD2Q25 4096^2 two nodes match four (FP32) and beat it (FP16); rD3Q53 256^3
// one node beats two by 7%.  MRTLB_STEP_VEC (1, 2 or 4) overrides it for
// tuning runs.
static int pick_vec(int storage, int kind, int model, int nx) {
  // Measured on MI355X: one node per lane on the 3D lattices (register
  // pressure), for rows under 512 nodes and for the NCDE; otherwise 2 nodes
  // (FP32/FP64) or 4 nodes (16-bit storage, 8-byte accesses per lane).
  const bool small = storage == kFP16Dev || storage == kBF16Dev || storage == kI16Dev;
  int v = (kind == kRD3Q53 || kind == kRD3Q45 || kind == kRD3Q33 || kind == kD3Q27 || nx < 512 || model == MRTLB_NCDE ||
           model == MRTLB_CDE) ? 1
                                                                                            : (small ? 4 : 2);
  if (const char* e = std::getenv("MRTLB_STEP_VEC")) {
    const int o = std::atoi(e);
    if (o == 1 || o == 2 || o == 4) v = o;
  }
  // only the 2D NSE step kernels are built with several nodes per thread
  const bool is3d = kind == kRD3Q53 || kind == kRD3Q45 || kind == kRD3Q33 || kind == kD3Q27;
  if (is3d || kind == kCustom || model == MRTLB_NCDE || model == MRTLB_CDE) v = 1;
  while (v > 1 && (nx % v != 0 || nx < 4 * v)) v >>= 1;
  return v;
}

// Order of the step kernel's tiles over the chip.  Where a grid row holds
// several tiles, neighbouring tiles share the cache lines at their x-shifted
// edges, and contiguous tile ranges per XCD keep them in one L2.  Where one
// tile spans a whole row (the 3D grids), tiles share no lines, and the
// dispatch order, which deals consecutive tiles to the XCDs in turn, keeps
// the rows in flight in a narrow band.  Measured on MI355X: rD3Q53 256^3
// int16 +4% and D3Q27 +4% in dispatch order; rD2Q25 4096^2 FP32 +3% and the
// rD2Q13 NCDE batch +9% (FP32) in XCD ranges.  One 2D solve with 16-bit
// storage runs 1-3% faster in dispatch order (rD2Q25, rD2Q21, D2Q21K, D2Q9
// and the rD2Q13 CDE at 4096^2), while a batch of many solves with 16-bit
// storage keeps XCD ranges (the NCDE batch: +8% in int16), so `batched`
// selects the rule for a launch over several solves' job tables.
// MRTLB_XCD_ORDER (0 or 1) overrides it for tuning runs.
static bool pick_xcd_order(int64_t nxp, int vec, int dim, int storage, bool batched) {
  bool v = nxp > (int64_t)kBlock * vec;
  const bool narrow = storage == kFP16Dev || storage == kBF16Dev || storage == kI16Dev;
  if (dim == 2 && narrow && !batched) v = false;
  if (const char* e = std::getenv("MRTLB_XCD_ORDER")) {
    const int o = std::atoi(e);
    if (o == 0 || o == 1) v = o == 1;
  }
  return v;
}

// Occupancy cap of the step kernel.  The NSE steps with 32- and 64-bit
// storage run at the rate of their access pattern, b short streams per
// lane; with fewer workgroups resident per compute unit fewer streams
// compete for the DRAM banks and the pattern runs faster.  Measured on
// MI355X, 4096^2, three workgroups per CU against the eight the registers
// allow: streaming alone +4%, the rD2Q25 FP32 step +1.2%, rD2Q21 +1.9%,
// D2Q9 +3%, the gradient form of M2G +1.1%; two per CU pay further where a
// workgroup streams b >= 25 populations at two nodes per lane (rD2Q25 FP32
// +0.8%, FP64 +1.4% over three) and cost elsewhere (D2Q9 -4%, the
// one-node-per-lane gradient form -10%).  In 3D (256^3, against no cap)
// two per CU pay where a node stores at least 180 bytes (rD3Q53 FP32
// +2.3%, with a mass source +2.4%, rD3Q45 FP32 +1.9%, D3Q27 FP64 +5.1%) and
// three elsewhere (D3Q27 FP32 +1.8%; rD3Q33 FP32 level at 256^3 and +2.0%
// at 128^3, where two cost 5%); the gradient form takes three (two cost it
// 1.7%).  The 3D CDE steps follow the same rule (FP32 at 256^3: rD3Q53 +5%
// at two, rD3Q33 +3% and D3Q27 +2% at three).  The 2D NCDE and CDE steps
// (one node per lane) with 32- and 64-bit storage take four (the 256-solve
// NCDE batch +3.7%, the CDE at 4096^2 +1.5%; three cost the batch 7%, two
// cost the CDE 7%).  The cap is left off
// where the collision's share of the time needs the occupancy: the 16-bit
// storages (rD2Q25 int16 +0.6%, D2Q21K int16 -1.4%, rD3Q53 int16 -3%, the
// NCDE batch int16 -44% and the CDE int16 -37% at three) and the
// user-supplied lattices.  A capped step
// workgroup reserves a third or a half of the CU's LDS, which it does not
// use.  On smaller grids the cap leaves the chip part-empty in the last
// rounds of workgroups, so it applies only where the launch fills at least
// eight rounds of the capped residency (measured, cap against none: rD2Q25
// FP32 2048^2 +3.6% and 1024^2 +0.3%; D2Q9 FP32 1024^2, 2.7 rounds, -2%;
// rD3Q53 FP32 128^3 +1.0%, 96^3 -3%, 64^3 -5%; D3Q27 FP32 128^3 +2.6%, 96^3
// -1.6%, 64^3 -14%).  A batched launch decides on the workgroups of all its
// solves.  MRTLB_STEP_WG_PER_CU (0: no cap, 1-8) overrides it, at any size,
// for tuning runs.
static uint32_t pick_step_lds(int lds_per_cu, int lds_per_block, int cus, uint32_t nblocks, int dim, int kind,
                              int model, int storage, int b, int vec, bool m2g) {
  const bool nse = model == MRTLB_NSE_INC || model == MRTLB_NSE_COMP;
  const bool wide = storage == kFP32 || storage == kFP32Dev || storage == kFP64 || storage == kFP32DevF64;
  int wg = 0;
  if (kind != kCustom && wide) {
    if (dim == 3)
      wg = (size_t)b * elem_bytes(storage) >= 180 && !m2g ? 2 : 3;
    else
      wg = !nse ? 4 : b >= 25 && vec >= 2 ? 2 : 3;
  }
  if (wg > 0 && (uint64_t)nblocks < 8ull * (uint64_t)wg * (uint64_t)(cus > 0 ? cus : 0)) wg = 0;
  if (const char* e = std::getenv("MRTLB_STEP_WG_PER_CU")) {
    const int o = std::atoi(e);
    if (o >= 0 && o <= 8) wg = o;
  }
  if (wg <= 0 || lds_per_cu <= 0 || lds_per_block <= 0) return 0;
  // a multiple of 4 KiB, within one workgroup's limit, that lets wg
  // workgroups, not wg + 1, share the CU (else no cap)
  const uint32_t lds = (uint32_t)std::min(lds_per_cu / wg, lds_per_block) / 4096u * 4096u;
  return lds * (uint32_t)wg <= (uint32_t)lds_per_cu && lds * (uint32_t)(wg + 1) > (uint32_t)lds_per_cu ? lds : 0;
}

// S2 on the normal second-order component rows (FP64).  Standard lattices
// (k = 1), eqs. (4-27), (4-27-1): S2 = (diag(1/s_sa) + a b^T / d)^-1 with
// 1/s_sa = 1/2 + 2 nu / g_a, 1/s_ba = 1/2 + d nu_b / g_a, g_a = c_a^2 - cs^2,
// a_a = (1/s_ba - 1/s_sa) g_a, b_b = 1 / g_b, where nu = cs^2 (1/s_shear - 1/2)
// and nu_b = (2/d) cs^2 (1/s_bulk - 1/2) (eq. 4-29 with k = 1).  Multispeed
// lattices: s_bulk on the trace, s_shear on the deviator.  Returns false if
// the block is singular or not finite.
static bool s2_normal_block(const HostLattice& L, const mrtlb_model_desc& m, double S2[3][3]) {
  const int D = L.D;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S2[a][b] = 0;
  if (!L.standard) {
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) S2[a][b] = m.s_bulk / D + m.s_shear * ((a == b) - 1.0 / D);
    return true;
  }
  const double nu = L.cs2 * (1.0 / m.s_shear - 0.5);
  const double nu_b = (2.0 / D) * L.cs2 * (1.0 / m.s_bulk - 0.5);
  double A[3][6];
  for (int a = 0; a < D; ++a) {
    const double g = L.c[a] * L.c[a] - L.cs2;
    const double iss = 0.5 + 2 * nu / g, isb = 0.5 + D * nu_b / g;
    for (int b = 0; b < D; ++b) {
      const double gb = L.c[b] * L.c[b] - L.cs2;
      A[a][b] = (a == b ? iss : 0.0) + (isb - iss) * g / (gb * D);
      A[a][D + b] = a == b;
    }
  }
  // Gauss-Jordan with partial pivoting on [A | I]
  for (int col = 0; col < D; ++col) {
    int piv = col;
    for (int r = col + 1; r < D; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    if (!(std::fabs(A[piv][col]) > 1e-300)) return false;
    for (int k = 0; k < 2 * D; ++k) std::swap(A[col][k], A[piv][k]);
    const double inv = 1.0 / A[col][col];
    for (int k = 0; k < 2 * D; ++k) A[col][k] *= inv;
    for (int r = 0; r < D; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int k = 0; k < 2 * D; ++k) A[r][k] -= f * A[col][k];
    }
  }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      S2[a][b] = A[a][D + b];
      if (!std::isfinite(S2[a][b])) return false;
    }
  return true;
}

template <class Real>
static void fill_params(const mrtlb_solve& s, KParams<Real>& P) {
  const HostLattice& L = s.L;
  const int D = L.D;
  std::memset(&P, 0, sizeof P);
  P.nx = s.nx; P.ny = s.ny; P.nz = s.nz; P.N = s.N;
  P.nxp = s.nxp;
  P.pop_bytes = (uint32_t)((size_t)L.B * (size_t)s.ny * (size_t)s.nz * (size_t)s.nxp * elem_bytes(s.storage));
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
  // 16-bit deviation storage (see KParams): FP16/BF16 hold
  // (f - w rho_ref) * 128 / w; int16 holds (f - w rho_ref) / (A_j w) as a
  // signed 16-bit fraction, A_j from the caller's flow bounds, else the
  // uniform kI16Range.  Opposite populations share one scale.
  const mrtlb_model_desc& md = s.model;
  const bool bounded = md.u_bound > 0 || md.dev_bound > 0;
  std::vector<double> unit(L.B, 1.0), inv(L.B, 1.0);
  for (int j = 0; j < L.B; ++j) {
    if (s.storage == kFP16Dev || s.storage == kBF16Dev) {
      unit[j] = L.w[j] / 128.0;
      inv[j] = 128.0 / L.w[j];
    } else if (s.storage == kI16Dev) {
      double A = kI16Range;
      if (bounded) {
        double cn = 0;
        for (int a = 0; a < D; ++a) cn += L.c[a] * L.c[a] * L.e[j * D + a] * L.e[j * D + a];
        const double t = std::sqrt(cn) * md.u_bound / L.cs2;
        const double r = md.dev_bound;
        A = 2.0 * (r + (1.0 + r) * (std::expm1(t) + md.u_bound * md.u_bound / (2.0 * L.cs2)));
        if (md.model == MRTLB_NCDE) {
          // the diffusion term of the NCDE equilibrium: cs^2 (Phi - phi) I in
          // M2 adds (Phi - phi)(|c_j|^2 - d cs^2) / (2 cs^2) to f_eq,j / w_j,
          // with |Phi(phi) - phi| <= r max(|k - 1|, |k (1 + D2 r^2 / 3) - 1|)
          // for |phi| <= r, k = D0 / K, Phi = k (phi + D2 phi^3 / 3)
          const double k = md.D0 / (L.cs2 * (1.0 / md.s1 - 0.5));
          const double dphi = r * std::max(std::fabs(k - 1.0), std::fabs(k * (1.0 + md.D2 * r * r / 3.0) - 1.0));
          A += 2.0 * dphi * std::fabs(cn - D * L.cs2) / (2.0 * L.cs2);
        }
      }
      unit[j] = A * L.w[j] / 32767.0;
      inv[j] = 1.0 / (A * L.w[j]);
    }
  }
  for (int j = 0; j < L.B; ++j) {
    int q = j;
    for (int k = 0; k < L.B; ++k) {
      bool opp = true;
      for (int a = 0; a < D; ++a) opp = opp && L.e[k * D + a] == -L.e[j * D + a];
      if (opp) q = k;
    }
    const int src = q < j ? q : j;
    P.w[j] = (Real)L.w[j];
    P.wsc[j] = (Real)unit[src];
    P.iwsc[j] = (Real)inv[src];
    P.wo[j] = (Real)(s.storage == kFP16Dev || s.storage == kBF16Dev || s.storage == kI16Dev ? L.w[src] * inv[src]
                                                                                            : L.w[j]);
  }
  P.kin = (Real)(s.storage == kI16Dev ? 1.0 / 32767.0 : 1.0);
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
    P.in3p[a] = L.standard ? (Real)0 : (Real)(1.0 / L.norms[row_aaa(D, a)]);
    for (int b = 0; b < D; ++b) {
      if (b != a) P.in3m[a][b] = (Real)(1.0 / L.norms[row_abb(D, a, b)]);
      if (b > a) P.in2o[off_index(a, b)] = (Real)(1.0 / L.norms[row_off(D, a, b)]);
    }
  }
  if (D == 3) P.inxyz = (Real)(1.0 / L.norms[row_xyz()]);
  const mrtlb_model_desc& m = s.model;
  P.s1 = (Real)m.s1; P.ss = (Real)m.s_shear; P.sb = (Real)m.s_bulk; P.s3 = (Real)m.s3; P.sh = (Real)m.s_high;
  double S2[3][3];
  s2_normal_block(L, m, S2);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      P.k2[a][b] = (Real)((a == b) - S2[a][b]);
      P.g2[a][b] = (Real)((a == b) - 0.5 * S2[a][b]);
    }
  const bool dev = s.storage != kFP64 && s.storage != kFP32;
  P.rho_ref = (Real)(dev && m.model != MRTLB_NCDE && m.model != MRTLB_CDE ? m.rho0 : 0.0);
  P.rho0 = (Real)m.rho0;
  if (m.model == MRTLB_NCDE) {
    const double K = L.cs2 * (1.0 / m.s1 - 0.5);
    P.phi_coef = (Real)(m.D0 / K);
    P.D2 = (Real)m.D2;
  }
  if (m.model == MRTLB_NCDE) {
    const bool three = m.three_level != 0;
    P.sq = (Real)m.src_q;
    P.sk = (Real)m.src_k;
    P.sqh = (Real)(three ? 0.0 : 0.5 * m.src_q);
    P.sci = (Real)(three ? 1.0 : 1.0 / (1.0 - 0.5 * m.src_k));
    P.sa = (Real)(three ? 1.5 : 1.0);
    P.sp = (Real)(three ? -0.5 : 0.0);
    P.sinit = (Real)(three ? 0.0 : 0.5);
  } else {
    P.sci = (Real)1;
  }
  P.cb = L.B;
  P.cmx = P.cmy = P.cmz = 0;
  P.cnr = P.cnp = 0;
  if (L.kind == kCustom) {
    std::vector<int> mult;
    (void)velocity_slots(L, s.crays, &P.cnr, &P.cnp, &mult);
  }
  for (int j = 0; j < L.B; ++j) {
    for (int a = 0; a < 3; ++a) P.ce[j][a] = (int8_t)(a < D ? L.e[j * D + a] : 0);
    P.cmx = std::max(P.cmx, std::abs((int)P.ce[j][0]));
    P.cmy = std::max(P.cmy, std::abs((int)P.ce[j][1]));
    P.cmz = std::max(P.cmz, std::abs((int)P.ce[j][2]));
  }
  // NSE: force and mass source divided between G (share g) and F (eq.
  // M-NSEs-2); h = 1 for the shifted f_bar, 0 for the three-level scheme
  const bool nse = m.model == MRTLB_NSE_INC || m.model == MRTLB_NSE_COMP;
  const double gsh = nse ? m.g_share : 0.0, h = nse && m.three_level ? 0.0 : 1.0;
  const double cS = 0.5 * (gsh * m.lambda1 + (1 - gsh) * h);
  const double fh = nse ? 0.5 * (gsh * m.lambda2 + (1 - gsh) * h) : 0.5;
  P.msrc = (Real)(nse ? m.mass_src : 0.0);
  P.sfield = s.sfield;
  P.cS = (Real)cS;
  P.fh = (Real)fh;
  P.g1 = (Real)(1.0 - m.s1 * fh);
  P.hf = (Real)(nse && m.three_level ? 0.5 * (1 - gsh) : 0.0);
  for (int a = 0; a < 3; ++a) {
    double s2i = 0;                   // (S2 I)_a: row sum of the normal block
    for (int b = 0; b < D; ++b) s2i += S2[a][b];
    P.kx2[a] = (Real)(a < D ? L.cs2 * s2i * (cS - 0.5) : 0.0);
  }
  for (int a = 0; a < 3; ++a) {
    P.adv[a] = (Real)(a < D ? m.adv_u[a] : 0.0);
    const bool gn = m.model == MRTLB_NCDE && a < D;
    P.gbt[a] = (Real)(gn ? m.gn_bt[a] : 0.0);
    P.gdd[a] = (Real)(gn ? m.gn_dd[a] : 0.0);
  }
}

template <class Real>
static Job<Real> make_job(const mrtlb_solve& s, int parity, const KParams<Real>& P) {
  Job<Real> J;
  std::memset(&J, 0, sizeof J);
  J.P = P;
  J.fin = s.f[parity];
  J.fout = s.f[parity ^ 1];
  J.force = static_cast<const Real*>(s.force);
  J.fprev = nullptr;
  J.phi_prev = static_cast<const Real*>(s.phi[parity]);
  J.phi_out = static_cast<Real*>(s.phi[parity ^ 1]);
  J.sat = reinterpret_cast<int*>(static_cast<char*>(s.jobs) + kFlagOffset);
  J.mtab = s.mtab;
  J.block_begin = 0;
  J.nblocks = s.nblocks;
  J.vec = s.vec;
  return J;
}

// --- kernel dispatch -------------------------------------------------------

static hipError_t dispatch(int kind, const LaunchReq& r) {
  switch (kind) {
    case kRD2Q25: return launch_rd2q25(r);
    case kRD2Q13: return launch_rd2q13(r);
    case kRD3Q53: return launch_rd3q53(r);
    case kRD3Q33: return launch_rd3q33(r);
    case kRD2Q21: return launch_rd2q21(r);
    case kD2Q21K: return launch_d2q21k(r);
    case kRD3Q45: return launch_rd3q45(r);
    case kRD2Q17_1: return launch_rd2q17_1(r);
    case kRD2Q17_2: return launch_rd2q17_2(r);
    case kRD2Q17_3: return launch_rd2q17_3(r);
    case kRD2Q17_4: return launch_rd2q17_4(r);
    case kRD2Q17_5: return launch_rd2q17_5(r);
    case kD2Q9: return launch_d2q9(r);
    case kD3Q27: return launch_d3q27(r);
    case kCustom: return launch_custom(r);
  }
  return hipErrorInvalidValue;
}

static LaunchReq base_req(const mrtlb_solve& s, int op, const void* jobs) {
  LaunchReq r;
  r.op = op;
  r.storage = s.storage;
  r.model = s.model.model;
  r.force = s.has_force != 0;
  r.vec = s.vec;
  r.transform = s.transform;
  r.m2g = s.model.m2g_form == 1;
  r.xcd_order = s.xcd_order;
  r.dim = s.L.D;
  r.custom_b = s.L.kind == kCustom ? s.L.B : 0;
  r.custom_rays = s.crays;
  r.lds = (op == kOpStep || op == kOpStream) ? s.step_lds : 0u;
  r.jobs = jobs;
  r.njobs = 1;
  r.blocks = (op == kOpStep || op == kOpStream) ? s.nblocks : s.nblocks_node;
  r.stream = s.ctx->stream;
  r.pd = s.pd;
  return r;
}

static const void* job_ptr(const mrtlb_solve& s, int parity) {
  const size_t jsz = is_double(s.storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  return static_cast<const char*>(s.jobs) + jsz * parity;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (mrtlb_conserved_noalloc): a
// file-scope device array of kScratchBytes, one copy on every GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is a stand-in, not a
// device address): the device address comes from hipGetSymbolAddress, once
// per device with that device current, at context creation, and is kept per
// device.  Every call on a GPU shares its array; calls that overlap on one
// GPU (two threads, or contexts with different streams) race.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)4 << 20;
// planes of the state sums: b populations, d force components, the mass-source field
constexpr int kMaxPlanes = kMaxB + 4;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on `device` (which must be current).
static mrtlb_status scratch_setup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(MRTLB_EINVAL, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(MRTLB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return MRTLB_OK;
}

}  // namespace mrtlb

// ===========================================================================
// C ABI
// ===========================================================================

// Entry points keep the C linkage of their declarations in mrtlb.h.

const char* mrtlb_last_error(void) { return g_last_error.c_str(); }

int mrtlb_version(void) { return (1 << 16) | 0; }

mrtlb_status mrtlb_host_alloc(size_t bytes, void** out) {
  if (!out || bytes == 0) return fail(MRTLB_EINVAL, "NULL out or zero size");
  *out = nullptr;
  if (hipHostMalloc(out, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(MRTLB_ENOMEM, "page-locked host allocation failed");
  }
  return MRTLB_OK;
}

void mrtlb_host_free(void* p) {
  if (p) (void)hipHostFree(p);
}

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
  if (hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
          hipSuccess ||
      hipDeviceGetAttribute(&c->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    (void)hipGetLastError();
    c->lds_per_cu = c->lds_per_block = c->cus = 0;
  }
  {
    const mrtlb_status sst = scratch_setup(device, &c->scratch);
    if (sst != MRTLB_OK) {
      delete c;
      return sst;
    }
  }
  c->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
  // keep the stream-ordered allocator's freed staging memory for reuse
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  (void)hipGetLastError();
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
  (void)hipStreamSynchronize(c->stream);
  if (c->job_dev) (void)hipFree(c->job_dev);
  if (c->job_host) (void)hipHostFree(c->job_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (int i = 0; i < kSideStreams; ++i) {
    if (c->side[i]) (void)hipStreamSynchronize(c->side[i]);
    if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
    if (c->side_done[i]) (void)hipEventDestroy(c->side_done[i]);
  }
  if (c->staged) (void)hipEventDestroy(c->staged);
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

static mrtlb_status check_model(const mrtlb_model_desc& m, const HostLattice& L) {
  if (m.model != MRTLB_NSE_INC && m.model != MRTLB_NSE_COMP && m.model != MRTLB_NCDE && m.model != MRTLB_CDE)
    return fail(MRTLB_EINVAL, "unknown model");
  const double r[6] = {m.s0, m.s1, m.s_shear, m.s_bulk, m.s3, m.s_high};
  for (double v : r)
    if (!(v > 0 && v < 2)) return fail(MRTLB_EINVAL, "relaxation rates must lie in (0, 2)");
  if (m.model == MRTLB_NSE_INC && !(m.rho0 > 0)) return fail(MRTLB_EINVAL, "rho0 must be positive");
  if (!(m.u_bound >= 0 && m.u_bound < 1e3) || !(m.dev_bound >= 0 && m.dev_bound < 1e3))
    return fail(MRTLB_EINVAL, "u_bound and dev_bound must be finite and >= 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(m.gn_bt[a]) || !std::isfinite(m.gn_dd[a]))
      return fail(MRTLB_EINVAL, "gn_bt and gn_dd must be finite");
  if (!std::isfinite(m.src_q) || !std::isfinite(m.src_k) || !(std::fabs(m.src_k) < 1.0))
    return fail(MRTLB_EINVAL, "src_q must be finite and |src_k| < 1");
  const bool nse = m.model == MRTLB_NSE_INC || m.model == MRTLB_NSE_COMP;
  if ((m.src_q != 0 || m.src_k != 0) && m.model != MRTLB_NCDE)
    return fail(MRTLB_EINVAL, "the source q + k phi belongs to the NCDE model");
  if (m.three_level != 0 && m.model != MRTLB_NCDE && !nse)
    return fail(MRTLB_EINVAL, "the three-level scheme belongs to the NCDE and NSE models");
  if (!(m.g_share >= 0 && m.g_share <= 1) || !std::isfinite(m.lambda1) || !std::isfinite(m.lambda2))
    return fail(MRTLB_EINVAL, "g_share must lie in [0, 1] and lambda1, lambda2 must be finite");
  if (!nse && m.g_share != 0) return fail(MRTLB_EINVAL, "g_share belongs to the NSE models (0 otherwise)");
  if (!std::isfinite(m.mass_src)) return fail(MRTLB_EINVAL, "mass_src must be finite");
  if (m.mass_src != 0 && !nse) return fail(MRTLB_EINVAL, "the mass source belongs to the NSE models");
  if (m.m2g_form != 0 && m.m2g_form != 1) return fail(MRTLB_EINVAL, "m2g_form must be 0 or 1");
  if (m.m2g_form == 1 && !nse) return fail(MRTLB_EINVAL, "the gradient form of M2G belongs to the NSE models");
  if (m.m2g_form == 1 && L.kind == kCustom)
    return fail(MRTLB_EINVAL, "the gradient form of M2G runs on the compiled lattices");
  if (m.m2g_form == 1 && m.model == MRTLB_NSE_COMP && L.standard)
    return fail(MRTLB_EINVAL, "the compressible gradient form of M2G is built for the multispeed lattices (k = 0)");
  if (L.kind == kCustom && m.model != MRTLB_NSE_INC && m.model != MRTLB_NSE_COMP)
    return fail(MRTLB_EINVAL, "custom lattices carry the NSE models only");
  if (L.standard) {
    double S2[3][3];
    if (!s2_normal_block(L, m, S2)) return fail(MRTLB_EINVAL, "singular S2 block for these rates and this lattice");
  }
  return MRTLB_OK;
}

// User-supplied lattices: register class of the step kernel (b rounded up to
// 16, 32 or 64) and the per-velocity table (weight and monomials of each
// e_j, kCMono<D> reals per population, in the compute precision).
static int custom_class(const HostLattice& L) {
  return L.kind != kCustom ? 0 : L.B <= 16 ? 16 : L.B <= 32 ? 32 : 64;
}
static size_t custom_table_bytes(const HostLattice& L, int storage) {
  if (L.kind != kCustom) return 0;
  const size_t K = L.D == 3 ? kCSlot<3> : kCSlot<2>;
  return (size_t)L.B * (K * (is_double(storage) ? 8 : 4) + kCInts * 4);
}

// The step uses rays (measured on MI355X): for the unscaled storages, when
// the register class is at most 32 slots or rays hold at least half of the
// populations; in the 64-slot class a few rays do not pay for the registers
// the ray form takes (rD3Q33's set: 3 rays, 7% slower; rD3Q53's: 13 rays,
// 8% faster; rD2Q25's set +9%, the knight D2Q21's +12%), and the 16-bit
// storages are slower with them (int16: 11% on rD2Q25's set).
static bool custom_rays(const HostLattice& L, int storage) {
  if (L.kind != kCustom || storage == kFP16Dev || storage == kBF16Dev || storage == kI16Dev) return false;
  int nr = 0, np = 0;
  std::vector<int> mult;
  (void)velocity_slots(L, true, &nr, &np, &mult);
  return nr > 0 && (custom_class(L) <= 32 || 8 * nr >= L.B);
}

template <class Real>
static std::vector<char> custom_table(const HostLattice& L, bool rays, const KParams<Real>& P, int64_t ny,
                                      int64_t nxp) {
  const int D = L.D, K = D == 3 ? kCSlot<3> : kCSlot<2>;
  int nr = 0, np = 0;
  std::vector<int> mult;
  const std::vector<int> slot = velocity_slots(L, rays, &nr, &np, &mult);
  std::vector<Real> t((size_t)L.B * K, Real(0));
  std::vector<uint32_t> ie((size_t)L.B * kCInts, 0);
  for (int s = 0; s < L.B; ++s) {
    const int j = slot[s];
    uint32_t* w = ie.data() + (size_t)s * kCInts;
    w[0] = (uint32_t)j;
    for (int a = 0; a < D; ++a) w[1 + a] = (uint32_t)L.e[j * D + a];
    const int64_t ey = L.e[j * D + 1], ez = D == 3 ? L.e[j * D + 2] : 0;
    w[4] = (uint32_t)(((-ez * ny - ey) * L.B + j) * nxp);   // modulo 2^32
    double e[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) e[a] = L.e[j * D + a];
    Real* r = t.data() + (size_t)s * K;
    r[0] = (Real)L.w[j];
    r[1] = P.wsc[j];
    r[2] = P.iwsc[j];
    Real* m = r + 2;     // monomial k at m[k], k >= 1
    for (int a = 0; a < D; ++a) {
      m[cm_1(D, a)] = (Real)e[a];
      m[cm_2n(D, a)] = (Real)(e[a] * e[a]);
      m[cm_3p(D, a)] = (Real)(e[a] * e[a] * e[a]);
      for (int c = 0; c < D; ++c) {
        if (c == a) continue;
        m[cm_3m(D, a, c)] = (Real)(e[a] * e[c] * e[c]);
        if (c > a) m[cm_2o(D, a, c)] = (Real)(e[a] * e[c]);
      }
    }
    if (D == 3) m[cm_xyz()] = (Real)(e[0] * e[1] * e[2]);
    if (s < 4 * nr && s % 4 == 2) {      // the ray's multiplier c, c^2, c^3 after the monomials
      const double c = mult[s / 4];
      const int km = D == 3 ? kCMono<3> : kCMono<2>;
      m[km] = (Real)c;
      m[km + 1] = (Real)(c * c);
      m[km + 2] = (Real)(c * c * c);
    }
  }
  std::vector<char> out(t.size() * sizeof(Real) + ie.size() * sizeof(uint32_t));
  std::memcpy(out.data(), t.data(), t.size() * sizeof(Real));
  std::memcpy(out.data() + t.size() * sizeof(Real), ie.data(), ie.size() * sizeof(uint32_t));
  return out;
}

mrtlb_status mrtlb_solve_footprint(const mrtlb_lattice* lat, const int64_t n[3], int storage, int model,
                                   int has_force, size_t* bytes) {
  if (!lat || !n || !bytes) return fail(MRTLB_EINVAL, "NULL argument");
  if (storage < kFP64 || storage > kFP32DevF64) return fail(MRTLB_EINVAL, "unknown storage");
  const int D = lat->L.D;
  const int64_t nz = D == 3 ? n[2] : 1;
  if (n[0] < 1 || n[1] < 1 || nz < 1) return fail(MRTLB_EINVAL, "grid sizes must be >= 1");
  const int64_t N = n[0] * n[1] * nz;
  const size_t real = is_double(storage) ? 8 : 4;
  const int64_t rows = N / n[0];
  size_t b = 2 * (size_t)lat->L.B * (size_t)(rows * row_pitch(n[0], storage)) * elem_bytes(storage);
  const int kind = model & 0xff;
  if (has_force) b += (size_t)(D + 1) * (size_t)N * real;      // force, mass-source field
  if (kind == MRTLB_NCDE) b += 2 * (size_t)N * real;
  if (kind == MRTLB_CDE) b += (size_t)D * (size_t)N * real;    // velocity field
  if (model & MRTLB_FOOTPRINT_M2G_GRADIENT)                     // history of rho (and rho u), two slots
    b += 2 * (size_t)(kind == MRTLB_NSE_COMP ? D + 1 : 1) * (size_t)N * real;
  b += kJobsBytes + sizeof(KParams<double>);
  b += custom_table_bytes(lat->L, storage);
  *bytes = b;
  return MRTLB_OK;
}

static void release(mrtlb_solve* s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  if (!s->external)
    for (void* p : {s->f[0], s->f[1]})
      if (p) (void)hipFree(p);
  for (void* p : {s->force, s->fprev, s->phi[0], s->phi[1], s->jobs, s->pd, s->part, s->mtab})
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

static mrtlb_status create_solve(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                 const int64_t n[3], int storage, int has_force, void* ext0, void* ext1,
                                 mrtlb_solve** out) {
  if (!ctx || !lat || !model || !n || !out) return fail(MRTLB_EINVAL, "NULL argument");
  const bool external = ext0 != nullptr;
  *out = nullptr;
  const int D = lat->L.D;
  mrtlb_status st = check_model(*model, lat->L);
  if (st != MRTLB_OK) return st;
  if (has_force && (model->model == MRTLB_NCDE || model->model == MRTLB_CDE))
    return fail(MRTLB_EINVAL, "the NCDE and CDE models take no force field");
  if (model->mass_src != 0 && !has_force)
    return fail(MRTLB_EINVAL, "a mass source runs in the forced kernel: create the solve with has_force "
                              "(a zero force field is fine)");
  if (model->m2g_form == 1 && (storage == kFP16Dev || storage == kBF16Dev || storage == kI16Dev))
    return fail(MRTLB_EINVAL, "the gradient form of M2G runs with the FP32 and FP64 storages");
  size_t bytes = 0;
  st = mrtlb_solve_footprint(lat, n, storage, model->model | (model->m2g_form == 1 ? MRTLB_FOOTPRINT_M2G_GRADIENT : 0),
                             has_force, &bytes);
  if (st != MRTLB_OK) return st;
  const int64_t nz = D == 3 ? n[2] : 1;
  if (external)   // the population buffers are the caller's
    bytes -= 2 * (size_t)lat->L.B * (size_t)(n[1] * nz * row_pitch(n[0], storage)) * elem_bytes(storage);
  const int maxe = lattice_maxe(lat->L);
  if (n[0] < maxe || n[1] < maxe || (D == 3 && nz < maxe))
    return fail(MRTLB_EINVAL, "every grid size must be at least the largest lattice offset");
  if (n[0] * n[1] * nz >= ((int64_t)1 << 31)) return fail(MRTLB_EINVAL, "node count must be below 2^31");
  // kernels address a population buffer with 32-bit byte offsets
  if ((uint64_t)(n[1] * nz * row_pitch(n[0], storage)) * (uint64_t)lat->L.B * elem_bytes(storage) >=
      ((uint64_t)1 << 32))
    return fail(MRTLB_EINVAL, "one population buffer (b * N * element size) must be smaller than 4 GiB");
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
  s->nxp = (int)row_pitch(n[0], storage);
  s->bytes = bytes;
  // step kernel: each thread owns vec consecutive x-slots of the padded rows,
  // a workgroup kBlock * vec consecutive slots
  s->vec = pick_vec(storage, s->L.kind, s->model.model, s->nx);
  if (s->model.m2g_form == 1) s->vec = 1;     // the gradient-form kernels run one node per lane
  s->xcd_order = pick_xcd_order(s->nxp, s->vec, s->L.D, storage, false);
  s->crays = custom_rays(s->L, storage);
  const uint32_t slots = (uint32_t)s->ny * (uint32_t)s->nz * (uint32_t)s->nxp;
  s->nblocks = (slots + (uint32_t)(kBlock * s->vec) - 1) / (uint32_t)(kBlock * s->vec);
  s->step_lds = pick_step_lds(ctx->lds_per_cu, ctx->lds_per_block, ctx->cus, s->nblocks, s->L.D, s->L.kind,
                              s->model.model, storage, s->L.B, s->vec, s->model.m2g_form == 1);
  s->nblocks_node = (s->N + kBlock - 1) / kBlock;
  (void)hipSetDevice(ctx->device);
  const size_t pop = (size_t)s->L.B * (size_t)s->ny * s->nz * s->nxp * elem_bytes(storage);
  const size_t real = is_double(storage) ? 8 : 4;
  auto alloc = [&](void** p, size_t sz) { return hipMalloc(p, sz) == hipSuccess; };
  s->external = external;
  if (external) {
    s->f[0] = ext0;
    s->f[1] = ext1;
  }
  bool ok = (external || (alloc(&s->f[0], pop) && alloc(&s->f[1], pop))) &&
            alloc(&s->jobs, kJobsBytes) &&
            alloc(&s->pd, sizeof(KParams<double>));
  if (ok && has_force) {
    ok = alloc(&s->force, (size_t)(D + 1) * s->N * real);
    if (ok) ok = hipMemset(s->force, 0, (size_t)(D + 1) * s->N * real) == hipSuccess;
  }
  if (ok && model->model == MRTLB_NCDE) ok = alloc(&s->phi[0], s->N * real) && alloc(&s->phi[1], s->N * real);
  if (ok && model->m2g_form == 1) {
    const size_t hb = (size_t)(model->model == MRTLB_NSE_COMP ? D + 1 : 1) * s->N * real;
    ok = alloc(&s->phi[0], hb) && alloc(&s->phi[1], hb);
  }
  // the CDE's velocity field lives where the NSE force field would
  if (ok && model->model == MRTLB_CDE) ok = alloc(&s->force, (size_t)D * s->N * real);
  // a user-supplied lattice's slot table rides in the jobs' table slot
  if (ok && s->L.kind == kCustom) ok = alloc(&s->mtab, custom_table_bytes(s->L, storage));
  if (!ok) {
    release(s);
    delete s;
    (void)hipGetLastError();
    return fail(MRTLB_ENOMEM, "device allocation failed");
  }
  fill_params(*s, s->Pd);
  fill_params(*s, s->Pf);
  if (s->L.kind == kCustom) {
    const size_t tb = custom_table_bytes(s->L, storage);
    ok = (is_double(storage) ? hipMemcpy(s->mtab, custom_table(s->L, s->crays, s->Pd, s->ny, s->nxp).data(), tb,
                                         hipMemcpyHostToDevice)
                             : hipMemcpy(s->mtab, custom_table(s->L, s->crays, s->Pf, s->ny, s->nxp).data(), tb,
                                         hipMemcpyHostToDevice)) == hipSuccess;
  }
  if (!ok || hipMemcpy(s->pd, &s->Pd, sizeof s->Pd, hipMemcpyHostToDevice) != hipSuccess ||
      upload_jobs(s) != MRTLB_OK) {
    release(s);
    delete s;
    return fail(MRTLB_EDEVICE, "parameter upload failed");
  }
  ctx->used += bytes;
  *out = s;
  return MRTLB_OK;
}

mrtlb_status mrtlb_solve_create(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                const int64_t n[3], int storage, int has_force, mrtlb_solve** out) {
  return create_solve(ctx, lat, model, n, storage, has_force, nullptr, nullptr, out);
}

mrtlb_status mrtlb_population_bytes(const mrtlb_lattice* lat, const int64_t n[3], int storage, size_t* bytes) {
  if (!lat || !n || !bytes) return fail(MRTLB_EINVAL, "NULL argument");
  if (storage < kFP64 || storage > kFP32DevF64) return fail(MRTLB_EINVAL, "unknown storage");
  const int64_t nz = lat->L.D == 3 ? n[2] : 1;
  if (n[0] < 1 || n[1] < 1 || nz < 1) return fail(MRTLB_EINVAL, "grid sizes must be >= 1");
  *bytes = (size_t)lat->L.B * (size_t)(n[1] * nz * row_pitch(n[0], storage)) * elem_bytes(storage);
  return MRTLB_OK;
}

mrtlb_status mrtlb_solve_create_external(mrtlb_ctx* ctx, const mrtlb_lattice* lat, const mrtlb_model_desc* model,
                                         const int64_t n[3], int storage, int has_force, void* f0, void* f1,
                                         mrtlb_solve** out) {
  if (!f0 || !f1) return fail(MRTLB_EINVAL, "external population buffers must not be NULL");
  if (f0 == f1) return fail(MRTLB_EINVAL, "the two population buffers must differ");
  if (((uintptr_t)f0 | (uintptr_t)f1) % 16 != 0)
    return fail(MRTLB_EINVAL, "external population buffers must be 16-byte aligned");
  size_t pop = 0;
  const mrtlb_status st = mrtlb_population_bytes(lat, n, storage, &pop);
  if (st != MRTLB_OK) return st;
  const uintptr_t a = (uintptr_t)f0, b = (uintptr_t)f1;
  if ((a < b ? b - a : a - b) < pop) return fail(MRTLB_EINVAL, "the two population buffers overlap");
  if (!ctx) return fail(MRTLB_EINVAL, "NULL argument");
  for (void* p : {f0, f1}) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != ctx->device) {
      (void)hipGetLastError();
      return fail(MRTLB_EINVAL, "external population buffers must be device memory on the context's device");
    }
  }
  return create_solve(ctx, lat, model, n, storage, has_force, f0, f1, out);
}

void mrtlb_solve_destroy(mrtlb_solve* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->ctx->stream);
  release(s);
  s->ctx->used -= s->bytes;
  delete s;
}

int64_t mrtlb_solve_steps(const mrtlb_solve* s) { return s ? s->steps : -1; }

// Staging: device FP64 copies of host fields, from the stream-ordered
// allocator: allocation and release are ordered on the context stream and,
// unlike hipFree, do not wait for the whole device.
struct DevBuf {
  void* p = nullptr;
  hipStream_t st = nullptr;
  hipError_t alloc(size_t bytes, hipStream_t s) {
    st = s;
    return hipMallocAsync(&p, bytes, s);
  }
  ~DevBuf() { if (p) (void)hipFreeAsync(p, st); }
};

// int16 saturation flag: cleared when the state is (re)written from the
// host, raised by the kernels, read after the synchronous calls.
static mrtlb_status clear_saturation(mrtlb_solve* s) {
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(s->jobs) + kFlagOffset, &zero, sizeof zero, hipMemcpyHostToDevice,
                         s->ctx->stream));
  return MRTLB_OK;
}

// Call with the context stream synchronized.
static mrtlb_status check_saturation(mrtlb_solve* s) {
  if (s->storage != kI16Dev) return MRTLB_OK;
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, static_cast<char*>(s->jobs) + kFlagOffset, sizeof flag, hipMemcpyDeviceToHost));
  if (flag)
    return fail(MRTLB_ENUMERIC, "int16 storage saturated: a population left the fixed-point range set by "
                                "u_bound and dev_bound (raise them); the state is clamped");
  return MRTLB_OK;
}

// FP64 mass and momentum of the solve's current state: per-plane partial
// sums on the device (fixed order), then a fixed-order sum on the host.
// Planes of the FP64 sums of a solve's state (populations, then the force
// components) and the chunks each is summed in.
static void sum_layout(const mrtlb_solve* s, int* planes, uint32_t* nchunks) {
  const int nf = s->force && s->model.model != MRTLB_CDE ? s->L.D + s->sfield : 0;
  const uint32_t chunk = kBlock * kChunkIters;
  *planes = s->L.B + nf;
  *nchunks = (s->N + chunk - 1) / chunk;
}

// Device doubles plane_totals needs in its work buffer.
static size_t sum_work_doubles(const mrtlb_solve* s) {
  int planes;
  uint32_t nchunks;
  sum_layout(s, &planes, &nchunks);
  return (size_t)planes * nchunks + (size_t)planes;
}

// FP64 total of every plane into plane[] (host, kMaxPlanes entries): partial
// sums per chunk, then per plane in chunk order, both on the device, in
// `work` (sum_work_doubles entries of device memory); synchronizes.
static mrtlb_status plane_totals(mrtlb_solve* s, double* work, double* plane) {
  int planes;
  uint32_t nchunks;
  sum_layout(s, &planes, &nchunks);
  hipStream_t st = s->ctx->stream;
  // KParams is the first member of the job in device memory
  const void* params = job_ptr(*s, s->cur);
  hipError_t err = launch_plane_sums(s->storage, s->f[s->cur], s->N, s->L.B, s->force, planes - s->L.B, params, work,
                                     nchunks, st);
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("sum launch: ") + hipGetErrorString(err));
  double* totals = work + (size_t)planes * nchunks;
  err = launch_plane_totals(work, nchunks, planes, totals, st);
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("total launch: ") + hipGetErrorString(err));
  HIP_TRY(hipMemcpyAsync(plane, totals, (size_t)planes * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MRTLB_OK;
}

// Mass and momentum from the plane totals (fixed order), then the state checks.
static mrtlb_status totals_from_planes(mrtlb_solve* s, const double* plane, double* mass, double* momentum) {
  const int B = s->L.B, D = s->L.D;
  const int nf = s->force && s->model.model != MRTLB_CDE ? D : 0;
  double m = 0, mom[3] = {0, 0, 0};
  const double ref = s->storage != kFP64 && s->storage != kFP32 && s->model.model != MRTLB_NCDE &&
                             s->model.model != MRTLB_CDE
                         ? s->model.rho0
                         : 0.0;
  for (int j = 0; j < B; ++j) {
    m += plane[j];
    for (int a = 0; a < D; ++a) mom[a] += s->L.c[a] * s->L.e[j * D + a] * plane[j];
  }
  m += ref * (double)s->N;
  if (s->model.model == MRTLB_NCDE && s->model.three_level == 0 && (s->model.src_q != 0 || s->model.src_k != 0))
    m = (m + 0.5 * s->model.src_q * (double)s->N) / (1.0 - 0.5 * s->model.src_k);   // phi = sum f_bar + S/2
  // rho = sum f + cS S, rho u = sum c f + fh F
  if (s->model.model == MRTLB_NSE_INC || s->model.model == MRTLB_NSE_COMP)
    m += s->Pd.cS * (s->sfield ? plane[B + D] : s->Pd.msrc * (double)s->N);
  for (int a = 0; a < std::min(nf, D); ++a) mom[a] += s->Pd.fh * plane[B + a];
  bool finite = std::isfinite(m);
  for (int a = 0; a < D; ++a) finite = finite && std::isfinite(mom[a]);
  *mass = m;
  if (momentum)
    for (int a = 0; a < 3; ++a) momentum[a] = a < D ? mom[a] : 0.0;
  if (!finite) return fail(MRTLB_ENUMERIC, "non-finite value in the solve's state");
  return check_saturation(s);
}

// FP64 mass and momentum of the solve's current state, with the solve's own
// work buffer (grown on demand).
static mrtlb_status state_sums(mrtlb_solve* s, double* mass, double* momentum) {
  const size_t need = sum_work_doubles(s) * sizeof(double);
  if (need > s->part_bytes) {
    if (s->part) HIP_TRY(hipFree(s->part));
    s->part = nullptr;
    s->part_bytes = 0;
    HIP_TRY(hipMalloc(&s->part, need));
    s->part_bytes = need;
  }
  double plane[kMaxPlanes];
  mrtlb_status st = plane_totals(s, static_cast<double*>(s->part), plane);
  if (st != MRTLB_OK) return st;
  return totals_from_planes(s, plane, mass, momentum);
}

mrtlb_status mrtlb_conserved(mrtlb_solve* s, double* mass, double* momentum) {
  if (!s || !mass) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  double m = 0, mom[3] = {0, 0, 0};
  mrtlb_status st = state_sums(s, &m, mom);
  *mass = m;
  if (momentum)
    for (int a = 0; a < s->L.D; ++a) momentum[a] = mom[a];
  return st;
}

mrtlb_status mrtlb_conserved_noalloc(mrtlb_solve* s, double* mass, double* momentum) {
  if (!s || !mass) return fail(MRTLB_EINVAL, "NULL argument");
  const size_t need = sum_work_doubles(s);
  if (need > kScratchDoubles)
    return fail(MRTLB_EINVAL, "the solve's sums need " + std::to_string(need * sizeof(double)) +
                                  " B of scratch, more than the " + std::to_string(kScratchBytes) +
                                  " B of the allocation-free path; use mrtlb_conserved");
  HIP_TRY(hipSetDevice(s->ctx->device));
  if (!s->ctx->scratch) return fail(MRTLB_EDEVICE, "no scratch address for this device");
  double plane[kMaxPlanes];
  mrtlb_status st = plane_totals(s, static_cast<double*>(s->ctx->scratch), plane);
  if (st != MRTLB_OK) return st;
  double m = 0, mom[3] = {0, 0, 0};
  st = totals_from_planes(s, plane, &m, mom);
  *mass = m;
  if (momentum)
    for (int a = 0; a < s->L.D; ++a) momentum[a] = mom[a];
  return st;
}

// Momentum is a conserved total only for the NSE models without a force.
static bool corrects_momentum(const mrtlb_solve* s) { return s->model.model != MRTLB_NCDE && !s->has_force; }

static mrtlb_status record_reference(mrtlb_solve* s) {
  s->have_ref = false;
  s->pending = false;
  s->since_check = 0;
  if (s->drift_every <= 0) return MRTLB_OK;
  mrtlb_status st = state_sums(s, &s->ref_mass, s->ref_mom);
  if (st != MRTLB_OK) return st;
  s->have_ref = true;
  return MRTLB_OK;
}

// After drift_every steps: FP64 totals against the reference; the per-node
// difference is applied on the next step.
static mrtlb_status drift_check(mrtlb_solve* s) {
  s->since_check = 0;
  if (!s->have_ref) return record_reference(s);
  double m = 0, mom[3] = {0, 0, 0};
  mrtlb_status st = state_sums(s, &m, mom);
  if (st != MRTLB_OK) return st;
  const double n = (double)s->N;
  s->dm0 = (s->ref_mass - m) / n;
  for (int a = 0; a < 3; ++a) s->dm1[a] = corrects_momentum(s) && a < s->L.D ? (s->ref_mom[a] - mom[a]) / n : 0.0;
  s->pending = true;
  return MRTLB_OK;
}

template <class Real>
static KParams<Real> with_drift(const mrtlb_solve& s, KParams<Real> P) {
  if (s.pending) {
    P.dm0 = (Real)s.dm0;
    for (int a = 0; a < 3; ++a) P.dm1[a] = (Real)s.dm1[a];
  }
  return P;
}

mrtlb_status mrtlb_set_drift_correction(mrtlb_solve* s, int64_t every) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (every < 0) return fail(MRTLB_EINVAL, "every must be >= 0");
  if (every > 0 && s->model.model == MRTLB_CDE)
    return fail(MRTLB_EINVAL, "the CDE does not conserve its total (S_G = -u . grad phi)");
  if (every > 0 && s->model.model == MRTLB_NCDE && (s->model.src_q != 0 || s->model.src_k != 0))
    return fail(MRTLB_EINVAL, "an NCDE with a source does not conserve its total");
  if (every > 0 && s->model.mass_src != 0) return fail(MRTLB_EINVAL, "a mass source does not conserve the mass");
  HIP_TRY(hipSetDevice(s->ctx->device));
  s->drift_every = every;
  return record_reference(s);
}

// --- MFMA transform ---------------------------------------------------------

static uint16_t host_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float host_bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
static uint16_t host_f16_bits(_Float16 v) {
  uint16_t b;
  std::memcpy(&b, &v, 2);
  return b;
}

// Operand tables of the MFMA transform (layout in mfma_layout.h) from the
// solve's storage scales wsc_j and output weights wo_j: forward
// E[P][j] = e_j^P wsc_j / sigma as f16 hi + lo with |E| <= 16384, the
// per-row constant 99328 sum_j E[P][j] that the shifted chunks of the int16
// numbers add (q = f_lo + 2 f_hi - 99328), and backward e_j^P wo_j as bf16
// hi + lo.
static void build_mfma_tables(mrtlb_solve& s, std::vector<uint32_t>& words) {
  const HostLattice& L = s.L;
  const int B = L.B;
  KParams<float>& P = s.Pf;
  double wmax = 0;
  for (int j = 0; j < B; ++j) wmax = std::max(wmax, (double)P.wsc[j]);
  const double sigma = wmax * 8.0 / 16384.0;
  std::vector<_Float16> eh(kMono * 64, (_Float16)0.0f), el(kMono * 64, (_Float16)0.0f);
  for (int p = 0; p < kMono; ++p) {
    double bias = 0;
    for (int j = 0; j < B; ++j) {
      const int* e = &L.e[j * 3];
      const double v = mono(p, e[0], e[1], e[2]) * (double)P.wsc[j] / sigma;
      const _Float16 hi = (_Float16)v;
      const _Float16 lo = (_Float16)(v - (double)hi);
      eh[p * 64 + j] = hi;
      el[p * 64 + j] = lo;
      bias += (double)hi + (double)lo;
    }
    P.mbias[p] = (float)(99328.0 * bias);
  }
  P.msig = (float)sigma;
  words.assign((size_t)kMfmaTabVec * 4, 0u);
  for (int part = 0; part < 2; ++part)
    for (int k = 0; k < 4; ++k)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 8; ++t) {
          const int row = lane % 32, K = 16 * k + 8 * (lane / 32) + t;
          uint16_t bits = 0;
          if (row < kMono && K < B) bits = host_f16_bits(part == 0 ? eh[row * 64 + K] : el[row * 64 + K]);
          words[((size_t)((part * 4 + k) * 64 + lane)) * 4 + t / 2] |= (uint32_t)bits << (16 * (t % 2));
        }
  for (int part = 0; part < 2; ++part)
    for (int m = 0; m < 2; ++m)
      for (int k = 0; k < 2; ++k)
        for (int lane = 0; lane < 64; ++lane)
          for (int t = 0; t < 8; ++t) {
            const int j = 32 * m + lane % 32, K = 16 * k + 8 * (lane / 32) + t;
            uint16_t bits = 0;
            if (j < B && K < kMono) {
              const int* e = &L.e[j * 3];
              const float v = (float)(mono(K, e[0], e[1], e[2]) * (double)P.wo[j]);
              const uint16_t hi = host_bf16_rne(v);
              bits = part == 0 ? hi : host_bf16_rne(v - host_bf16_value(hi));
            }
            words[((size_t)kMfmaFwdVec + (size_t)(((part * 2 + m) * 2 + k) * 64 + lane)) * 4 + t / 2] |=
                (uint32_t)bits << (16 * (t % 2));
          }
}

mrtlb_status mrtlb_solve_set_transform(mrtlb_solve* s, int transform) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (transform != MRTLB_TRANSFORM_VALU && transform != MRTLB_TRANSFORM_MFMA)
    return fail(MRTLB_EINVAL, "unknown transform");
  HIP_TRY(hipSetDevice(s->ctx->device));
  if (transform == MRTLB_TRANSFORM_MFMA) {
    int maxe = 0;
    for (int v : s->L.e) maxe = std::max(maxe, v < 0 ? -v : v);
    if (s->L.D != 3 || s->L.kind == kCustom || maxe > 2 || s->L.B > 64)
      return fail(MRTLB_EINVAL, "the MFMA transform is built for the 3D lattices (rD3Q53, rD3Q45, rD3Q33, D3Q27)");
    if (s->storage != kI16Dev) return fail(MRTLB_EINVAL, "the MFMA transform runs with the int16 deviation storage");
    if ((s->model.model != MRTLB_NSE_INC && s->model.model != MRTLB_NSE_COMP) || s->has_force ||
        s->model.m2g_form != 0)
      return fail(MRTLB_EINVAL, "the MFMA transform runs the NSE models without a force field (closed-form M2G)");
    if (s->nxp % 64 != 0)
      return fail(MRTLB_EINVAL, "the MFMA transform needs a row pitch (nx rounded up to 32) that is a multiple of 64");
    if (!s->mtab) {
      if (s->ctx->used + (size_t)kMfmaTabBytes > s->ctx->budget)
        return fail(MRTLB_ENOMEM, "the MFMA tables exceed the remaining HBM budget");
      if (hipMalloc(&s->mtab, kMfmaTabBytes) != hipSuccess) {
        (void)hipGetLastError();
        s->mtab = nullptr;
        return fail(MRTLB_ENOMEM, "device allocation failed");
      }
      s->ctx->used += kMfmaTabBytes;
      s->bytes += kMfmaTabBytes;
    }
    std::vector<uint32_t> words;
    build_mfma_tables(*s, words);
    HIP_TRY(hipMemcpyAsync(s->mtab, words.data(), kMfmaTabBytes, hipMemcpyHostToDevice, s->ctx->stream));
    HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  }
  s->transform = transform;
  return upload_jobs(s);
}

// The CDE's velocity field (d x N, FP64 on the host) into the solve's
// device field, in the compute precision; synchronous.
// A d x N node field (the NSE force, the CDE velocity) into the solve's
// field buffer, in the compute precision of the stepping kernels.
static mrtlb_status upload_node_field(mrtlb_solve* s, const double* v, const char* what) {
  const int D = s->L.D;
  for (size_t i = 0; i < (size_t)D * s->N; ++i)
    if (!std::isfinite(v[i])) return fail(MRTLB_ENUMERIC, std::string("non-finite ") + what);
  hipStream_t st = s->ctx->stream;
  if (is_double(s->storage)) {
    HIP_TRY(hipMemcpyAsync(s->force, v, (size_t)D * s->N * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  } else {
    std::vector<float> tmp((size_t)D * s->N);
    for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)v[i];
    HIP_TRY(hipMemcpyAsync(s->force, tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return MRTLB_OK;
}

static mrtlb_status upload_velocity(mrtlb_solve* s, const double* u) {
  return upload_node_field(s, u, "velocity field");
}

// The three-level scheme's F(t - dt) and S(t - dt): the force and mass
// source of the last step, kept until the next step has used them.
static mrtlb_status keep_source_history(mrtlb_solve* s, bool* history) {
  *history = s->model.three_level != 0 && s->model.g_share < 1.0 && s->steps > 0;
  if (!*history || s->hist_pending) return MRTLB_OK;
  const size_t bytes = (size_t)(s->L.D + 1) * s->N * (is_double(s->storage) ? 8 : 4);
  if (!s->fprev && hipMalloc(&s->fprev, bytes) != hipSuccess) {
    s->fprev = nullptr;
    return fail(MRTLB_ENOMEM, "out of device memory for the previous force field");
  }
  HIP_TRY(hipMemcpyAsync(s->fprev, s->force, bytes, hipMemcpyDeviceToDevice, s->ctx->stream));
  return MRTLB_OK;
}

static bool nse_with_force(const mrtlb_solve* s) {
  return (s->model.model == MRTLB_NSE_INC || s->model.model == MRTLB_NSE_COMP) && s->has_force;
}

mrtlb_status mrtlb_set_force_field(mrtlb_solve* s, const double* force) {
  if (!s || !force) return fail(MRTLB_EINVAL, "NULL argument");
  if (!nse_with_force(s)) return fail(MRTLB_EINVAL, "the force field belongs to an NSE solve created with has_force");
  HIP_TRY(hipSetDevice(s->ctx->device));
  bool history = false;
  mrtlb_status st = keep_source_history(s, &history);
  if (st != MRTLB_OK) return st;
  st = upload_node_field(s, force, "force field");
  if (st != MRTLB_OK) return st;
  if (history) s->hist_pending = true;
  return MRTLB_OK;
}

mrtlb_status mrtlb_set_mass_source_field(mrtlb_solve* s, const double* S) {
  if (!s || !S) return fail(MRTLB_EINVAL, "NULL argument");
  if (!nse_with_force(s)) return fail(MRTLB_EINVAL, "the mass source belongs to an NSE solve created with has_force");
  for (uint32_t i = 0; i < s->N; ++i)
    if (!std::isfinite(S[i])) return fail(MRTLB_ENUMERIC, "non-finite mass source");
  HIP_TRY(hipSetDevice(s->ctx->device));
  bool history = false;
  mrtlb_status st = keep_source_history(s, &history);
  if (st != MRTLB_OK) return st;
  hipStream_t stream = s->ctx->stream;
  char* plane = static_cast<char*>(s->force) + (size_t)s->L.D * s->N * (is_double(s->storage) ? 8 : 4);
  if (is_double(s->storage)) {
    HIP_TRY(hipMemcpyAsync(plane, S, (size_t)s->N * 8, hipMemcpyHostToDevice, stream));
  } else {
    std::vector<float> tmp(s->N);
    for (uint32_t i = 0; i < s->N; ++i) tmp[i] = (float)S[i];
    HIP_TRY(hipMemcpyAsync(plane, tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  if (!s->sfield) {
    s->sfield = 1;
    s->Pd.sfield = s->Pf.sfield = 1;
    HIP_TRY(hipMemcpy(s->pd, &s->Pd, sizeof s->Pd, hipMemcpyHostToDevice));
    st = upload_jobs(s);
    if (st != MRTLB_OK) return st;
  }
  if (history) s->hist_pending = true;
  return MRTLB_OK;
}

mrtlb_status mrtlb_set_velocity_field(mrtlb_solve* s, const double* u) {
  if (!s || !u) return fail(MRTLB_EINVAL, "NULL argument");
  if (s->model.model != MRTLB_CDE) return fail(MRTLB_EINVAL, "the velocity field belongs to the CDE model");
  HIP_TRY(hipSetDevice(s->ctx->device));
  return upload_velocity(s, u);
}

mrtlb_status mrtlb_init_fields(mrtlb_solve* s, const double* rho, const double* u, const double* force) {
  if (!s || !rho) return fail(MRTLB_EINVAL, "NULL argument");
  const int D = s->L.D;
  const bool ncde = s->model.model == MRTLB_NCDE;
  const bool cde = s->model.model == MRTLB_CDE;
  if (!ncde && !u) return fail(MRTLB_EINVAL, "u is required for the NSE models and the CDE");
  if ((force != nullptr) != (s->has_force != 0)) return fail(MRTLB_EINVAL, "force must be given iff the solve has a force field");
  for (uint32_t i = 0; i < s->N; ++i)
    if (!std::isfinite(rho[i])) return fail(MRTLB_ENUMERIC, "non-finite initial density/phi");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  DevBuf dr, du, df;
  HIP_TRY(dr.alloc((size_t)s->N * 8, st));
  HIP_TRY(hipMemcpyAsync(dr.p, rho, (size_t)s->N * 8, hipMemcpyHostToDevice, st));
  if (cde) {
    const mrtlb_status vs = upload_velocity(s, u);
    if (vs != MRTLB_OK) return vs;
  } else if (!ncde) {
    HIP_TRY(du.alloc((size_t)D * s->N * 8, st));
    HIP_TRY(hipMemcpyAsync(du.p, u, (size_t)D * s->N * 8, hipMemcpyHostToDevice, st));
  }
  if (force) {
    HIP_TRY(df.alloc((size_t)D * s->N * 8, st));
    HIP_TRY(hipMemcpyAsync(df.p, force, (size_t)D * s->N * 8, hipMemcpyHostToDevice, st));
    // the stepping kernels read the force in the compute precision
    const mrtlb_status fs = upload_node_field(s, force, "force field");
    if (fs != MRTLB_OK) return fs;
  }
  s->cur = 0;
  s->steps = 0;
  s->hist_pending = false;           // the force was constant before t = 0
  // the init kernel writes f into buffer cur^1 and phi into both history
  // slots; run it with the parity-1 job so that fout = f[0]
  mrtlb_status rs = upload_jobs(s);
  if (rs != MRTLB_OK) return rs;
  rs = clear_saturation(s);
  if (rs != MRTLB_OK) return rs;
  LaunchReq r = base_req(*s, kOpInit, job_ptr(*s, 1));
  r.in0 = (const double*)dr.p;
  r.in1 = (const double*)du.p;
  r.in2 = (const double*)df.p;
  hipError_t err = dispatch(s->L.kind, r);
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("init launch: ") + hipGetErrorString(err));
  HIP_TRY(hipStreamSynchronize(st));
  return record_reference(s);
}

mrtlb_status mrtlb_step(mrtlb_solve* s, int64_t nsteps) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (nsteps < 0) return fail(MRTLB_EINVAL, "nsteps must be >= 0");
  HIP_TRY(hipSetDevice(s->ctx->device));
  for (int64_t k = 0; k < nsteps; ++k) {
    const void* jp = job_ptr(*s, s->cur);
    if (s->pending || s->hist_pending) {
      // a drift-corrected step, or the three-level step after a force
      // change, runs from job slot 2
      void* slot = static_cast<char*>(s->jobs) + 2 * (is_double(s->storage) ? sizeof(Job<double>) : sizeof(Job<float>));
      if (is_double(s->storage)) {
        Job<double> J = make_job(*s, s->cur, with_drift(*s, s->Pd));
        if (s->hist_pending) J.fprev = static_cast<const double*>(s->fprev);
        HIP_TRY(hipMemcpyAsync(slot, &J, sizeof J, hipMemcpyHostToDevice, s->ctx->stream));
        HIP_TRY(hipStreamSynchronize(s->ctx->stream));
      } else {
        Job<float> J = make_job(*s, s->cur, with_drift(*s, s->Pf));
        if (s->hist_pending) J.fprev = static_cast<const float*>(s->fprev);
        HIP_TRY(hipMemcpyAsync(slot, &J, sizeof J, hipMemcpyHostToDevice, s->ctx->stream));
        HIP_TRY(hipStreamSynchronize(s->ctx->stream));
      }
      jp = slot;
      s->pending = false;
      s->hist_pending = false;
    }
    hipError_t e = dispatch(s->L.kind, base_req(*s, kOpStep, jp));
    if (e != hipSuccess) return fail(MRTLB_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    s->cur ^= 1;
    s->steps += 1;
    if (s->drift_every > 0 && ++s->since_check >= s->drift_every) {
      mrtlb_status st = drift_check(s);
      if (st != MRTLB_OK) return st;
    }
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

mrtlb_status mrtlb_stream_only(mrtlb_solve* s, int64_t npasses, double* ms) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (npasses < 0) return fail(MRTLB_EINVAL, "npasses must be >= 0");
  if (s->L.kind == kCustom) return fail(MRTLB_EINVAL, "streaming alone is built for the compiled lattices only");
  HIP_TRY(hipSetDevice(s->ctx->device));
  if (ms) HIP_TRY(hipEventRecord(s->ctx->ev0, s->ctx->stream));
  for (int64_t k = 0; k < npasses; ++k) {
    hipError_t e = dispatch(s->L.kind, base_req(*s, kOpStream, job_ptr(*s, s->cur)));
    if (e != hipSuccess) return fail(MRTLB_EDEVICE, std::string("stream launch: ") + hipGetErrorString(e));
    s->cur ^= 1;
  }
  if (ms) {
    HIP_TRY(hipEventRecord(s->ctx->ev1, s->ctx->stream));
    HIP_TRY(hipEventSynchronize(s->ctx->ev1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, s->ctx->ev0, s->ctx->ev1));
    *ms = t;
  }
  return MRTLB_OK;
}

mrtlb_status mrtlb_solve_launch_shape(const mrtlb_solve* s, int* nodes_per_lane, int* xcd_ranges, int* wg_per_cu,
                                      int64_t* workgroups) {
  if (!s) return fail(MRTLB_EINVAL, "solve is NULL");
  if (nodes_per_lane) *nodes_per_lane = s->vec;
  if (xcd_ranges) *xcd_ranges = s->xcd_order ? 1 : 0;
  if (wg_per_cu) *wg_per_cu = s->step_lds > 0 ? (int)((uint32_t)s->ctx->lds_per_cu / s->step_lds) : 0;
  if (workgroups) *workgroups = (int64_t)s->nblocks;
  return MRTLB_OK;
}

static mrtlb_status reserve_jobs(mrtlb_ctx* c, size_t bytes) {
  if (bytes <= c->job_cap) return MRTLB_OK;
  size_t cap = std::max<size_t>(bytes, 2 * c->job_cap);
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->job_dev) HIP_TRY(hipFree(c->job_dev));
  if (c->job_host) HIP_TRY(hipHostFree(c->job_host));
  c->job_dev = c->job_host = nullptr;
  c->job_cap = 0;
  HIP_TRY(hipMalloc(&c->job_dev, cap));
  HIP_TRY(hipHostMalloc(&c->job_host, cap, hipHostMallocDefault));
  c->job_cap = cap;
  return MRTLB_OK;
}

// One group (same lattice, storage, model, force, nodes per thread).  Members
// are ordered by decreasing step count, so the solves still running at step
// k form a prefix of the job table: launch k covers jobs [0, m_k).  A
// segment of launches uses three job tables: the first launch (pending
// corrections and force history applied) and one per parity of the
// ping-pong buffers for the later launches.
using Group = std::vector<std::pair<mrtlb_solve*, int64_t>>;

static std::vector<uint32_t> group_prefix(const Group& g) {
  std::vector<uint32_t> prefix(g.size() + 1, 0);
  for (size_t i = 0; i < g.size(); ++i) prefix[i + 1] = prefix[i] + g[i].first->nblocks;
  return prefix;
}

// Steps of the group's next segment: up to the first member due for its FP64
// drift check.
static int64_t group_segment(const Group& g, int64_t done) {
  int64_t seg = g[0].second - done;
  for (const auto& m : g) {
    const mrtlb_solve& s = *m.first;
    if (s.drift_every > 0 && m.second > done) seg = std::min(seg, s.drift_every - s.since_check);
  }
  return seg;
}

template <class Real>
static void stage_group(const Group& g, const std::vector<uint32_t>& prefix, Job<Real>* jobs) {
  const size_t n = g.size();
  for (size_t i = 0; i < n; ++i) {
    const mrtlb_solve& s = *g[i].first;
    const KParams<Real>& P = *reinterpret_cast<const KParams<Real>*>(is_double(s.storage) ? (const void*)&s.Pd
                                                                                          : (const void*)&s.Pf);
    Job<Real> J0 = make_job(s, s.cur, with_drift(s, P));
    if (s.hist_pending) J0.fprev = static_cast<const Real*>(s.fprev);
    J0.block_begin = prefix[i];
    jobs[i] = J0;
    for (int par = 0; par < 2; ++par) {
      Job<Real> J = make_job(s, s.cur ^ par, P);
      J.block_begin = prefix[i];
      jobs[(size_t)(1 + par) * n + i] = J;
    }
  }
}

// Launches of steps [done, done + seg) of the group on `stream`, job tables at `table_dev`.
template <class Real>
static mrtlb_status launch_group(const Group& g, const std::vector<uint32_t>& prefix, const void* table_dev,
                                 int64_t done, int64_t seg, hipStream_t stream) {
  const size_t n = g.size();
  int m = (int)n;
  // several solves in one launch: tile order and occupancy cap for the batch
  const mrtlb_solve& a = *g[0].first;
  const bool xcd = pick_xcd_order(a.nxp, a.vec, a.L.D, a.storage, true);
  const uint32_t lds = pick_step_lds(a.ctx->lds_per_cu, a.ctx->lds_per_block, a.ctx->cus, prefix[n], a.L.D, a.L.kind,
                                     a.model.model, a.storage, a.L.B, a.vec, a.model.m2g_form == 1);
  for (int64_t k = 0; k < seg; ++k) {
    while (m > 0 && g[m - 1].second <= done + k) --m;
    const size_t table = k == 0 ? 0 : 1 + (size_t)(k & 1);
    const void* jp = static_cast<const char*>(table_dev) + table * n * sizeof(Job<Real>);
    LaunchReq r = base_req(*g[0].first, kOpStep, jp);
    if (n > 1) {
      r.xcd_order = xcd;
      r.lds = lds;
    }
    r.njobs = m;
    r.blocks = prefix[m];
    r.stream = stream;
    hipError_t e = dispatch(g[0].first->L.kind, r);
    if (e != hipSuccess) return fail(MRTLB_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
  }
  return MRTLB_OK;
}

// Host state after a segment has run (the stream synchronized): parities,
// step counts, and the FP64 drift checks that fall due.
static mrtlb_status finish_segment(const Group& g, int64_t done, int64_t seg) {
  for (const auto& m : g) {
    mrtlb_solve* s = m.first;
    const int64_t adv = std::max<int64_t>(0, std::min(m.second, done + seg) - done);
    if (adv == 0) continue;
    s->pending = false;
    s->hist_pending = false;
    s->cur ^= (int)(adv & 1);
    s->steps += adv;
    if (s->drift_every > 0 && (s->since_check += adv) >= s->drift_every) {
      mrtlb_status r2 = drift_check(s);
      if (r2 != MRTLB_OK) return r2;
    }
  }
  return MRTLB_OK;
}

// A group on the context stream, segment by segment.
template <class Real>
static mrtlb_status batch_group(Group& g) {
  std::stable_sort(g.begin(), g.end(), [](const auto& a, const auto& b) { return a.second > b.second; });
  mrtlb_ctx* c = g[0].first->ctx;
  const size_t n = g.size();
  mrtlb_status rs = reserve_jobs(c, 3 * n * sizeof(Job<Real>));
  if (rs != MRTLB_OK) return rs;
  hipStream_t st = c->stream;
  const std::vector<uint32_t> prefix = group_prefix(g);
  const int64_t total = g[0].second;
  int64_t done = 0;
  while (done < total) {
    const int64_t seg = group_segment(g, done);
    // the previous segment's copy out of the staging buffer has completed:
    // every segment ends with a stream synchronization
    stage_group<Real>(g, prefix, static_cast<Job<Real>*>(c->job_host));
    HIP_TRY(hipMemcpyAsync(c->job_dev, c->job_host, 3 * n * sizeof(Job<Real>), hipMemcpyHostToDevice, st));
    rs = launch_group<Real>(g, prefix, c->job_dev, done, seg, st);
    if (rs != MRTLB_OK) return rs;
    HIP_TRY(hipStreamSynchronize(st));
    rs = finish_segment(g, done, seg);
    if (rs != MRTLB_OK) return rs;
    done += seg;
  }
  return MRTLB_OK;
}

static size_t table_bytes(const Group& g) {
  const size_t job = is_double(g[0].first->storage) ? sizeof(Job<double>) : sizeof(Job<float>);
  return (3 * g.size() * job + 255) / 256 * 256;
}

// Groups that run in one segment (no drift check due inside the call), each
// on a side stream of the context so that their launches overlap on the
// device: one copy stages every group's job tables, an event releases the
// side streams after it, and the context stream waits for every group's
// last launch.
static mrtlb_status batch_concurrent(mrtlb_ctx* c, std::vector<Group>& groups) {
  size_t bytes = 0;
  std::vector<size_t> off;
  for (auto& g : groups) {
    std::stable_sort(g.begin(), g.end(), [](const auto& a, const auto& b) { return a.second > b.second; });
    off.push_back(bytes);
    bytes += table_bytes(g);
  }
  mrtlb_status rs = reserve_jobs(c, bytes);
  if (rs != MRTLB_OK) return rs;
  if (!c->side[0]) {
    for (int i = 0; i < kSideStreams; ++i) {
      HIP_TRY(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&c->side_done[i], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&c->staged, hipEventDisableTiming));
  }
  std::vector<std::vector<uint32_t>> prefix;
  for (size_t k = 0; k < groups.size(); ++k) {
    prefix.push_back(group_prefix(groups[k]));
    char* host = static_cast<char*>(c->job_host) + off[k];
    if (is_double(groups[k][0].first->storage))
      stage_group<double>(groups[k], prefix.back(), reinterpret_cast<Job<double>*>(host));
    else
      stage_group<float>(groups[k], prefix.back(), reinterpret_cast<Job<float>*>(host));
  }
  HIP_TRY(hipMemcpyAsync(c->job_dev, c->job_host, bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->staged, c->stream));
  bool used[kSideStreams] = {};
  for (size_t k = 0; k < groups.size(); ++k) {
    const int si = (int)(k % kSideStreams);
    hipStream_t st = c->side[si];
    if (!used[si]) HIP_TRY(hipStreamWaitEvent(st, c->staged, 0));
    used[si] = true;
    const void* dev = static_cast<const char*>(c->job_dev) + off[k];
    const int64_t total = groups[k][0].second;
    rs = is_double(groups[k][0].first->storage) ? launch_group<double>(groups[k], prefix[k], dev, 0, total, st)
                                                 : launch_group<float>(groups[k], prefix[k], dev, 0, total, st);
    if (rs != MRTLB_OK) return rs;
  }
  for (int si = 0; si < kSideStreams; ++si) {
    if (!used[si]) continue;
    HIP_TRY(hipEventRecord(c->side_done[si], c->side[si]));
    HIP_TRY(hipStreamWaitEvent(c->stream, c->side_done[si], 0));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& g : groups) {
    rs = finish_segment(g, 0, g[0].second);
    if (rs != MRTLB_OK) return rs;
  }
  return MRTLB_OK;
}

mrtlb_status mrtlb_batch_step(mrtlb_solve* const* solves, int n, const int64_t* nsteps) {
  if (!solves || n < 0 || (n > 0 && !nsteps)) return fail(MRTLB_EINVAL, "bad argument");
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return fail(MRTLB_EINVAL, "NULL solve in batch");
    if (nsteps[i] < 0) return fail(MRTLB_EINVAL, "nsteps must be >= 0");
    if (solves[i]->ctx != solves[0]->ctx) return fail(MRTLB_EINVAL, "solves of a batch must share a context");
    for (int k = 0; k < i; ++k)
      if (solves[k] == solves[i]) return fail(MRTLB_EINVAL, "a solve appears twice in the batch");
  }
  if (n == 0) return MRTLB_OK;
  HIP_TRY(hipSetDevice(solves[0]->ctx->device));
  // group by (lattice kind, storage, model, force, nodes per thread) in order
  // of first appearance; solves with nsteps == 0 are left alone
  std::vector<int> done(n, 0);
  std::vector<Group> groups;
  for (int i = 0; i < n; ++i) {
    if (done[i] || nsteps[i] == 0) continue;
    Group grp;
    const mrtlb_solve* a = solves[i];
    for (int k = i; k < n; ++k) {
      const mrtlb_solve* b = solves[k];
      // one launch serves one kernel: same lattice kind and dimension (user-
      // supplied lattices share a kind; their register class too), storage,
      // model, force and VEC
      if (!done[k] && nsteps[k] > 0 && b->L.kind == a->L.kind && b->L.D == a->L.D &&
          custom_class(b->L) == custom_class(a->L) && b->storage == a->storage &&
          b->crays == a->crays &&
          b->model.model == a->model.model && b->has_force == a->has_force && b->vec == a->vec &&
          b->transform == a->transform && b->model.m2g_form == a->model.m2g_form) {
        grp.emplace_back(solves[k], nsteps[k]);
        done[k] = 1;
      }
    }
    groups.push_back(std::move(grp));
  }
  // Several groups whose launches run in one segment overlap on side
  // streams; the rest (and a single group) run on the context stream.
  // MRTLB_BATCH_OVERLAP=0 runs every group on the context stream (A/B runs).
  const char* ov = std::getenv("MRTLB_BATCH_OVERLAP");
  const bool overlap = !(ov && ov[0] == '0');
  std::vector<Group> together, alone;
  for (auto& g : groups) {
    int64_t total = 0;
    for (const auto& m : g) total = std::max(total, m.second);
    int64_t seg = total;
    for (const auto& m : g)
      if (m.first->drift_every > 0) seg = std::min(seg, m.first->drift_every - m.first->since_check);
    (overlap && seg >= total ? together : alone).push_back(std::move(g));
  }
  if (together.size() == 1) alone.insert(alone.begin(), std::move(together[0]));
  if (together.size() > 1) {
    mrtlb_status st = batch_concurrent(solves[0]->ctx, together);
    if (st != MRTLB_OK) return st;
  }
  for (auto& g : alone) {
    mrtlb_status st = is_double(g[0].first->storage) ? batch_group<double>(g) : batch_group<float>(g);
    if (st != MRTLB_OK) return st;
  }
  return MRTLB_OK;
}

static mrtlb_status gather_launch(mrtlb_solve* s, int what, double* d0, double* d1) {
  LaunchReq r = base_req(*s, what == 1 ? kOpPopulations : kOpMoments, job_ptr(*s, s->cur));
  r.out0 = d0;
  r.out1 = d1;
  hipError_t err = dispatch(s->L.kind, r);
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("gather launch: ") + hipGetErrorString(err));
  return MRTLB_OK;
}

mrtlb_status mrtlb_read_moments(mrtlb_solve* s, double* rho, double* u) {
  if (!s || !rho) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const int D = s->L.D;
  DevBuf dr, du;
  HIP_TRY(dr.alloc((size_t)s->N * 8, s->ctx->stream));
  if (u) HIP_TRY(du.alloc((size_t)D * s->N * 8, s->ctx->stream));
  mrtlb_status st = gather_launch(s, 0, (double*)dr.p, (double*)du.p);
  if (st != MRTLB_OK) return st;
  HIP_TRY(hipMemcpyAsync(rho, dr.p, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, du.p, (size_t)D * s->N * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  return check_saturation(s);
}

mrtlb_status mrtlb_read_populations(mrtlb_solve* s, double* f) {
  if (!s || !f) return fail(MRTLB_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  DevBuf d;
  const size_t n = (size_t)s->L.B * s->N;
  HIP_TRY(d.alloc(n * 8, s->ctx->stream));
  mrtlb_status st = gather_launch(s, 1, (double*)d.p, nullptr);
  if (st != MRTLB_OK) return st;
  HIP_TRY(hipMemcpyAsync(f, d.p, n * 8, hipMemcpyDeviceToHost, s->ctx->stream));
  HIP_TRY(hipStreamSynchronize(s->ctx->stream));
  return check_saturation(s);
}

mrtlb_status mrtlb_write_populations(mrtlb_solve* s, const double* f) {
  if (!s || !f) return fail(MRTLB_EINVAL, "NULL argument");
  const size_t n = (size_t)s->L.B * s->N;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) return fail(MRTLB_ENUMERIC, "non-finite population");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t st = s->ctx->stream;
  DevBuf d;
  HIP_TRY(d.alloc(n * 8, s->ctx->stream));
  HIP_TRY(hipMemcpyAsync(d.p, f, n * 8, hipMemcpyHostToDevice, st));
  mrtlb_status cs = clear_saturation(s);
  if (cs != MRTLB_OK) return cs;
  // write into the current buffer: the parity-(cur^1) job has fout = f[cur]
  LaunchReq r = base_req(*s, kOpScatter, job_ptr(*s, s->cur ^ 1));
  r.in0 = (const double*)d.p;
  hipError_t err = dispatch(s->L.kind, r);
  if (err != hipSuccess) return fail(MRTLB_EDEVICE, std::string("scatter launch: ") + hipGetErrorString(err));
  HIP_TRY(hipStreamSynchronize(st));
  return record_reference(s);
}


