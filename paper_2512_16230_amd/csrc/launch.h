// Host-side launch interface between the ABI layer and the per-lattice
// translation units that instantiate the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrtlb {

enum LaunchOp { kOpStep = 0, kOpInit = 1, kOpMoments = 2, kOpPopulations = 3, kOpScatter = 4, kOpStream = 5 };

struct LaunchReq {
  int op = kOpStep;
  int storage = 0;
  int model = 0;             // ModelKind
  bool force = false;        // NSE with a body-force field
  int vec = 1;               // step kernel: nodes per thread along x (1, 2, 4)
  int transform = 0;         // step kernel: Hermite transforms on VALU (0) or MFMA (1)
  bool m2g = false;          // NSE: the gradient form of M2G_bar (history fields, one node per lane)
  bool xcd_order = true;     // step kernel: tiles in contiguous ranges per XCD (else the dispatch order)
  uint32_t lds = 0;          // step and streaming kernels: LDS bytes each workgroup reserves (occupancy cap)
  int dim = 2;               // lattice dimension (user-supplied lattices)
  int custom_b = 0;          // user-supplied lattices: b (sizes the step kernel's register slots)
  bool custom_rays = false;  // user-supplied lattices: the step's slot table holds rays
  const void* jobs = nullptr;
  int njobs = 1;
  uint32_t blocks = 0;
  hipStream_t stream = nullptr;
  const void* pd = nullptr;  // device KParams<double>
  const double* in0 = nullptr;   // init: rho_or_phi; scatter: populations
  const double* in1 = nullptr;   // init: u
  const double* in2 = nullptr;   // init: force
  double* out0 = nullptr;        // gather: rho_or_phi or populations
  double* out1 = nullptr;        // gather: u
};

hipError_t launch_rd2q25(const LaunchReq& r);
hipError_t launch_rd2q13(const LaunchReq& r);
hipError_t launch_rd3q53(const LaunchReq& r);
hipError_t launch_rd3q33(const LaunchReq& r);
hipError_t launch_rd2q21(const LaunchReq& r);
hipError_t launch_d2q21k(const LaunchReq& r);
hipError_t launch_rd3q45(const LaunchReq& r);
hipError_t launch_rd2q17_1(const LaunchReq& r);
hipError_t launch_rd2q17_2(const LaunchReq& r);
hipError_t launch_rd2q17_3(const LaunchReq& r);
hipError_t launch_rd2q17_4(const LaunchReq& r);
hipError_t launch_rd2q17_5(const LaunchReq& r);
hipError_t launch_d2q9(const LaunchReq& r);
hipError_t launch_d3q27(const LaunchReq& r);
hipError_t launch_custom(const LaunchReq& r);

// FP64 sums of every population plane (and force plane) in chunks.
hipError_t launch_plane_sums(int storage, const void* base, uint32_t N, int npop, const void* force, int nforce,
                             const void* params, double* partial, uint32_t nchunks, hipStream_t stream);
// totals[p] = sum over c of partial[p * nchunks + c], in chunk order.
hipError_t launch_plane_totals(const double* partial, uint32_t nchunks, int planes, double* totals,
                               hipStream_t stream);

}  // namespace mrtlb
