// Lattice-independent kernels: FP64 plane sums for the conserved quantities
// (partial sums per chunk, then totals per plane).
#include "device.h"

namespace mrtlb {

hipError_t launch_plane_sums(int storage, const void* base, uint32_t N, int npop, const void* force, int nforce,
                             const void* params, double* partial, uint32_t nchunks, hipStream_t stream) {
  hipError_t err = hipErrorInvalidValue;
  with_storage(storage, [&](auto stc) {
    constexpr int ST = decltype(stc)::value;
    using Real = typename StoreT<ST>::Real;
    hipLaunchKernelGGL((k_plane_sums<ST>), dim3(nchunks, npop + nforce), dim3(kBlock), 0, stream, base, N, npop,
                       static_cast<const Real*>(force), nforce, static_cast<const KParams<Real>*>(params), partial,
                       nchunks);
    err = hipGetLastError();
  });
  return err;
}

// Per-plane totals of the partial sums, one wavefront per plane: lane l
// adds chunks l, l + 64, ... in order, then a fixed butterfly combines the
// lanes (a fixed order, so every caller gets the same bits).
__global__ __launch_bounds__(64) void k_plane_totals(const double* __restrict__ partial, uint32_t nchunks,
                                                     double* __restrict__ totals) {
  const int p = blockIdx.x;
  double acc = 0;
  for (uint32_t c = threadIdx.x; c < nchunks; c += 64) acc += partial[(size_t)p * nchunks + c];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) totals[p] = acc;
}

hipError_t launch_plane_totals(const double* partial, uint32_t nchunks, int planes, double* totals,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_plane_totals, dim3(planes), dim3(64), 0, stream, partial, nchunks, totals);
  return hipGetLastError();
}

}  // namespace mrtlb
