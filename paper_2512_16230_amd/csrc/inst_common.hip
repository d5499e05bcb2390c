// Lattice-independent kernels: FP64 plane sums for the conserved quantities.
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

}  // namespace mrtlb
