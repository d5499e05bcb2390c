// Kernel instantiations for the d2q21k lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_d2q21k(const LaunchReq& r) { return launch_lattice<LatD2Q21K>(r); }
}  // namespace mrtlb
