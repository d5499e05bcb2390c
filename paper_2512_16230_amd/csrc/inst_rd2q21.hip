// Kernel instantiations for the rd2q21 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q21(const LaunchReq& r) { return launch_lattice<LatRD2Q21>(r); }
}  // namespace mrtlb
