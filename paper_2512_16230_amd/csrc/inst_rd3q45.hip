// Kernel instantiations for the rd3q45 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd3q45(const LaunchReq& r) { return launch_lattice<LatRD3Q45>(r); }
}  // namespace mrtlb
