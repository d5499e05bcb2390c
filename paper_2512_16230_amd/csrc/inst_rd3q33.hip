// Kernel instantiations for the rd3q33 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd3q33(const LaunchReq& r) { return launch_lattice<LatRD3Q33>(r); }
}  // namespace mrtlb
