// Kernel instantiations for the rd3q53 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd3q53(const LaunchReq& r) { return launch_lattice<LatRD3Q53>(r); }
}  // namespace mrtlb
