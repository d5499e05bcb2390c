// Kernel instantiations for the rd2q25 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q25(const LaunchReq& r) { return launch_lattice<LatRD2Q25>(r); }
}  // namespace mrtlb
