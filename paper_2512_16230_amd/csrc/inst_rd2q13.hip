// Kernel instantiations for the rd2q13 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q13(const LaunchReq& r) { return launch_lattice<LatRD2Q13>(r); }
}  // namespace mrtlb
