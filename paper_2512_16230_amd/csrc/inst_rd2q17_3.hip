// Kernel instantiations for the D2Q17 case-3 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q17_3(const LaunchReq& r) { return launch_lattice<LatRD2Q17_3>(r); }
}  // namespace mrtlb
