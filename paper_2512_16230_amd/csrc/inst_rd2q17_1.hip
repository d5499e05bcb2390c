// Kernel instantiations for the D2Q17 case-1 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q17_1(const LaunchReq& r) { return launch_lattice<LatRD2Q17_1>(r); }
}  // namespace mrtlb
