// Kernel instantiations for the D2Q17 case-2 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q17_2(const LaunchReq& r) { return launch_lattice<LatRD2Q17_2>(r); }
}  // namespace mrtlb
