// Kernel instantiations for the D2Q17 case-4 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q17_4(const LaunchReq& r) { return launch_lattice<LatRD2Q17_4>(r); }
}  // namespace mrtlb
