// Kernel instantiations for the D2Q17 case-5 lattice.
#include "launchers.h"

namespace mrtlb {
hipError_t launch_rd2q17_5(const LaunchReq& r) { return launch_lattice<LatRD2Q17_5>(r); }
}  // namespace mrtlb
