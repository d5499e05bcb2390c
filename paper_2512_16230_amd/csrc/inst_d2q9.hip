// Kernel instantiations for the standard D2Q9 lattice (k = 1 model).
#include "launchers.h"

namespace mrtlb {
hipError_t launch_d2q9(const LaunchReq& r) { return launch_lattice<LatD2Q9>(r); }
}  // namespace mrtlb
