// Kernel instantiations for the standard D3Q27 lattice (k = 1 model).
#include "launchers.h"

namespace mrtlb {
hipError_t launch_d3q27(const LaunchReq& r) { return launch_lattice<LatD3Q27>(r); }
}  // namespace mrtlb
