// User-supplied 2D velocity sets: kernel instantiations and the dispatch
// of every user-supplied lattice by dimension.
#include "custom.h"

namespace mrtlb {

hipError_t launch_custom_2d(const LaunchReq& r) { return launch_custom_dim<2>(r); }

hipError_t launch_custom(const LaunchReq& r) { return r.dim == 3 ? launch_custom_3d(r) : launch_custom_2d(r); }

}  // namespace mrtlb
