// User-supplied 3D velocity sets: kernel instantiations.
#include "custom.h"

namespace mrtlb {

hipError_t launch_custom_3d(const LaunchReq& r) { return launch_custom_dim<3>(r); }

}  // namespace mrtlb
