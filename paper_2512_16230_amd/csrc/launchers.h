// Host launchers of one lattice's kernels (step, initialisation, read-out,
// restore), included by the per-lattice translation units inst_*.hip.
#pragma once

#include "device.h"
#include "mfma.h"

namespace mrtlb {

template <class L>
hipError_t launch_lattice(const LaunchReq& r) {
  hipError_t err = hipErrorInvalidValue;
  const dim3 grid(r.blocks), block(kBlock);
  // a tile total of 0 leaves the dispatch order (xcd_remap is the identity)
  const uint32_t tb = r.xcd_order ? r.blocks : 0u;
  with_storage(r.storage, [&](auto stc) {
    constexpr int ST = decltype(stc)::value;
    using Real = typename StoreT<ST>::Real;
    const auto* J = static_cast<const Job<Real>*>(r.jobs);
    const auto* PD = static_cast<const KParams<double>*>(r.pd);
    const bool ncde = r.model == kNcde;
    const bool cde = r.model == kCde;
    // the gradient form of M2G_bar is built for the FP32 and FP64 storages
    constexpr bool kGradBuilt = ST == kFP64 || ST == kFP32 || ST == kFP32Dev || ST == kFP32DevF64;
    switch (r.op) {
      case kOpStep: {
        // Several nodes per thread are built only where the host picks them:
        // the NSE models on the 2D lattices.  Any other request is refused.
        bool launched = false;
        auto step = [&](auto vc) {
          constexpr int V = decltype(vc)::value;
          if (ncde) {
            if constexpr (V == 1) {
              hipLaunchKernelGGL((k_step<L, ST, kNcde, false, V>), grid, block, r.lds, r.stream, J, r.njobs, tb);
              launched = true;
            }
          } else if (cde) {
            if constexpr (V == 1) {
              hipLaunchKernelGGL((k_step<L, ST, kCde, false, V>), grid, block, r.lds, r.stream, J, r.njobs, tb);
              launched = true;
            }
          } else if constexpr (L::D == 2 || V == 1) {
            if (r.force)
              hipLaunchKernelGGL((k_step<L, ST, kNseComp, true, V>), grid, block, r.lds, r.stream, J, r.njobs, tb);
            else
              hipLaunchKernelGGL((k_step<L, ST, kNseComp, false, V>), grid, block, r.lds, r.stream, J, r.njobs, tb);
            launched = true;
          }
        };
        if (r.m2g) {
          if constexpr (kGradBuilt) {
            if (!ncde && !cde && r.vec == 1) {
              if (r.force)
                hipLaunchKernelGGL((k_step<L, ST, kNseGrad, true, 1>), grid, block, r.lds, r.stream, J, r.njobs, tb);
              else
                hipLaunchKernelGGL((k_step<L, ST, kNseGrad, false, 1>), grid, block, r.lds, r.stream, J, r.njobs, tb);
              launched = true;
            }
          }
        } else if (r.transform == 1) {
          // MFMA transforms: 3D lattices, int16 storage, the NSE models without a force field
          if constexpr (L::D == 3 && ST == kI16Dev) {
            if (!ncde && !cde && !r.force) {
              hipLaunchKernelGGL((k_step_mfma<L, kNseComp>), grid, block, 0, r.stream, J, r.njobs, tb);
              launched = true;
            }
          }
        } else if (r.vec == 4) {
          step(std::integral_constant<int, 4>{});
        } else if (r.vec == 2) {
          step(std::integral_constant<int, 2>{});
        } else {
          step(std::integral_constant<int, 1>{});
        }
        if (!launched) return;
        break;
      }
      case kOpInit:
        if (r.m2g) {
          if constexpr (kGradBuilt) {
            hipLaunchKernelGGL((k_init<L, ST, kNseGrad>), grid, block, 0, r.stream, J, PD, r.in0, r.in1, r.in2, r.blocks);
          } else {
            return;
          }
        } else if (ncde) {
          hipLaunchKernelGGL((k_init<L, ST, kNcde>), grid, block, 0, r.stream, J, PD, r.in0, r.in1, r.in2, r.blocks);
        } else if (cde) {
          hipLaunchKernelGGL((k_init<L, ST, kCde>), grid, block, 0, r.stream, J, PD, r.in0, r.in1, r.in2, r.blocks);
        } else {
          hipLaunchKernelGGL((k_init<L, ST, kNseComp>), grid, block, 0, r.stream, J, PD, r.in0, r.in1, r.in2, r.blocks);
        }
        break;
      case kOpMoments:
        if (ncde) {
          hipLaunchKernelGGL((k_gather<L, ST, kNcde, 0>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        } else if (cde) {
          hipLaunchKernelGGL((k_gather<L, ST, kCde, 0>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        } else {
          hipLaunchKernelGGL((k_gather<L, ST, kNseComp, 0>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        }
        break;
      case kOpPopulations:
        hipLaunchKernelGGL((k_gather<L, ST, kNseComp, 1>), grid, block, 0, r.stream, J, PD, r.out0, r.out1);
        break;
      case kOpScatter:
        hipLaunchKernelGGL((k_scatter<L, ST>), grid, block, 0, r.stream, J, PD, r.in0);
        break;
      case kOpStream:
        // the step kernel's launch shape: VEC 2 and 4 on the 2D lattices only
        if constexpr (L::D == 2) {
          if (r.vec == 4)
            hipLaunchKernelGGL((k_stream<L, ST, 4>), grid, block, r.lds, r.stream, J, tb);
          else if (r.vec == 2)
            hipLaunchKernelGGL((k_stream<L, ST, 2>), grid, block, r.lds, r.stream, J, tb);
          else
            hipLaunchKernelGGL((k_stream<L, ST, 1>), grid, block, r.lds, r.stream, J, tb);
        } else {
          if (r.vec != 1) return;
          hipLaunchKernelGGL((k_stream<L, ST, 1>), grid, block, r.lds, r.stream, J, tb);
        }
        break;
      default:
        return;
    }
    err = hipGetLastError();
  });
  return err;
}

}  // namespace mrtlb
