// BF16-split sigma kernel (see k_sigma.hip for the method and the FP64/FP32 kernels).
#include "internal.h"

namespace pprpa {

hipError_t launch_sigma_bf16(const Geometry& g, const SigmaPlan& plan, const SigmaLaunch& la,
                             hipStream_t s) {
  (void)g;
  (void)plan;
  (void)la;
  (void)s;
  return hipErrorNotSupported;
}

}  // namespace pprpa
