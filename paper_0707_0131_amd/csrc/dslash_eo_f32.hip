// Odd-even (Schur complement) stencil launches for FP32 storage: instantiates the
// odd-even kernels of stencil_impl.h for this precision in a translation unit of its own.
#include "stencil_impl.h"

namespace eigcg {

hipError_t launch_stencil_eo_f32(const StencilLaunch& L, hipStream_t s) {
  return launch_eo<float2, float2>(L, s);
}

}  // namespace eigcg
