// Odd-even (Schur complement) stencil launches for 16-bit storage: instantiates the
// odd-even kernels of stencil_impl.h for this precision in a translation unit of its own.
#include "stencil_impl.h"

namespace eigcg {

hipError_t launch_stencil_eo_f16(const StencilLaunch& L, hipStream_t s) {
  return launch_eo<f16x2, f16x2>(L, s);
}

}  // namespace eigcg
