// Odd-even (Schur complement) stencil launches for FP64 storage: instantiates the
// odd-even kernels of stencil_impl.h for this precision in a translation unit of its own.
#include "stencil_impl.h"

namespace eigcg {

hipError_t launch_stencil_eo_f64(const StencilLaunch& L, hipStream_t s) {
  return launch_eo<double2, double2>(L, s);
}

}  // namespace eigcg
