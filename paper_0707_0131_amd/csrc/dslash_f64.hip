// Stencil launches for FP64 storage (and the precision dispatcher): instantiates the kernels of
// stencil_impl.h for this precision in a translation unit of its own.
#include "stencil_impl.h"

namespace eigcg {

hipError_t launch_stencil_f64(const StencilLaunch& L, hipStream_t s) {
  return launch_typed<double2, double2>(L, s);
}

hipError_t launch_finalize_cg(ColState* st, int ncols, uint32_t mask, const double* part_a,
                              const double* part_b, int nb, double* hist, int hist_stride,
                              const double* spec_s, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_cg, dim3(ncols), dim3(kBlock), 0, s, st, ncols, mask, part_a,
                     part_b, nb, hist, hist_stride, spec_s);
  return hipGetLastError();
}

hipError_t launch_stencil(const StencilLaunch& L, hipStream_t s) {
  if (L.ncols <= 0 || L.ncols > kMaxCols) return hipErrorInvalidValue;
  if (L.g->eo) {
    if (L.prec == kF64) return launch_stencil_eo_f64(L, s);
    if (L.prec == kF32) return launch_stencil_eo_f32(L, s);
    return launch_stencil_eo_f16(L, s);
  }
  if (L.prec == kF64) return launch_stencil_f64(L, s);
  if (L.prec == kF32) return launch_stencil_f32(L, s);
  return launch_stencil_f16(L, s);
}

}  // namespace eigcg
