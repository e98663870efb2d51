// Advection kernels for F32 node storage (see advect_impl.h).
#include "advect_impl.h"

namespace streami {
int launch_advect_f32(const AdvectArgs& a, int layout, bool periodic, int mode, bool batched, int grid,
                      hipStream_t st) {
  return launch_advect_fmt<FMT_F32>(a, layout, periodic, mode, batched, grid, st);
}
int launch_surrogate_f32(const SurrogateArgs& s, int layout, bool periodic, bool pre, int grid,
                          hipStream_t st) {
  return launch_surrogate_fmt<FMT_F32>(s, layout, periodic, pre, grid, st);
}
}  // namespace streami
