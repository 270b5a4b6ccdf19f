// Compiled variants: 3D Q^3 Euler (64 modes x 5 variables), FP64 and mixed
// precision: cooperative stage kernels on 16 x 2 x 2 tiles (the volume pass
// through LDS one slab of points at a time); the limiter, wave-speed,
// projection and queue kernels one thread per cell with rolled point loops
// (they spill: they run once per run or on the few queued cells).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    OpsCoop<3, 3, SYS_EULER, double, 16, 2, 2>::make(),
    OpsCoop<3, 3, SYS_EULER, float, 16, 2, 2>::make(),
};
int variants_v3d_q3_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
