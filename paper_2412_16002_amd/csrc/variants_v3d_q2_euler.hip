// Compiled variants: 3D Q^2 Euler (27 modes x 5 variables), FP64 and mixed
// precision: cooperative stage kernels on 16 x 2 x 2 tiles; the limiter,
// wave-speed and projection kernels one thread per cell (rolled point loops).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    OpsCoop<3, 2, SYS_EULER, double, 16, 2, 2>::make(), OpsCoop<3, 2, SYS_EULER, float, 16, 2, 2>::make(),
};
int variants_v3d_q2_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
