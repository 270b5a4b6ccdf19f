// Compiled variants: 3D P^3 (total degree) Euler, FP64 and mixed precision:
// the cooperative stage kernels of Q^3 on 16 x 2 x 2 tiles with the modes
// outside P^3 held at zero and never stored (the FP64 volume pass goes
// through LDS one slab of points at a time).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    OpsCoop<3, 3, SYS_EULER, double, 16, 2, 2, SP_P>::make(),
    OpsCoop<3, 3, SYS_EULER, float, 16, 2, 2, SP_P>::make(),
};
int variants_v3d_p3_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
