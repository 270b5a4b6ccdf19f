// Compiled variants: 3D P^3 and Q^3 advection, FP64 and mixed precision:
// cooperative stage kernels on 16 x 2 x 2 tiles (one wavefront per tile).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    OpsCoop<3, 3, SYS_ADV, double, 16, 2, 2, SP_P>::make(), OpsCoop<3, 3, SYS_ADV, float, 16, 2, 2, SP_P>::make(),
    OpsCoop<3, 3, SYS_ADV, double, 16, 2, 2>::make(),       OpsCoop<3, 3, SYS_ADV, float, 16, 2, 2>::make(),
};
int variants_v3d_k3_adv(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
