// Compiled variant: 3D P^2 (total degree) Euler, mixed precision only.  The
// FP64 form, fully unrolled, spills ~3.5 KB per lane and is not built; the
// mixed form keeps its state in VGPRs and AGPRs (one wavefront per SIMD).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<3, 2, SP_P, SYS_EULER, float>::make(),
};
int variants_v3d_p2_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
