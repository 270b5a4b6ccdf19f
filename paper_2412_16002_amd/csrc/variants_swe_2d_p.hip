// Compiled variants: shallow water (flat bottom), 2D P^1..P^3; FP64 and mixed
// precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<2, 1, SP_P, SYS_SWE, double>::make(), Ops<2, 1, SP_P, SYS_SWE, float>::make(),
    Ops<2, 2, SP_P, SYS_SWE, double>::make(), Ops<2, 2, SP_P, SYS_SWE, float>::make(),
    Ops<2, 3, SP_P, SYS_SWE, double>::make(), Ops<2, 3, SP_P, SYS_SWE, float>::make(),
};
int variants_swe_2d_p(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
