// Compiled variants: shallow water (flat bottom), 1D P^1..P^3 and 2D Q^1..Q^3;
// FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<1, 1, SP_Q, SYS_SWE, double>::make(), Ops<1, 1, SP_Q, SYS_SWE, float>::make(),
    Ops<1, 2, SP_Q, SYS_SWE, double>::make(), Ops<1, 2, SP_Q, SYS_SWE, float>::make(),
    Ops<1, 3, SP_Q, SYS_SWE, double>::make(), Ops<1, 3, SP_Q, SYS_SWE, float>::make(),
    Ops<2, 1, SP_Q, SYS_SWE, double>::make(), Ops<2, 1, SP_Q, SYS_SWE, float>::make(),
    Ops<2, 2, SP_Q, SYS_SWE, double>::make(), Ops<2, 2, SP_Q, SYS_SWE, float>::make(),
    Ops<2, 3, SP_Q, SYS_SWE, double>::make(), Ops<2, 3, SP_Q, SYS_SWE, float>::make(),
};
int variants_swe_1d_q(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
