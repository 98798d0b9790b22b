// Instantiates the advance kernel for the launch shapes of group J.
#include "advance_impl.h"
#include "variants.h"

namespace mdeos {
#define X(B, A, E, L, W, M, T, P) MDEOS_DEFINE_VARIANT(B, A, E, L, W, M, T, P)
MDEOS_VARIANTS_J(X)
#undef X
}  // namespace mdeos
