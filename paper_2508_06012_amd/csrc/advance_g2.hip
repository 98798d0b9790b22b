// Instantiates the advance kernel for the launch shape of group G2 (embedded-atom potential, minimum image, 8 atoms per thread).
#include "advance_impl.h"
#include "variants.h"

namespace mdeos {
#define X(B, A, E, L, W, M, T, P) MDEOS_DEFINE_VARIANT(B, A, E, L, W, M, T, P)
MDEOS_VARIANTS_G2(X)
#undef X
}  // namespace mdeos
