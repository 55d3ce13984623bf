// Kernel instantiations for Matern smoothness nu = 1.5.
#include "launch.h"

namespace vecchia {

int launch_nu15(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<1, true>(variant, a, s) : launch_variant<1, false>(variant, a, s);
}

}  // namespace vecchia
