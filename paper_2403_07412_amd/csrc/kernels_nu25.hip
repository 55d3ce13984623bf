// Kernel instantiations for Matern smoothness nu = 2.5.
#include "launch.h"

namespace vecchia {

int launch_nu25(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<2, true>(variant, a, s) : launch_variant<2, false>(variant, a, s);
}

}  // namespace vecchia
