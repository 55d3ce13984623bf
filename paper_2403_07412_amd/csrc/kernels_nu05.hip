// Kernel instantiations for Matern smoothness nu = 0.5.
#include "launch.h"

namespace vecchia {

int launch_nu05(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<0, true>(variant, a, s) : launch_variant<0, false>(variant, a, s);
}

}  // namespace vecchia
