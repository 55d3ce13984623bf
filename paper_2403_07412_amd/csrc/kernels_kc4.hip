// Kernel instantiations for covariance code 4: Matern nu = 0.5, great-circle distance.
#include "launch.h"

namespace vecchia {

int launch_kc4(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<4, true>(variant, a, s) : launch_variant<4, false>(variant, a, s);
}

}  // namespace vecchia
