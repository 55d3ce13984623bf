// Kernel instantiations for covariance code 5: Matern nu = 1.5, great-circle distance.
#include "launch.h"

namespace vecchia {

int launch_kc5(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<5, true>(variant, a, s) : launch_variant<5, false>(variant, a, s);
}

}  // namespace vecchia
