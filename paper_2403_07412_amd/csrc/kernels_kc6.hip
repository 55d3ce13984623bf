// Kernel instantiations for covariance code 6: Matern nu = 2.5, great-circle distance.
#include "launch.h"

namespace vecchia {

int launch_kc6(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<6, true>(variant, a, s) : launch_variant<6, false>(variant, a, s);
}

}  // namespace vecchia
