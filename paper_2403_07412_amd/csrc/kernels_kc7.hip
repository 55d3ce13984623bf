// Kernel instantiations for covariance code 7: power exponential, great-circle distance.
#include "launch.h"

namespace vecchia {

int launch_kc7(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<7, true>(variant, a, s) : launch_variant<7, false>(variant, a, s);
}

}  // namespace vecchia
