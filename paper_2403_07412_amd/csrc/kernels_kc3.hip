// Kernel instantiations for covariance code 3: power exponential, Euclidean distance.
#include "launch.h"

namespace vecchia {

int launch_kc3(bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    return grad ? launch_variant<3, true>(variant, a, s) : launch_variant<3, false>(variant, a, s);
}

}  // namespace vecchia
