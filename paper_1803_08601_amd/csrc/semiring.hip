// Forward product over the (min, +), (max, +) and (max, *) semirings with the
// same kernels and launch shapes as the ordinary product (tiles.hpp).

#include "tiles.hpp"

namespace spmmk {

hipError_t launch_forward_semiring(int semiring, int dtype, bool merge, const Shape& s,
                                   const ForwardArgs& a, hipStream_t st) {
    switch (semiring) {
    case 1: return launch_forward<MinPlus>(dtype, merge, s, a, st, nullptr);
    case 2: return launch_forward<MaxPlus>(dtype, merge, s, a, st, nullptr);
    case 3: return launch_forward<MaxTimes>(dtype, merge, s, a, st, nullptr);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spmmk
