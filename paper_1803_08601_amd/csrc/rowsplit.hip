// Forward product over the ordinary (+, *) semiring: row split (Sec. 4.1) and
// merge-based Phases 2-3 (Sec. 4.2). Kernels and tile functions: tiles.hpp.

#include "tiles.hpp"

namespace spmmk {

hipError_t launch_forward_plus_times(int dtype, bool merge, const Shape& s,
                                     const ForwardArgs& a, hipStream_t st, hipEvent_t ev_after) {
    return launch_forward<PlusTimes>(dtype, merge, s, a, st, ev_after);
}

}  // namespace spmmk
