// Multi-output contiguous evolve passes for complex64 grids (the
// matrix-core variants of the radix-16 stages included).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass_multi_c64(int n, bool mx) { return find_pass_multi_t<float2>(n, mx); }
}  // namespace fb
