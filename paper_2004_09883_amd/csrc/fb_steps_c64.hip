// Multi-output contiguous evolve passes for complex64 grids (the
// matrix-core variants of the radix-16 stages included).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_multi_c64(int n, bool mx);
PassInfo find_pass_multi_c64(int n, bool mx)
{
    const PassInfo r = find_pass_multi_t<float2, FB_LIST_B3>(n, mx);
    return r.launch ? r : find_pass3_multi_c64(n, mx);
}
}  // namespace fb
