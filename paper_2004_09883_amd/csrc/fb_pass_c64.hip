// Pencil passes for complex64 grids (binary32 arithmetic; the matrix-core
// variants of the radix-16 stages included).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_c64(int n, bool contig, bool mx);
PassInfo find_pass_c64(int n, bool contig, bool mx)
{
    const PassInfo r = find_pass_t<float2, FB_LIST_B3>(n, contig, mx);
    return r.launch ? r : find_pass3_c64(n, contig, mx);
}
}  // namespace fb
