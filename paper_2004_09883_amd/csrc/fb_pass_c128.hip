// Pencil passes for complex128 grids (binary64 arithmetic).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_c128(int n, bool contig);
PassInfo find_pass_c128(int n, bool contig, bool mx)
{
    const PassInfo r = find_pass_t<double2, FB_LIST_B3>(n, contig, mx);
    return r.launch ? r : find_pass3_c128(n, contig);
}
}  // namespace fb
