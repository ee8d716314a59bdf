// Strided pencil passes for complex64 grids over pencil pairs (16-byte
// accesses).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_pair(int n, bool mx);
PassInfo find_pass_pair(int n, bool mx)
{
    const PassInfo r = find_pass_pair_t<FB_LIST_B3>(n, mx);
    return r.launch ? r : find_pass3_pair(n, mx);
}
}  // namespace fb
