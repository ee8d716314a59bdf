// Multi-output contiguous evolve passes for complex128 grids: several
// evolution steps of the spectral block from one read of the spectrum.
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_multi_c128(int n);
PassInfo find_pass_multi_c128(int n)
{
    const PassInfo r = find_pass_multi_t<double2, FB_LIST_B3>(n, false);
    return r.launch ? r : find_pass3_multi_c128(n);
}
}  // namespace fb
