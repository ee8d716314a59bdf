// Multi-output contiguous evolve passes for complex64 grids, axis lengths
// 2^a 3^b with b >= 2.
#define FB_LENGTHS_3B
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_multi_c64(int n, bool mx) { return find_pass_multi_t<float2, FB_LIST_B3>(n, mx); }
}  // namespace fb
