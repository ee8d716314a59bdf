// Strided pencil-pair passes for complex64 grids, axis lengths 2^a 3^b with
// b >= 2.
#define FB_LENGTHS_3B
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_pair(int n, bool mx) { return find_pass_pair_t<FB_LIST_B3>(n, mx); }
}  // namespace fb
