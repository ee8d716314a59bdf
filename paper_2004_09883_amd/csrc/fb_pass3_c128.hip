// Pencil passes for complex128 grids, axis lengths 2^a 3^b with b >= 2.
#define FB_LENGTHS_3B
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_c128(int n, bool contig) { return find_pass_t<double2, FB_LIST_B3>(n, contig, false); }
}  // namespace fb
