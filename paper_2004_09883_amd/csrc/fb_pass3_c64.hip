// Pencil passes for complex64 grids, axis lengths 2^a 3^b with b >= 2 (the
// matrix-core variants where the length has radix-16 stages and the tile is
// whole wavefronts).
#define FB_LENGTHS_3B
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass3_c64(int n, bool contig, bool mx) { return find_pass_t<float2, FB_LIST_B3>(n, contig, mx); }
}  // namespace fb
