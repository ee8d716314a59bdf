// Pencil passes for complex128 grids (binary64 arithmetic).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass_c128(int n, bool contig, bool mx) { return find_pass_t<double2>(n, contig, mx); }
}  // namespace fb
