// Strided pencil passes for complex64 grids over pencil pairs (16-byte
// accesses).
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass_pair(int n, bool mx) { return find_pass_pair_t(n, mx); }
}  // namespace fb
