// Multi-output contiguous evolve passes for complex128 grids: several
// evolution steps of the spectral block from one read of the spectrum.
#include "fb_pass_inst.hpp"

namespace fb {
PassInfo find_pass_multi_c128(int n) { return find_pass_multi_t<double2>(n, false); }
}  // namespace fb
