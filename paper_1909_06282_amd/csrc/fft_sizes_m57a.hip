// Kernel instantiations for grid sizes: 40 56 200 (one translation unit per
// group, so the build compiles the groups in parallel).
#include "fft_passes.hpp"

namespace lpt2 {
LPT2_INSTANTIATE_SIZE(40)
LPT2_INSTANTIATE_SIZE(56)
LPT2_INSTANTIATE_SIZE(200)
}  // namespace lpt2
