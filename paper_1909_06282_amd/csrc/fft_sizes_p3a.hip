// Kernel instantiations for grid sizes: 24 48 96 192 (one translation unit per
// group, so the build compiles the groups in parallel).
#include "fft_passes.hpp"

namespace lpt2 {
LPT2_INSTANTIATE_SIZE(24)
LPT2_INSTANTIATE_SIZE(48)
LPT2_INSTANTIATE_SIZE(96)
LPT2_INSTANTIATE_SIZE(192)
}  // namespace lpt2
