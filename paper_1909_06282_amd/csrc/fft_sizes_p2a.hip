// Kernel instantiations for grid sizes: 8 16 32 64 128 (one translation unit per
// group, so the build compiles the groups in parallel).
#include "fft_passes.hpp"

namespace lpt2 {
LPT2_INSTANTIATE_SIZE(8)
LPT2_INSTANTIATE_SIZE(16)
LPT2_INSTANTIATE_SIZE(32)
LPT2_INSTANTIATE_SIZE(64)
LPT2_INSTANTIATE_SIZE(128)
}  // namespace lpt2
