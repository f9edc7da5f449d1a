// Kernel instantiations for grid sizes: 768 (one translation unit per
// group, so the build compiles the groups in parallel).
#include "fft_passes.hpp"

namespace lpt2 {
LPT2_INSTANTIATE_SIZE(768)
}  // namespace lpt2
