// Instantiates the fused analysis kernel with the lookup corrections for
// plans whose queries have several jet-energy scales.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<true, false, true>(int, bool, int, int, bool);
}  // namespace hepk
