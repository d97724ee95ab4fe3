// Instantiates the fused analysis kernel with the lookup corrections and
// per-event records, for plans whose queries have one jet-energy scale.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<false, true, true>(int, bool, int, int, bool);
}  // namespace hepk
