// Instantiates the fused analysis kernel with the lookup corrections and
// per-event records, for plans whose queries have several jet-energy scales.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<true, true, true>(int, bool, int, int, bool);
}  // namespace hepk
