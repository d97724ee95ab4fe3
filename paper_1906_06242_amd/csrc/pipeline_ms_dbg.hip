// Instantiates the fused analysis kernel with per-event records
// (hepk_pipeline_debug), for plans whose queries have several jet-energy
// scales.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<true, true, false>(int, bool, int, int, bool);
}  // namespace hepk
