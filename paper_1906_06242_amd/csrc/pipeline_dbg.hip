// Instantiates the fused analysis kernel with per-event records
// (hepk_pipeline_debug), for plans whose queries have one jet-energy scale.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<false, true, false>(int, bool, int, int, bool);
}  // namespace hepk
