// Instantiates the fused analysis kernel for plans whose queries have
// several jet-energy scales (compiled apart from pipeline.hip so the sets of
// kernels build in parallel).
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<true, false, false>(int, bool, int, int, bool);
}  // namespace hepk
