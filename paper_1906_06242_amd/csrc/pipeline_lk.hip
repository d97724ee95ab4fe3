// Instantiates the fused analysis kernel with the lookup corrections (event
// weights from lookup histograms, shifted jet energies, squared weights) for
// plans whose queries have one jet-energy scale.
#include "pipeline_kernel.hpp"

namespace hepk {
template KernelFn pick_kernel<false, false, true>(int, bool, int, int, bool);
}  // namespace hepk
