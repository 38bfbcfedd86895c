// Instantiates the single-mesh step and force kernels for FP64, H8 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_d8(const OpArgs &o) { return run_ops<double, 8, 0>(o); }

}  // namespace dj
