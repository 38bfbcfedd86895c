// Instantiates the single-mesh step and force kernels for FP64, T4 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_d4(const OpArgs &o) { return run_ops<double, 4, 0>(o); }

}  // namespace dj
