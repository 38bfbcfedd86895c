// Instantiates the single-mesh step and force kernels for FP32, T4 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_f4(const OpArgs &o) { return run_ops<float, 4, 0>(o); }

}  // namespace dj
