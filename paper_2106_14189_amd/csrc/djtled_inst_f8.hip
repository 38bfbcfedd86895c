// Instantiates the single-mesh step and force kernels for FP32, H8 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_f8(const OpArgs &o) { return run_ops<float, 8, 0>(o); }

}  // namespace dj
