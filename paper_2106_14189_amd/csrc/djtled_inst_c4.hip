// Instantiates the single-mesh step and force kernels for FP32 classical TLED form, T4 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_c4(const OpArgs &o) { return run_ops<float, 4, DJ_FORM_TLED>(o); }

}  // namespace dj
