// Instantiates the single-mesh step and force kernels for FP32 classical TLED form, H8 elements.
#include "djtled_step.h"

namespace dj {

hipError_t inst_c8(const OpArgs &o) { return run_ops<float, 8, DJ_FORM_TLED>(o); }

}  // namespace dj
