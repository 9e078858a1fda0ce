// Evaluation + elimination kernels of register class 48 (largest y-degree 48).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(48)
}  // namespace snc
