// Evaluation + elimination kernels of register class 32 (largest y-degree 32).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(32)
}  // namespace snc
