// Evaluation + elimination kernels of register class 16 (largest y-degree 16).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(16)
}  // namespace snc
