// Evaluation + elimination kernels of register class 64 (largest y-degree 64).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(64)
}  // namespace snc
