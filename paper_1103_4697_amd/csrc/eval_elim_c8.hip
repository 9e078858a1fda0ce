// Evaluation + elimination kernels of register class 8 (largest y-degree 8).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(8)
}  // namespace snc
