// Evaluation + elimination kernels of register class 40 (largest y-degree 40).
#include "eval_elim.hpp"

namespace snc {
SNC_EVAL_ELIM_CLASS(40)
}  // namespace snc
