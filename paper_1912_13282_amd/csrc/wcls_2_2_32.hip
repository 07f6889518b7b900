// Size class: d = 2, degree 2, n + m <= 32.
#include "weights_kernels.hpp"

RBF_WEIGHTS_CLASS(2, 2, 32)
