// Size class: d = 3, degree 3, n + m <= 56.
#include "weights_kernels.hpp"

RBF_WEIGHTS_CLASS(3, 3, 56)
