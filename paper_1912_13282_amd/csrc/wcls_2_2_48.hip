// Size class: d = 2, degree 2, n + m <= 48.
#include "weights_kernels.hpp"

RBF_WEIGHTS_CLASS(2, 2, 48)
