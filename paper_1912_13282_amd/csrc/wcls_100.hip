// Size class: systems of n + m <= 100 unknowns (any dimension and degree).
#include "weights_kernels.hpp"

RBF_WEIGHTS_CLASS(100)
