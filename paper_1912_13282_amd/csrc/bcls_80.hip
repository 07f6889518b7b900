// Batched persistent form, size class n + m <= 80 (any dimension and degree).
#include "batched_kernels.hpp"

RBF_BATCHED_CLASS(80)
