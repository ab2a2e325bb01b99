// Fused residual / JVP / Newton-operator / block-column kernels for order p = 4.
#include "fr_fused.hpp"

FR_FUSED_INSTANTIATE(4)
