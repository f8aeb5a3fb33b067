// Fused operator kernels of order p = 2 (one translation unit per order).
#include "apply_kernels.hpp"

MFHEX_DEFINE_ORDER(2)
