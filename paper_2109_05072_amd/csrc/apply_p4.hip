// Fused operator kernels of order p = 4 (one translation unit per order).
#include "apply_kernels.hpp"

MFHEX_DEFINE_ORDER(4)
