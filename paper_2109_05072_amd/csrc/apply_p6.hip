// Fused operator kernels of order p = 6 (one translation unit per order).
#include "apply_kernels.hpp"

MFHEX_DEFINE_ORDER(6)
