// Kernels of libnek instantiated for N + 1 = 8.
#include "nek_np.hpp"

NEK_DEFINE_NP_OPS(8)
