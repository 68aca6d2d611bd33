// Kernels of libnek instantiated for N + 1 = 16.
#include "nek_np.hpp"

NEK_DEFINE_NP_OPS(16)
