// Kernels of libnek instantiated for N + 1 = 10.
#include "nek_np.hpp"

NEK_DEFINE_NP_OPS(10)
