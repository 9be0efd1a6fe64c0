// Three-dimensional weights, m = 4, supports 35 <= n <= 76 (identity padding
// to K = 111): the Laplacian.
#include "weights3_k105.h"
RBFFD_W3_M4_ANY_INSTANCE(0)
