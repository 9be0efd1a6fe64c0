// Three-dimensional weights, m = 4, n = 70: d/dz.
#include "weights3_k105.h"
RBFFD_W3_K105_INSTANCE(3)
