// Cell kernels of the 3-D degree-2 operator.
#include "ops_inst.hpp"
MFH_DEFINE_OPS(3, 2)
