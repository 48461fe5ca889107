// Cell kernels of the 2-D degree-3 operator.
#include "ops_inst.hpp"
MFH_DEFINE_OPS(2, 3)
