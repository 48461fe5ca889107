// Cell kernels of the 2-D degree-4 operator.
#include "ops_inst.hpp"
MFH_DEFINE_OPS(2, 4)
