// Row kernels for transform lengths 3 * 2^k and 5 * 2^k in float precision.
#define HK_REAL float
#define HK_NS ns_f32o
#define HK_SUFFIX f32
#include "hk_inst_odd.hpp"
