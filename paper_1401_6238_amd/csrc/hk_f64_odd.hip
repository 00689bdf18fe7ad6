// Row kernels for transform lengths 3 * 2^k and 5 * 2^k in double precision.
#define HK_REAL double
#define HK_NS ns_f64o
#define HK_SUFFIX f64
#include "hk_inst_odd.hpp"
