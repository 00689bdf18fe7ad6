// Kernels of the Hankel tensor-vector product in double precision (complex
// elements are pairs of double).
#define HK_REAL double
#define HK_NS ns_f64
#define HK_SUFFIX f64
#include "hk_inst.hpp"
