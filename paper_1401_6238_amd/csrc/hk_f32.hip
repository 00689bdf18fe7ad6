// Kernels of the Hankel tensor-vector product in float precision (complex
// elements are pairs of float).
#define HK_REAL float
#define HK_NS ns_f32
#define HK_SUFFIX f32
#include "hk_inst.hpp"
