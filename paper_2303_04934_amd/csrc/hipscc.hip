// Single translation unit of the hipscc library: kernels (kernels.h, bag.h,
// policy.h) and the host runtime behind the C ABI (runtime.hip).
#include "runtime.hip"
