// complex64 instantiation of the MFMA block solves.
#include "solve_kernel.h"

namespace fb {
template int launch_variant<float>(int, const c64*, const c64*, const int16_t*, int64_t, int,
                                   int, const SolveJob*, hipStream_t, const int32_t*);
}  // namespace fb
