// complex128 instantiation of the MFMA block solves.
#include "solve_kernel.h"

namespace fb {
template int launch_variant<double>(int, const c128*, const c128*, const int16_t*, int64_t, int,
                                    int, const SolveJob*, hipStream_t, const int32_t*);
}  // namespace fb
