// Operator and preconditioner applications with the FP32 operator copy on
// complex128 vectors (mixed solves): instances of matvec_launch (tp_matvec.h),
// one translation unit per element type so that the instances compile in
// parallel.
#include "tp_matvec.h"

namespace tp {

hipError_t matvec_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st) {
    return matvec_launch<float, c128, c128>(pl, x, y, R, st);
}
hipError_t matvec_fp32_wide_timed(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st,
                                  hipEvent_t *ev) {
    return matvec_launch<float, c128, c128>(pl, x, y, R, st, ev);
}
hipError_t precond_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R,
                             hipStream_t st) {
    return matvec_launch<float, c128, c128, true>(pl, x, y, R, st, nullptr, base);
}

}  // namespace tp
