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
// The mixed solver's two operator instances (FP32 on x32 -> y32, FP64 on
// x64 -> y64, complex128 vectors): one launch per stage for both where the
// path allows it, else the two applications in turn.
hipError_t matvec_mixed_both(tp_plan pl, Cols<const c128> x32, Cols<c128> y32, Cols<const c128> x64,
                             Cols<c128> y64, int R, hipStream_t st) {
    if (pl->opt_dual_launch && matvec_dual_launch<c128, c128>(pl, x32, y32, x64, y64, R, st))
        return hipGetLastError();
    hipError_t e = matvec_launch<float, c128, c128>(pl, x32, y32, R, st);
    if (e) return e;
    return matvec_launch<double, c128, c128>(pl, x64, y64, R, st);
}

hipError_t precond_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R,
                             hipStream_t st) {
    return matvec_launch<float, c128, c128, true>(pl, x, y, R, st, nullptr, base);
}

}  // namespace tp
