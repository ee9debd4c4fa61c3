// Operator and preconditioner applications with the FP32 operator copy on complex64 vectors: instances of
// matvec_launch (tp_matvec.h), one translation unit per element type so that
// the instances compile in parallel.
#include "tp_matvec.h"

namespace tp {

hipError_t matvec_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st) {
    return matvec_launch<float, c64, c64>(pl, x, y, R, st);
}
hipError_t matvec_fp32_timed(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st, hipEvent_t *ev) {
    return matvec_launch<float, c64, c64>(pl, x, y, R, st, ev);
}
hipError_t precond_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, Cols<const c64> base, int R, hipStream_t st) {
    return matvec_launch<float, c64, c64, true>(pl, x, y, R, st, nullptr, base);
}

}  // namespace tp
