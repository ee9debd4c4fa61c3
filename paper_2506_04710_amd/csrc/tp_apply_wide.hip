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

// One column of a preconditioned mixed solve, where the preconditioner's
// output is the operator's input: the preconditioner's last pass (inverse x
// transforms and crop, adding the base column) and the operator's first pass
// (embedding and forward x transforms) in one launch.  Workgroup = one row of
// cells and one chunk of channels in both passes: it writes the
// preconditioner's output for exactly the elements that it then reads back
// (after a barrier) as the operator's input, for the FP32
// instance (Arnoldi steps: v_j -> W -> Z W) or the FP64 one (residual steps:
// x += M^-1 u, then Z x); the idle instance's pass exits at once.  The same
// arithmetic on the same values as the two separate launches.
__global__ void __launch_bounds__(256) k_pre_inv_x_op_fwd_x(const c64 *pin, int Nx, int b, FFTDesc fx, int lg,
                                                            int nchunk, Cols<c128> py, Cols<const c128> pbase,
                                                            long N, int Nr, Cols<const c128> x32,
                                                            Cols<const c128> x64, c64 *o32, c128 *o64, RimMap rm) {
    extern __shared__ char smem_raw[];
    const int blk = blockIdx.x, iy = blk / nchunk, ch = blk - iy * nchunk;
    const Cols<const c128> nox{nullptr, 0, nullptr};
    inv_x_fin_body<float, c128, c128>(pin, 1, Nx, b, fx, lg, nchunk, py, 1, pbase, (int)gridDim.x, nullptr, nullptr,
                                      nullptr, nox, N, Nr, 0, MirrorParts<float>{nullptr, fx.P, 0, 0, 0}, rm, blk,
                                      smem_raw);
    // the barrier orders the workgroup's global stores before its loads
    // (workgroup scope; its waves share one compute unit's vector cache)
    __syncthreads();
    fwd_x_body<float, c128>(x32, 1, Nx, b, fx, lg, o32, rm, ch, iy, smem_raw);
    __syncthreads();
    fwd_x_body<double, c128>(x64, 1, Nx, b, fx, lg, o64, rm, ch, iy, smem_raw);
}

// Preconditioner (FP32, out = base + M^-1 in) followed by both operator
// instances of a mixed solve on one column, with the joined pass above where
// the preconditioner and the operator take the pair-stream path with separate
// x and y passes (no dense rim pass) and the same channel chunks; otherwise
// returns false and launches nothing.
// Whether the joined pass applies to the plan as its options stand (one
// column); *lg receives the channel chunk of both passes.
bool precond_op_joined_ok(tp_plan pl, int *lg) {
    const int R = 1;
    if (!pl->opt_dual_launch || !pl->gridA32 || !pl->G32 || !pl->G64 || !pl->S32 || !pl->has_precond)
        return false;
    if (pl->Nr > 0 && pl->nrc == 0) return false;            // a dense rim: rows finished apart
    const Path pp = choose_path<float, true>(pl, R);
    const Path p32 = choose_path<float, false>(pl, R), p64 = choose_path<double, false>(pl, R);
    // (these include the conditions of the shared launches on one column)
    if (!pp.pairs || pp.lg2 >= 0 || !p32.pairs || !p64.pairs || p32.rim || p64.rim || p32.lg2 >= 0 ||
        p64.lg2 >= 0)
        return false;
    const int C = pl->bc, l = fft_lgcc(pl->Px, C, 8, fftx_maxcc(C, pl->Ny));
    if (fft_lgcc(pl->Px, C, 16, fftx_maxcc(C, pl->Ny)) != l) return false;
    *lg = l;
    return true;
}

static bool precond_op_mixed_launch(tp_plan pl, Cols<const c128> pin, Cols<c128> pout, Cols<const c128> pbase,
                                    Cols<const c128> x32, Cols<c128> y32, Cols<const c128> x64, Cols<c128> y64,
                                    hipStream_t st) {
    const int R = 1;
    int lg = 0;
    if (pl->only_stage >= 0 || !precond_op_joined_ok(pl, &lg)) return false;   // nothing launched
    const int Nx = pl->Nx, Ny = pl->Ny, b = pl->bc, Px = pl->Px, C = b;
    // the preconditioner's transforms and product, up to its inverse y pass
    // (launch errors surface through hipGetLastError in the caller)
    matvec_launch<float, c128, c128, true>(pl, pin, pout, R, st, nullptr, pbase, 4);
    const int nchunk = (C + (1 << lg) - 1) >> lg;
    const size_t sh = ((size_t)Px * (1 << lg) + Px) * 16;
    const RimMap rm{pl->rim_map, pl->b, pl->nrc, pl->N};
    hipLaunchKernelGGL(k_pre_inv_x_op_fwd_x, dim3(nchunk * Ny), dim3(256), sh, st,
                       reinterpret_cast<const c64 *>(pl->gridB), Nx, b, pl->fx, lg, nchunk, pout, pbase, pl->N,
                       pl->Nr, x32, x64, reinterpret_cast<c64 *>(pl->gridA32), reinterpret_cast<c128 *>(pl->gridA),
                       rm);
    // the operator's remaining stages (the checks above are those of the
    // shared launches on one column, so they apply)
    matvec_dual_launch<c128, c128>(pl, x32, y32, x64, y64, R, st, true);
    return true;
}

hipError_t precond_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R,
                             hipStream_t st) {
    return matvec_launch<float, c128, c128, true>(pl, x, y, R, st, nullptr, base);
}

// The mixed solver's preconditioner and operator applications of one
// super-step: the joined pass where it applies (one column), else the
// preconditioner and then both operator instances.
hipError_t precond_op_mixed(tp_plan pl, Cols<const c128> pin, Cols<c128> pout, Cols<const c128> pbase,
                            Cols<const c128> x32, Cols<c128> y32, Cols<const c128> x64, Cols<c128> y64, int R,
                            hipStream_t st) {
    if (R == 1 && precond_op_mixed_launch(pl, pin, pout, pbase, x32, y32, x64, y64, st))
        return hipGetLastError();
    hipError_t e = precond_fp32_wide(pl, pin, pout, pbase, R, st);
    if (e) return e;
    return matvec_mixed_both(pl, x32, y32, x64, y64, R, st);
}


}  // namespace tp
