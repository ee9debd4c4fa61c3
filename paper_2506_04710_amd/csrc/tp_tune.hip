// Autotuner: times the launch options that change a kernel of this plan at a
// given column count and keeps the fastest.  The candidates are kernel
// variants with the same results; the timed work is what a solve applies (the
// operator and, when the plan has one, the preconditioner).
#include <vector>

#include "tp_internal.h"

namespace tp {

#ifndef TP_MFMA_MIN_R
#define TP_MFMA_MIN_R 16
#endif

// One application of the timed work (operator, then preconditioner).
static hipError_t tune_apply(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int R,
                             hipStream_t st) {
    hipError_t e;
    if (which == TP_FP64) {
        const Cols<const c128> xc{(const c128 *)x, ldx, nullptr};
        const Cols<c128> yc{(c128 *)y, ldy, nullptr};
        if ((e = matvec_fp64(p, xc, yc, R, st))) return e;
        if (p->has_precond && p->S64) return precond_fp64(p, xc, yc, Cols<const c128>{nullptr, 0, nullptr}, R, st);
    } else if (which == TP_FP32) {
        const Cols<const c64> xc{(const c64 *)x, ldx, nullptr};
        const Cols<c64> yc{(c64 *)y, ldy, nullptr};
        if ((e = matvec_fp32(p, xc, yc, R, st))) return e;
        if (p->has_precond && p->S32) return precond_fp32(p, xc, yc, Cols<const c64>{nullptr, 0, nullptr}, R, st);
    } else {
        const Cols<const c128> xc{(const c128 *)x, ldx, nullptr};
        const Cols<c128> yc{(c128 *)y, ldy, nullptr};
        if ((e = matvec_fp32_wide(p, xc, yc, R, st))) return e;
        if (p->has_precond && p->S32)
            return precond_fp32_wide(p, xc, yc, Cols<const c128>{nullptr, 0, nullptr}, R, st);
    }
    return hipSuccess;
}

}  // namespace tp

using namespace tp;

extern "C" {

tp_status toeplitz_tune(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs, int reps,
                        void *hip_stream, tp_tune_result *res) {
    if (!res || reps < 1) return fail(TP_E_INVAL, "result is NULL or reps < 1");
    tp_status s = check_apply(p, which, x, ldx, y, ldy, nrhs);
    if (s != TP_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    // options that change a kernel here
    const bool pass_matters = nrhs == 1 && p->half && p->bc <= 128 && (p->nrc > 0 || p->has_precond);
    const int min_r = p->opt_mfma_min_r ? p->opt_mfma_min_r : TP_MFMA_MIN_R;
    const bool mfma_matters = nrhs >= min_r;
    std::vector<int> passes = pass_matters ? std::vector<int>{TP_PASS_FUSED, TP_PASS_PAIRS}
                                           : std::vector<int>{p->opt_spectrum_pass};
    std::vector<int> cols = mfma_matters ? (which == TP_FP64 ? std::vector<int>{16, 32} : std::vector<int>{16, 32, 64})
                                         : std::vector<int>{p->opt_mfma_cols};
    // the 2-D tiles: only where a 160 KB tile of 4 channels of the timed
    // operator's values holds the grid and a 48 KB one does not
    const size_t es = which == TP_FP64 ? 16 : 8;
    const size_t tile4 = ((size_t)p->Px * (p->Py * 4 + 16) + p->Px + p->Py) * es + (size_t)(p->Px + p->Py) * 4;
    const bool fft2_matters = tile4 > 48 * 1024 && tile4 <= 160 * 1024;
    std::vector<int> tiles = fft2_matters ? std::vector<int>{0, 160 * 1024} : std::vector<int>{p->opt_fft2_lds};
    // the persistent launch: timed where a combination takes it (it applies
    // at the default column tile only)
    const int def_cols = which == TP_FP64 ? 16 : 32;
    // the FP32 product with the block in LDS: column-group and row-tile shapes
    // whose workgroup fits (it replaces the column tile and the persistent launch)
    std::vector<int> plds{0};
    if (mfma_matters && which != TP_FP64 && p->bc <= 128) {
        const int nrt = (p->bc + 15) / 16;
        for (int pr : {0, 256})
            for (int cg : {2, 3, 6})
                for (int rt : {2, 3, 6})
                    if (cg * ((nrt + rt - 1) / rt) <= 16 && (pr == 0 || p->half)) plds.push_back(pr + cg * 16 + rt);
    }
    auto persistent = [&]() {
        const bool f64 = which == TP_FP64;
        return (path_flags(p, f64, false, nrhs) & TP_PATH_PERSISTENT) ||
               (p->has_precond && (path_flags(p, f64, true, nrhs) & TP_PATH_PERSISTENT));
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(TP_E_HIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(TP_E_HIP, "event create");
    }
    hipError_t e = hipSuccess;
    auto time_it = [&](double &ms) {
        for (int w = 0; w < 2 && e == hipSuccess; ++w) e = tune_apply(p, which, x, ldx, y, ldy, nrhs, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = tune_apply(p, which, x, ldx, y, ldy, nrhs, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        ms = (double)f / reps;
    };
    const int keep_pass = p->opt_spectrum_pass, keep_cols = p->opt_mfma_cols, keep_tile = p->opt_fft2_lds,
              keep_multi = p->opt_multi_fused, keep_plds = p->opt_prod_lds, keep_ro = p->opt_rim_overlap;
    // every option at its default first
    p->opt_spectrum_pass = TP_PASS_AUTO;
    p->opt_mfma_cols = 0;
    p->opt_fft2_lds = 0;
    p->opt_multi_fused = 0;
    p->opt_prod_lds = 0;
    p->opt_rim_overlap = 1;
    double ms_def = 0.0;
    time_it(ms_def);
    double best = -1.0;
    int bp = keep_pass, bc = keep_cols, bt = keep_tile, bm = keep_multi, bl = keep_plds, bro = keep_ro, n = 0;
    // the rim and the forward tiles in one launch or two: timed both ways where it applies
    auto overlap = [&]() {
        const bool f64 = which == TP_FP64;
        return (path_flags(p, f64, false, nrhs) & TP_PATH_RIM_OVERLAP) != 0;
    };
    bool multi_seen = false;
    for (int pv : passes)
        for (int cv : cols)
            for (int tv : tiles)
                for (int mv = 0; mv < 2; ++mv)
                    for (int lv : plds)
                        for (int ro = 1; ro >= 0; --ro) {
                            if (e != hipSuccess) break;
                            p->opt_spectrum_pass = pv;
                            p->opt_mfma_cols = cv;
                            p->opt_fft2_lds = tv;
                            p->opt_multi_fused = mv;
                            p->opt_prod_lds = lv;
                            p->opt_rim_overlap = 1;
                            if (mv == 1 && (cv != def_cols || lv != 0 || !persistent())) continue;
                            if (lv != 0 && cv != def_cols) continue;
                            if (ro == 0 && !overlap()) continue;   // the setting changes nothing here
                            p->opt_rim_overlap = ro;
                            multi_seen |= mv == 1;
                            double ms = 0.0;
                            time_it(ms);
                            ++n;
                            if (e == hipSuccess && (best < 0.0 || ms < best)) {
                                best = ms;
                                bp = pv;
                                bc = cv;
                                bt = tv;
                                bm = mv;
                                bl = lv;
                                bro = ro;
                            }
                        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    solver_drop_graphs(p);      // captured graphs hold the launch shapes
    if (e != hipSuccess) {
        p->opt_spectrum_pass = keep_pass;
        p->opt_mfma_cols = keep_cols;
        p->opt_fft2_lds = keep_tile;
        p->opt_multi_fused = keep_multi;
        p->opt_prod_lds = keep_plds;
        p->opt_rim_overlap = keep_ro;
        return hip_fail(e, "tune");
    }
    p->opt_spectrum_pass = bp;
    p->opt_mfma_cols = bc;
    p->opt_fft2_lds = bt;
    p->opt_multi_fused = bm;
    p->opt_prod_lds = bl;
    p->opt_rim_overlap = bro;
    res->spectrum_pass = pass_matters ? bp : TP_PASS_AUTO;
    res->mfma_cols = mfma_matters ? bc : 0;
    res->fft2_lds = fft2_matters ? bt : 0;
    res->multi_fused = multi_seen ? bm : 0;
    res->prod_lds = bl;
    res->rim_overlap = bro;
    res->candidates = n;
    res->ms = best;
    res->ms_default = ms_def;
    return TP_OK;
}

}  // extern "C"
