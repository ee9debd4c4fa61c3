// Declarations shared between the library's translation units.
#pragma once

#include <string>

#include "tp_common.h"

namespace tp {

// thread-local error message for toeplitz_last_error()
void set_error(const std::string &msg);
tp_status fail(tp_status s, const std::string &msg);
tp_status hip_fail(hipError_t e, const char *what);

// argument checks of an operator or preconditioner application (tp_capi.hip)
tp_status check_apply(tp_plan p, tp_prec which, const void *x, long ldx, const void *y, long ldy, int nrhs);
// TP_PATH_* bits of the launches an application takes at R columns
int path_flags(tp_plan pl, bool fp64, bool pre, int R);

// operator application (tp_matvec.h; instances in tp_apply_f64/f32/wide.hip)
hipError_t matvec_fp64(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st);
hipError_t matvec_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st);
// FP32 operator on complex128 vectors (inner solves of the mixed scheme)
hipError_t matvec_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st);
// the mixed solver's FP32 (x32 -> y32) and FP64 (x64 -> y64) operator instances
hipError_t matvec_mixed_both(tp_plan pl, Cols<const c128> x32, Cols<c128> y32, Cols<const c128> x64,
                             Cols<c128> y64, int R, hipStream_t st);
constexpr int kMatvecStages = 7;   // rim pass, x DFT, y DFT, product, inverse y, inverse x, rim finish
hipError_t matvec_fp64_timed(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st, hipEvent_t *ev);
hipError_t matvec_fp32_timed(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st, hipEvent_t *ev);
hipError_t matvec_fp32_wide_timed(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st,
                                  hipEvent_t *ev);
hipError_t spectrum_build(tp_plan pl, const c128 *gen_dev, c128 *tmp, hipStream_t st);
// block-circulant preconditioner: y = base + M^-1 x (base columns optional)
hipError_t precond_fp64(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R, hipStream_t st);
hipError_t precond_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, Cols<const c64> base, int R, hipStream_t st);
hipError_t precond_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R,
                             hipStream_t st);
bool precond_op_joined_ok(tp_plan pl, int *lg);
hipError_t precond_op_mixed(tp_plan pl, Cols<const c128> pin, Cols<c128> pout, Cols<const c128> pbase,
                            Cols<const c128> x32, Cols<c128> y32, Cols<const c128> x64, Cols<c128> y64, int R,
                            hipStream_t st);
// plan-time: invert every spectrum block in place (FP64, partial pivoting),
// scale by 1 / (Px Py)^2; *flag (device int) is set nonzero on a zero pivot
hipError_t precond_build(tp_plan pl, c128 *S, int *flag, hipStream_t st);
hipError_t dense_inverse(c128 *A, int n, int *flag, hipStream_t st);
hipError_t cast_to_c64(const c128 *in, c64 *out, long n, hipStream_t st);

// plan-time transform tables (tp_plan.cpp side of tp_capi.hip)
int choose_grid(int n);                     // smallest 2/3/5/7-smooth size >= 2n-1
int fft_factor(int P, int *radix, int *L);  // stage radices and sub-lengths; returns stage count
void fft_perm(int P, int nst, const int *radix, int *perm);

// rim slab width chosen for N columns
int rim_slab_width(long N);

// solver (tp_gmres.hip)
size_t solver_ws_bytes(long Nt, int restart, int max_rhs);
void solver_release(tp_plan pl);
void solver_drop_graphs(tp_plan pl);      // captured super-step graphs (they bake operator pointers)
tp_status solve_run(tp_plan pl, const c128 *v, long ldv, c128 *x, long ldx, int nrhs,
                    const tp_solve_opts &o, tp_solve_info *info, hipStream_t st);
long solver_max_nt();
tp_status batch_begin(tp_plan pl, const tp_solve_opts &o);
tp_status batch_admit(tp_plan pl, int slot, const c128 *v, c128 *x, double tol, int x0_given);
tp_status batch_release(tp_plan pl, int slot);
tp_status batch_step(tp_plan pl, int ngraphs);
tp_status batch_poll(tp_plan pl, int lag, int wait, int *phases, tp_solve_info *info);
tp_status batch_end(tp_plan pl);
hipStream_t solver_stream(tp_plan pl);
bool solver_batch_active(tp_plan pl);

// matrix-core kernels for many right-hand sides (tp_mfma.hip)
// FP32 product with the spectrum block in LDS (b <= 128; LDS prod_lds_bytes(b))
size_t prod_lds_bytes(int b);
hipError_t prod_lds(const c64 *G, const c64 *in, int b, int R, int Px, int Py, int kxh, c64 *out,
                    const void *const *act, hipStream_t st, int CG, int RT, bool pair);
template <typename T>
hipError_t prod_mfma(const cpx<T> *G, const cpx<T> *in, int b, int R, int Px, int Py, int kxh, cpx<T> *out,
                     const void *const *act, hipStream_t st, int cols);   // cols: columns per workgroup, 0 = default
template <typename T, typename In, typename Out>
hipError_t rim_mfma(const cpx<T> *B, const cpx<T> *BE, Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                    int nslab, cpx<T> *part, hipStream_t st);
template <typename T>
size_t rim_mfma_lds(bool nbe);

// post-steps (tp_post.hip)
size_t smatrix_work_bytes(int p);
tp_status port_smatrix(int p, const c128 *X, long ldx, const long *rows_h, const double *len_h, double Z0, c128 *S,
                       long lds, void *work, hipStream_t st);
tp_status far_field(int Nx, int Ny, int b, int Nr, double dx, double dy, const double *upos, const double *utan,
                    const double *rpos, const double *rtan, const c128 *I, long ldi, int nrhs, const double *dirs,
                    int nang, double k, double eta, c128 *F, hipStream_t st);

}  // namespace tp
