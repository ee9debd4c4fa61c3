// Schur-complement elimination of the rim.  With Z = [[A, B_er], [B, C]]
// (eq. matrixForm) the rim unknowns are eliminated through the rim rows'
// Schur complement S = C - B A^-1 B_er:
//   setup:  F = A^-1 B_er (Nr Toeplitz solves on the element operator A),
//           S = C - B F, S^-1 (one dense inverse);
//   solve:  w = A^-1 v_A,  x_r = S^-1 (v_r - B w),  x_A = w - F x_r.
// The Toeplitz solves run on a second plan of the same array without rim
// (the element operator alone), so the iterated operator is purely two-level
// block Toeplitz; B w is one FP64 pass over the dense block B.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tp_internal.h"

namespace tp {

static size_t al(size_t n) { return (n + 255) & ~(size_t)255; }

// B w for up to kSchurCols columns per launch: workgroup (s, t) sums row t
// of B against slab s of every column; the slab sums are added, in slab
// order, by their consumer.  part[(c * Nr + t) * kSchurSlabs + s].
constexpr int kSchurSlabs = 16;
constexpr int kSchurCols = 8;
__global__ void __launch_bounds__(256) k_schur_Bw(const c128 *__restrict__ B, long N, int Nr,
                                                  const c128 *__restrict__ w, long ldw, int ncols, int c0,
                                                  c128 *__restrict__ part) {
    __shared__ double red[2][kSchurCols][4];
    const int s = blockIdx.x, t = blockIdx.y;
    const long L = (N + kSchurSlabs - 1) / kSchurSlabs, e0 = (long)s * L, e1 = min(N, e0 + L);
    const int nc = min(kSchurCols, ncols - c0);
    c128 acc[kSchurCols];
#pragma unroll
    for (int c = 0; c < kSchurCols; ++c) acc[c] = c128{0, 0};
    const c128 *Bt = B + (long)t * N;
    for (long e = e0 + threadIdx.x; e < e1; e += kBlock) {
        const c128 bv = Bt[e];
#pragma unroll
        for (int c = 0; c < kSchurCols; ++c)
            if (c < nc) acc[c] = cmac(acc[c], bv, w[(long)(c0 + c) * ldw + e]);
    }
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kSchurCols; ++c) {
        if (c >= nc) break;
        const double re = wave_allsum(acc[c].x), im = wave_allsum(acc[c].y);
        if ((threadIdx.x & 63) == 0) {
            red[0][c][wv] = re;
            red[1][c][wv] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int c = threadIdx.x;
        const c128 v{((red[0][c][0] + red[0][c][1]) + red[0][c][2]) + red[0][c][3],
                     ((red[1][c][0] + red[1][c][1]) + red[1][c][2]) + red[1][c][3]};
        part[((long)(c0 + c) * Nr + t) * kSchurSlabs + s] = v;
    }
}

__device__ __forceinline__ c128 slab_sum(const c128 *__restrict__ part, long i) {
    c128 v = part[i * kSchurSlabs];
#pragma unroll
    for (int s = 1; s < kSchurSlabs; ++s) v = v + part[i * kSchurSlabs + s];
    return v;
}

static hipError_t launch_Bw(const c128 *B, long N, int Nr, const c128 *w, long ldw, int ncols, c128 *part,
                            hipStream_t st) {
    for (int c0 = 0; c0 < ncols; c0 += kSchurCols)
        hipLaunchKernelGGL(k_schur_Bw, dim3(kSchurSlabs, Nr), dim3(256), 0, st, B, N, Nr, w, ldw, ncols, c0, part);
    return hipGetLastError();
}

// S[i][r0 + c] = C[i][r0 + c] - (B F_c)[i]
__global__ void k_schur_S(const c128 *__restrict__ Cm, const c128 *__restrict__ part, int Nr, int r0,
                          c128 *__restrict__ S) {
    const int c = blockIdx.y, r = r0 + c;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Nr; i += gridDim.x * blockDim.x)
        S[(long)i * Nr + r] = Cm[(long)i * Nr + r] - slab_sum(part, (long)c * Nr + i);
}

// x_r = S^-1 (v_r - B w) for column blockIdx.x
__global__ void __launch_bounds__(256) k_schur_xr(const c128 *__restrict__ Sinv, const c128 *__restrict__ v, long ldv,
                                                  const c128 *__restrict__ part, long N, int Nr,
                                                  c128 *__restrict__ x, long ldx) {
    extern __shared__ char smem_raw[];
    c128 *g = reinterpret_cast<c128 *>(smem_raw);   // [Nr]
    const int r = blockIdx.x;
    for (int t = threadIdx.x; t < Nr; t += blockDim.x)
        g[t] = v[(long)r * ldv + N + t] - slab_sum(part, (long)r * Nr + t);
    __syncthreads();
    for (int i = threadIdx.x; i < Nr; i += blockDim.x) {
        c128 s = c128{0, 0};
        for (int t = 0; t < Nr; ++t) s = cmac(s, Sinv[(long)i * Nr + t], g[t]);
        x[(long)r * ldx + N + i] = s;
    }
}

// x_A -= F x_r (F stored [Nr][N]: column t of F contiguous over elements)
__global__ void __launch_bounds__(256) k_schur_xa(const c128 *__restrict__ F, long N, int Nr, c128 *__restrict__ x,
                                                  long ldx) {
    extern __shared__ char smem_raw[];
    c128 *xr = reinterpret_cast<c128 *>(smem_raw);   // [Nr]
    const int r = blockIdx.y;
    c128 *xc = x + (long)r * ldx;
    for (int t = threadIdx.x; t < Nr; t += blockDim.x) xr[t] = xc[N + t];
    __syncthreads();
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    c128 s = c128{0, 0};
    for (int t = 0; t < Nr; ++t) s = cmac(s, F[(long)t * N + e], xr[t]);
    xc[e] = xc[e] - s;
}

// red[r] = (||v_r - Y_r||^2, ||v_r||^2) for column blockIdx.x
__global__ void __launch_bounds__(1024) k_schur_norms(const c128 *__restrict__ v, long ldv, const c128 *__restrict__ Y,
                                                      long Nt, double *__restrict__ red) {
    __shared__ double part[2][16];
    const int r = blockIdx.x;
    double rr = 0, vv = 0;
    for (long e = threadIdx.x; e < Nt; e += blockDim.x) {
        const c128 a = v[(long)r * ldv + e], d = a - Y[(long)r * Nt + e];
        rr += d.x * d.x + d.y * d.y;
        vv += a.x * a.x + a.y * a.y;
    }
    rr = wave_allsum(rr);
    vv = wave_allsum(vv);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = rr;
        part[1][w] = vv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            a += part[0][i];
            b += part[1][i];
        }
        red[2 * r] = a;
        red[2 * r + 1] = b;
    }
}

struct SchurLayout {
    size_t F, Sinv, part, Y, red, flag, total;
};
static SchurLayout schur_layout(tp_plan p) {
    SchurLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += al(bytes);
        return o;
    };
    L.F = take((size_t)p->Nr * p->N * 16);
    L.Sinv = take((size_t)p->Nr * p->Nr * 16);
    L.part = take((size_t)p->max_rhs * p->Nr * kSchurSlabs * 16);
    L.Y = take((size_t)p->max_rhs * p->Nt * 16);
    L.red = take((size_t)p->max_rhs * 2 * 8);
    L.flag = take(sizeof(int));
    L.total = off;
    return L;
}

// A plan of the same array without rim: the element operator
static tp_status check_pair(tp_plan p, tp_plan a) {
    if (!p || !a) return fail(TP_E_INVAL, "plan is NULL");
    if (p->Nr < 1) return fail(TP_E_INVAL, "the plan has no rim to eliminate");
    if (p->nrc) return fail(TP_E_UNSUPPORTED, "the rim elimination needs the dense rim blocks (the plan holds a placed rim)");
    if (!p->G64 || !p->B64 || !p->C64) return fail(TP_E_UNSUPPORTED, "the rim elimination needs the FP64 operator");
    if (a->Nx != p->Nx || a->Ny != p->Ny || a->b != p->b || a->Nr != 0)
        return fail(TP_E_INVAL, "the element plan must have the same Nx, Ny, b and no rim");
    if (p->Nr > 2048) return fail(TP_E_INVAL, "Nr is limited to 2048");
    return TP_OK;
}

}  // namespace tp

using namespace tp;

extern "C" {

tp_status toeplitz_schur_bytes(tp_plan p, size_t *bytes) {
    if (!p || !bytes) return fail(TP_E_INVAL, "plan or bytes is NULL");
    if (p->Nr < 1) return fail(TP_E_INVAL, "the plan has no rim to eliminate");
    if (p->nrc) return fail(TP_E_UNSUPPORTED, "the rim elimination needs the dense rim blocks (the plan holds a placed rim)");
    *bytes = schur_layout(p).total;
    return TP_OK;
}

tp_status toeplitz_schur_create(tp_plan p, tp_plan a, void *dev_buf, size_t dev_bytes, const tp_solve_opts *opts,
                                void *hip_stream) {
    tp_status s = check_pair(p, a);
    if (s != TP_OK) return s;
    if (!dev_buf) return fail(TP_E_INVAL, "dev_buf is NULL");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0) return fail(TP_E_INVAL, "dev_buf must be 256-byte aligned");
    if (p->batch && solver_batch_active(p)) return fail(TP_E_INVAL, "a continuous batch is active on this plan");
    const SchurLayout L = schur_layout(p);
    if (dev_bytes < L.total) return fail(TP_E_NOMEM, "dev_buf smaller than toeplitz_schur_bytes()");
    char *base = static_cast<char *>(dev_buf);
    hipStream_t st = (hipStream_t)hip_stream;
    p->has_schur = 0;
    p->schurF = reinterpret_cast<c128 *>(base + L.F);
    p->schurSinv = reinterpret_cast<c128 *>(base + L.Sinv);
    p->schurPart = reinterpret_cast<c128 *>(base + L.part);
    p->schurY = reinterpret_cast<c128 *>(base + L.Y);
    p->schurRed = reinterpret_cast<double *>(base + L.red);
    p->schurFlag = reinterpret_cast<int *>(base + L.flag);
    const long N = p->N, Nt = p->Nt;
    const int Nr = p->Nr;
    // F = A^-1 B_er, a->max_rhs columns at a time (column r of B_er is row r
    // of the stored B_er^T, or of B when reciprocal)
    const c128 *Ber = p->BE64 ? p->BE64 : p->B64;
    tp_solve_opts o;
    toeplitz_solve_opts_default(&o);
    if (opts) o = *opts;
    o.x0_given = 0;
    std::vector<tp_solve_info> info(a->max_rhs);
    for (int r0 = 0; r0 < Nr; r0 += a->max_rhs) {
        const int R = std::min(a->max_rhs, Nr - r0);
        s = toeplitz_solve(a, Ber + (long)r0 * N, N, p->schurF + (long)r0 * N, N, R, &o, info.data(), hip_stream);
        if (s != TP_OK) return s == TP_E_NOCONV ? fail(s, "a solve with the element operator missed its tolerance") : s;
    }
    // S = C - B F, p->max_rhs columns at a time
    hipError_t e = hipSuccess;
    for (int r0 = 0; r0 < Nr && e == hipSuccess; r0 += p->max_rhs) {
        const int R = std::min(p->max_rhs, Nr - r0);
        if ((e = launch_Bw(p->B64, N, Nr, p->schurF + (long)r0 * N, N, R, p->schurPart, st))) break;
        hipLaunchKernelGGL(k_schur_S, dim3((unsigned)((Nr + 255) / 256), R), dim3(256), 0, st, p->C64, p->schurPart, Nr,
                           r0, p->schurSinv);
        e = hipGetLastError();
    }
    int hflag = 0;
    if (e || (e = hipMemsetAsync(p->schurFlag, 0, sizeof(int), st)) ||
        (e = dense_inverse(p->schurSinv, Nr, p->schurFlag, st)) ||
        (e = hipMemcpyAsync(&hflag, p->schurFlag, sizeof(int), hipMemcpyDeviceToHost, st)) ||
        (e = hipStreamSynchronize(st)))
        return hip_fail(e, "rim elimination setup");
    if (hflag) return fail(TP_E_BREAKDOWN, "the rim Schur complement C - B A^-1 B_er is singular");
    p->has_schur = 1;
    return TP_OK;
}

tp_status toeplitz_schur_solve(tp_plan p, tp_plan a, const void *v, long ldv, void *x, long ldx, int nrhs,
                               const tp_solve_opts *opts, tp_solve_info *info, void *hip_stream) {
    tp_status s = check_pair(p, a);
    if (s != TP_OK) return s;
    if (!p->has_schur) return fail(TP_E_INVAL, "the plan has no rim elimination (toeplitz_schur_create)");
    if (!v || !x || !info) return fail(TP_E_INVAL, "v, x or info is NULL");
    if ((p->batch && solver_batch_active(p)) || (a->batch && solver_batch_active(a)))
        return fail(TP_E_INVAL, "a continuous batch is active on one of the plans");
    if (nrhs < 1 || nrhs > p->max_rhs || nrhs > a->max_rhs)
        return fail(TP_E_INVAL, "nrhs must be in [1, max_rhs] of both plans");
    if (ldv < p->Nt || ldx < p->Nt) return fail(TP_E_INVAL, "leading dimension smaller than Nt");
    const char *va = (const char *)v, *xa = (const char *)x;
    const size_t vb = ((size_t)ldv * (nrhs - 1) + p->Nt) * 16, xb = ((size_t)ldx * (nrhs - 1) + p->Nt) * 16;
    if (va < xa + xb && xa < va + vb) return fail(TP_E_INVAL, "v and x overlap");
    tp_solve_opts o;
    toeplitz_solve_opts_default(&o);
    if (opts) o = *opts;
    const double tol = o.tol;
    // With F and S^-1 exact, the full residual is [A w - v_A; 0], so an
    // element solve to tol (relative to ||v_A|| <= ||v||) meets the target;
    // the factor 1/2 leaves room for the rounding in F and S^-1.
    o.tol = 0.5 * tol;
    o.x0_given = 0;
    hipStream_t st = (hipStream_t)hip_stream;
    const long N = p->N, Nt = p->Nt;
    const int Nr = p->Nr;
    const c128 *vc = (const c128 *)v;
    c128 *xc = (c128 *)x;
    // w = A^-1 v_A into x_A
    std::vector<tp_solve_info> ia(nrhs);
    s = toeplitz_solve(a, v, ldv, x, ldx, nrhs, &o, ia.data(), hip_stream);
    if (s != TP_OK && s != TP_E_NOCONV) return s;
    hipError_t e;
    // x_r = S^-1 (v_r - B w), x_A = w - F x_r
    if ((e = launch_Bw(p->B64, N, Nr, xc, ldx, nrhs, p->schurPart, st))) return hip_fail(e, "rim elimination solve");
    hipLaunchKernelGGL(k_schur_xr, dim3(nrhs), dim3(256), (size_t)Nr * sizeof(c128), st, p->schurSinv, vc, ldv,
                       p->schurPart, N, Nr, xc, ldx);
    hipLaunchKernelGGL(k_schur_xa, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), (size_t)Nr * sizeof(c128), st,
                       p->schurF, N, Nr, xc, ldx);
    // the true residual of the full system
    if ((e = hipGetLastError()) ||
        (e = matvec_fp64(p, Cols<const c128>{xc, ldx, nullptr}, Cols<c128>{p->schurY, Nt, nullptr}, nrhs, st)))
        return hip_fail(e, "rim elimination residual");
    hipLaunchKernelGGL(k_schur_norms, dim3(nrhs), dim3(1024), 0, st, vc, ldv, p->schurY, Nt, p->schurRed);
    std::vector<double> red(2 * (size_t)nrhs);
    if ((e = hipGetLastError()) ||
        (e = hipMemcpyAsync(red.data(), p->schurRed, red.size() * sizeof(double), hipMemcpyDeviceToHost, st)) ||
        (e = hipStreamSynchronize(st)))
        return hip_fail(e, "rim elimination residual");
    tp_status ret = TP_OK;
    for (int r = 0; r < nrhs; ++r) {
        const double rr = sqrt(red[2 * r]), vn = sqrt(red[2 * r + 1]);
        info[r].iters = ia[r].iters;
        info[r].outer_iters = ia[r].outer_iters;
        info[r].relres = vn > 0 ? rr / vn : (rr > 0 ? INFINITY : 0.0);
        info[r].status = info[r].relres <= tol ? TP_OK : TP_E_NOCONV;
        if (info[r].status != TP_OK) ret = TP_E_NOCONV;
    }
    if (ret != TP_OK) set_error("at least one column missed the tolerance");
    return ret;
}

}  // extern "C"
