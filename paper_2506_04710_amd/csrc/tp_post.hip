// Post-steps on solved currents: port scattering matrix (Sec. III-B) and the
// far field by per-part contraction (eqs. farfieldBasis, tensorProd).
#include "tp_internal.h"

namespace tp {

__device__ __forceinline__ c128 cdiv(c128 a, c128 b) {
    const double d = 1.0 / (b.x * b.x + b.y * b.y);
    return c128{(a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d};
}

// ----------------------------------------------------------- S-matrix
// One workgroup.  W is the augmented p x 2p system [I + Z0 Y | I - Z0 Y],
// row-major in global memory (L2-resident at these sizes); the waves of the
// workgroup share the CU's vector cache, so a barrier orders their accesses.
// Elimination with partial pivoting (largest modulus, ties to the lower row)
// reduces the left half to U; back substitution then solves U S = (right
// half), one column of S per thread.
__global__ void __launch_bounds__(1024) k_smatrix(int p, const c128 *__restrict__ X, long ldx,
                                                  const long *__restrict__ rows, const double *__restrict__ len,
                                                  int use_len, double Z0, c128 *__restrict__ W, c128 *__restrict__ S,
                                                  long lds, int *flag) {
    __shared__ int piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    const long w2 = 2L * p;
    for (long idx = tid; idx < (long)p * p; idx += nt) {
        const int i = (int)(idx / p), j = (int)(idx - (long)i * p);
        c128 y = X[rows[i] + (long)j * ldx];
        if (use_len) y = scale(y, 1.0 / (len[i] * len[j]));
        const double d = i == j ? 1.0 : 0.0;
        W[i * w2 + j] = c128{d + Z0 * y.x, Z0 * y.y};
        W[i * w2 + p + j] = c128{d - Z0 * y.x, -Z0 * y.y};
    }
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int k = 0; k < p; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < p; i += 64) {
                const c128 a = W[i * w2 + k];
                const double m = a.x * a.x + a.y * a.y;
                if (m > best) {
                    best = m;
                    bi = i;
                }
            }
            for (int o = 32; o >= 1; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (tid == 0) {
                piv = bi;
                if (!(best > 0.0) || !(best < INFINITY)) *flag = 1;
            }
        }
        __syncthreads();
        const int r = piv;
        if (r != k) {
            for (long j = k + tid; j < w2; j += nt) {
                const c128 t = W[k * w2 + j];
                W[k * w2 + j] = W[r * w2 + j];
                W[r * w2 + j] = t;
            }
            __syncthreads();
        }
        const c128 inv = cdiv(c128{1.0, 0.0}, W[k * w2 + k]);
        const long ncol = w2 - k - 1, nrow = p - k - 1;
        for (long idx = tid; idx < nrow * ncol; idx += nt) {
            const long i = k + 1 + idx / ncol, j = k + 1 + idx % ncol;
            const c128 l = W[i * w2 + k] * inv;
            W[i * w2 + j] = W[i * w2 + j] - l * W[k * w2 + j];
        }
        __syncthreads();
    }
    for (int c = tid; c < p; c += nt) {
        for (int i = p - 1; i >= 0; --i) {
            c128 acc = W[i * w2 + p + c];
            for (int j = i + 1; j < p; ++j) acc = acc - W[i * w2 + j] * W[j * w2 + p + c];
            acc = cdiv(acc, W[i * w2 + i]);
            W[i * w2 + p + c] = acc;
            S[i + (long)c * lds] = acc;
        }
    }
}

size_t smatrix_work_bytes(int p) { return 32 * (size_t)p * p + 16 * (size_t)p + 256; }

tp_status port_smatrix(int p, const c128 *X, long ldx, const long *rows_h, const double *len_h, double Z0, c128 *S,
                       long lds, void *work, hipStream_t st) {
    char *wb = static_cast<char *>(work);
    c128 *W = reinterpret_cast<c128 *>(wb);
    long *rows = reinterpret_cast<long *>(wb + 32 * (size_t)p * p);
    double *len = reinterpret_cast<double *>(rows + p);
    int *flag = reinterpret_cast<int *>(len + p);
    hipError_t e;
    if ((e = hipMemcpyAsync(rows, rows_h, sizeof(long) * p, hipMemcpyHostToDevice, st))) return hip_fail(e, "S-matrix rows");
    if (len_h && (e = hipMemcpyAsync(len, len_h, sizeof(double) * p, hipMemcpyHostToDevice, st)))
        return hip_fail(e, "S-matrix edge lengths");
    hipLaunchKernelGGL(k_smatrix, dim3(1), dim3(1024), 0, st, p, X, ldx, rows, len, len_h ? 1 : 0, Z0, W, S, lds,
                       flag);
    if ((e = hipGetLastError())) return hip_fail(e, "S-matrix kernel");
    int hflag = 0;
    if ((e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st)) || (e = hipStreamSynchronize(st)))
        return hip_fail(e, "S-matrix status");
    if (hflag) return fail(TP_E_BREAKDOWN, "I + Z0 Y is singular (zero pivot)");
    return TP_OK;
}

// ----------------------------------------------------------- far field
// Workgroup = one direction m and one current vector.  The element pattern
// (e_tau . t_n) exp(j k rhat . u_n) of every basis n is formed once in LDS
// (eq. farfieldBasis), together with the separable part phases
// exp(j k rhat_x ix dx) and exp(j k rhat_y iy dy); every thread then sums
// phase(part) * I * pattern over a strided share of the element unknowns
// (eq. tensorProd), adds the rim functions directly, and the workgroup reduces.
__global__ void __launch_bounds__(256) k_far_field(int Nx, int Ny, int b, int Nr, double dx, double dy,
                                                   const double *__restrict__ upos, const double *__restrict__ utan,
                                                   const double *__restrict__ rpos, const double *__restrict__ rtan,
                                                   const c128 *__restrict__ I, long ldi,
                                                   const double *__restrict__ dirs, int nang, double k, double eta,
                                                   c128 *__restrict__ F) {
    extern __shared__ char smem_raw[];
    c128 *pat = reinterpret_cast<c128 *>(smem_raw);   // [2][b]
    c128 *px = pat + 2 * b;                            // [Nx]
    c128 *py = px + Nx;                                // [Ny]
    __shared__ c128 red[2][4];
    const int m = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
    double st, ct, sp, cp;
    sincos(dirs[2 * m], &st, &ct);
    sincos(dirs[2 * m + 1], &sp, &cp);
    const double rx = st * cp, ry = st * sp, rz = ct;
    const double etx = ct * cp, ety = ct * sp, etz = -st;
    const double epx = -sp, epy = cp;
    for (int n = tid; n < b; n += blockDim.x) {
        double s, c;
        sincos(k * (rx * upos[3 * n] + ry * upos[3 * n + 1] + rz * upos[3 * n + 2]), &s, &c);
        const double tt = etx * utan[3 * n] + ety * utan[3 * n + 1] + etz * utan[3 * n + 2];
        const double tp = epx * utan[3 * n] + epy * utan[3 * n + 1];
        pat[n] = c128{tt * c, tt * s};
        pat[b + n] = c128{tp * c, tp * s};
    }
    for (int i = tid; i < Nx; i += blockDim.x) {
        double s, c;
        sincos(k * rx * (i * dx), &s, &c);
        px[i] = c128{c, s};
    }
    for (int i = tid; i < Ny; i += blockDim.x) {
        double s, c;
        sincos(k * ry * (i * dy), &s, &c);
        py[i] = c128{c, s};
    }
    __syncthreads();
    const c128 *Ir = I + (long)r * ldi;
    const long N = (long)Nx * Ny * b;
    c128 a0{0, 0}, a1{0, 0};
    for (long i = tid; i < N; i += blockDim.x) {
        const long e = i / b;
        const int n = (int)(i - e * b);
        const int iy = (int)(e / Nx), ix = (int)(e - (long)iy * Nx);
        const c128 t = Ir[i] * (px[ix] * py[iy]);
        a0 = cmac(a0, t, pat[n]);
        a1 = cmac(a1, t, pat[b + n]);
    }
    for (int q = tid; q < Nr; q += blockDim.x) {
        double s, c;
        sincos(k * (rx * rpos[3 * q] + ry * rpos[3 * q + 1] + rz * rpos[3 * q + 2]), &s, &c);
        const double tt = etx * rtan[3 * q] + ety * rtan[3 * q + 1] + etz * rtan[3 * q + 2];
        const double tp = epx * rtan[3 * q] + epy * rtan[3 * q + 1];
        const c128 t = Ir[N + q] * c128{c, s};
        a0 = a0 + scale(t, tt);
        a1 = a1 + scale(t, tp);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        a0 = a0 + c128{__shfl_xor(a0.x, o, 64), __shfl_xor(a0.y, o, 64)};
        a1 = a1 + c128{__shfl_xor(a1.x, o, 64), __shfl_xor(a1.y, o, 64)};
    }
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        red[0][w] = a0;
        red[1][w] = a1;
    }
    __syncthreads();
    if (tid < 2) {
        c128 s{0, 0};
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = s + red[tid][i];
        // -j k eta s
        F[((long)r * nang + m) * 2 + tid] = c128{k * eta * s.y, -k * eta * s.x};
    }
}

tp_status far_field(int Nx, int Ny, int b, int Nr, double dx, double dy, const double *upos, const double *utan,
                    const double *rpos, const double *rtan, const c128 *I, long ldi, int nrhs, const double *dirs,
                    int nang, double k, double eta, c128 *F, hipStream_t st) {
    const size_t sh = sizeof(c128) * (2 * (size_t)b + Nx + Ny);
    hipLaunchKernelGGL(k_far_field, dim3(nang, nrhs), dim3(256), sh, st, Nx, Ny, b, Nr, dx, dy, upos, utan, rpos,
                       rtan, I, ldi, dirs, nang, k, eta, F);
    hipError_t e = hipGetLastError();
    if (e) return hip_fail(e, "far-field kernel");
    return TP_OK;
}

}  // namespace tp
