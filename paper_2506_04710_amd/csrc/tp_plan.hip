// Plan-time kernels: the generator spectrum (circulant placement and 2-D
// DFT) and the block-circulant preconditioner (per-frequency inverses).
#include "tp_matvec.h"

namespace tp {

// ------------------------------------------------------ plan-time spectrum
// x pass over the generator rows: Z_{m,n} for m in (-Nx, Nx) sits at grid
// column m mod Px; the other columns are zero.
__global__ void __launch_bounds__(256) k_gen_fwd_x(const c128 *__restrict__ gen, int Nx, long bb, FFTDesc fx,
                                                   int lgCC, c128 *__restrict__ out) {
    extern __shared__ char smem_raw[];
    c128 *twl = reinterpret_cast<c128 *>(smem_raw);
    c128 *buf = twl + fx.P;
    const int CC = 1 << lgCC, P = fx.P, W = 2 * Nx - 1;
    const long c0 = (long)blockIdx.x * CC;
    const int ni = blockIdx.y;
    load_twiddles<double>(twl, fx);
    zero_lds<double>(buf, P * CC);
    __syncthreads();
    for (int i = threadIdx.x; i < W * CC; i += kBlock) {
        const int mi = i >> lgCC, cl = i & (CC - 1);
        const long c = c0 + cl;
        if (c < bb) {
            int g = mi - (Nx - 1);
            if (g < 0) g += P;
            buf[(fx.perm[g] << lgCC) + cl] = gen[((long)ni * W + mi) * bb + c];
        }
    }
    __syncthreads();
    lds_fft<double, false>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
        const int k = i >> lgCC, cl = i & (CC - 1);
        const long c = c0 + cl;
        if (c < bb) out[((long)ni * P + k) * bb + c] = buf[i];
    }
}

// y pass: rows n in (-Ny, Ny) at grid row n mod Py; result scaled by 1/(Px Py)
// and stored frequency-major, k = kx * Py + ky, as complex128 and/or complex64.
__global__ void __launch_bounds__(256) k_gen_fwd_y(const c128 *__restrict__ in, int Ny, int Px, long bb,
                                                   FFTDesc fy, int lgCC, double scl, c128 *__restrict__ G64,
                                                   c64 *__restrict__ G32) {
    extern __shared__ char smem_raw[];
    c128 *twl = reinterpret_cast<c128 *>(smem_raw);
    c128 *buf = twl + fy.P;
    const int CC = 1 << lgCC, P = fy.P, H = 2 * Ny - 1;
    const long c0 = (long)blockIdx.x * CC;
    const int kx = blockIdx.y;
    load_twiddles<double>(twl, fy);
    zero_lds<double>(buf, P * CC);
    __syncthreads();
    for (int i = threadIdx.x; i < H * CC; i += kBlock) {
        const int ni = i >> lgCC, cl = i & (CC - 1);
        const long c = c0 + cl;
        if (c < bb) {
            int g = ni - (Ny - 1);
            if (g < 0) g += P;
            buf[(fy.perm[g] << lgCC) + cl] = in[((long)ni * Px + kx) * bb + c];
        }
    }
    __syncthreads();
    lds_fft<double, false>(buf, lgCC, fy, twl);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
        const int ky = i >> lgCC, cl = i & (CC - 1);
        const long c = c0 + cl;
        if (c < bb) {
            const c128 v = scale(buf[i], scl);
            const long o = ((long)kx * P + ky) * bb + c;
            if (G64) G64[o] = v;
            if (G32) G32[o] = cvt<float>(v);
        }
    }
}

__global__ void k_cast_c64(const c128 *__restrict__ in, c64 *__restrict__ out, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = cvt<float>(in[i]);
}

hipError_t spectrum_build(tp_plan pl, const c128 *gen_dev, c128 *tmp, hipStream_t st) {
    const int Nx = pl->Nx, Ny = pl->Ny, Px = pl->Px, Py = pl->Py;
    const long bb = (long)pl->bc * pl->bc;
    const size_t es = sizeof(c128);
    {
        const int lg = fft_lgcc(Px, (int)std::min<long>(bb, 64), es);
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        dim3 grid((unsigned)((bb + (1 << lg) - 1) >> lg), 2 * Ny - 1);
        hipLaunchKernelGGL(k_gen_fwd_x, grid, dim3(256), sh, st, gen_dev, Nx, bb, pl->fx, lg, tmp);
    }
    {
        const int lg = fft_lgcc(Py, (int)std::min<long>(bb, 64), es);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((unsigned)((bb + (1 << lg) - 1) >> lg), pl->kxh);   // stored columns only
        hipLaunchKernelGGL(k_gen_fwd_y, grid, dim3(256), sh, st, tmp, Ny, Px, bb, pl->fy, lg,
                           1.0 / ((double)Px * (double)Py), pl->G64, pl->G32);
    }
    return hipGetLastError();
}

// ------------------------------------------------ preconditioner (plan time)
// In-place Gauss-Jordan inversion with partial pivoting of one b x b spectrum
// block per workgroup (row-major at S + k b^2), then scaling by scl.  Step k:
// the largest-modulus pivot in column k (ties to the lower row) is swapped
// into row k, row k is divided by it (its column-k entry becoming 1 / pivot),
// and every other row i loses f_i times row k, with f_i its column-k entry
// (which becomes -f_i / pivot).  The row interchanges are undone on the
// columns of the result, in reverse order.
__global__ void __launch_bounds__(256) k_block_inv(c128 *__restrict__ S, int b, double scl, int *flag) {
    extern __shared__ char smem_raw[];
    c128 *f = reinterpret_cast<c128 *>(smem_raw);   // [b]
    int *perm = reinterpret_cast<int *>(f + b);      // [b]
    __shared__ int piv;
    c128 *A = S + (long)blockIdx.x * b * b;
    const int tid = threadIdx.x;
    for (int k = 0; k < b; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < b; i += 64) {
                const c128 a = A[(long)i * b + k];
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
                perm[k] = bi;
                if (!(best > 0.0) || !(best < INFINITY)) *flag = 1;
            }
        }
        __syncthreads();
        const int r = piv;
        if (r != k) {
            for (int j = tid; j < b; j += kBlock) {
                const c128 t = A[(long)k * b + j];
                A[(long)k * b + j] = A[(long)r * b + j];
                A[(long)r * b + j] = t;
            }
            __syncthreads();
        }
        const c128 pv = A[(long)k * b + k];
        const double pd = 1.0 / (pv.x * pv.x + pv.y * pv.y);
        const c128 inv{pv.x * pd, -pv.y * pd};
        __syncthreads();
        for (int j = tid; j < b; j += kBlock) A[(long)k * b + j] = (j == k ? c128{1, 0} : A[(long)k * b + j]) * inv;
        for (int i = tid; i < b; i += kBlock)
            if (i != k) f[i] = A[(long)i * b + k];
        __syncthreads();
        for (long idx = tid; idx < (long)b * b; idx += kBlock) {
            const int i = (int)(idx / b), j = (int)(idx - (long)i * b);
            if (i == k) continue;
            A[idx] = (j == k ? c128{0, 0} : A[idx]) - f[i] * A[(long)k * b + j];
        }
        __syncthreads();
    }
    for (int k = b - 1; k >= 0; --k) {
        const int r = perm[k];
        if (r != k) {
            for (int i = tid; i < b; i += kBlock) {
                const c128 t = A[(long)i * b + k];
                A[(long)i * b + k] = A[(long)i * b + r];
                A[(long)i * b + r] = t;
            }
        }
        __syncthreads();
    }
    for (long idx = tid; idx < (long)b * b; idx += kBlock) A[idx] = scale(A[idx], scl);
}

// D[t] = 1 / C[t][t]
__global__ void k_diag_inv(const c128 *__restrict__ Cm, int Nr, c128 *__restrict__ D, int *flag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Nr) return;
    const c128 c = Cm[(long)t * Nr + t];
    const double dd = c.x * c.x + c.y * c.y;
    if (!(dd > 0.0) || !(dd < INFINITY)) *flag = 1;
    D[t] = c128{c.x / dd, -c.y / dd};
}

// In-place inverse of one dense n x n complex128 matrix (row-major), one
// workgroup; flag set when a pivot vanishes.
hipError_t dense_inverse(c128 *A, int n, int *flag, hipStream_t st) {
    const size_t sh = (size_t)n * (sizeof(c128) + sizeof(int));
    hipLaunchKernelGGL(k_block_inv, dim3(1), dim3(256), sh, st, A, n, 1.0, flag);
    return hipGetLastError();
}

hipError_t precond_build(tp_plan pl, c128 *S, int *flag, hipStream_t st) {
    const long P = (long)pl->Px * pl->Py;
    const double scl = 1.0 / ((double)P * (double)P);
    const size_t sh = (size_t)pl->bc * (sizeof(c128) + sizeof(int));
    // the stored blocks only: the inverse of a transposed block is the
    // transposed inverse, so a half spectrum gives a half preconditioner
    const long nblk = (long)pl->kxh * pl->Py;
    hipLaunchKernelGGL(k_block_inv, dim3((unsigned)nblk), dim3(256), sh, st, S, pl->bc, scl, flag);
    hipError_t e = hipGetLastError();
    if (e) return e;
    if (pl->Nr > 0 && pl->D64) {
        hipLaunchKernelGGL(k_diag_inv, dim3((pl->Nr + 255) / 256), dim3(256), 0, st, pl->C64, pl->Nr, pl->D64, flag);
        e = hipGetLastError();
    }
    return e;
}

hipError_t cast_to_c64(const c128 *in, c64 *out, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_cast_c64, dim3((unsigned)nb), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

template <typename T, bool PRE>
static int path_bits(tp_plan pl, int R) {
    const Path P = choose_path<T, PRE>(pl, R);
    return (P.fused ? TP_PATH_FUSED : 0) | (P.pairs ? TP_PATH_PAIRS : 0) | (P.mfma ? TP_PATH_MFMA : 0) |
           (P.rim ? TP_PATH_DENSE_RIM : 0) | (P.rim_mma ? TP_PATH_RIM_MFMA : 0) |
           (P.lg2 >= 0 ? TP_PATH_TILES2D : 0) | (P.fusedm ? TP_PATH_PERSISTENT : 0) |
           (P.rimfwd ? TP_PATH_RIM_OVERLAP : 0);
}

int path_flags(tp_plan pl, bool fp64, bool pre, int R) {
    if (fp64) return pre ? path_bits<double, true>(pl, R) : path_bits<double, false>(pl, R);
    return pre ? path_bits<float, true>(pl, R) : path_bits<float, false>(pl, R);
}

}  // namespace tp
