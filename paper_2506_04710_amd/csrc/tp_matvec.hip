// Operator application y = Z x for the array impedance matrix
// Z = [[A, B_er], [B, C]] (eq. matrixForm; B_er = B^T when reciprocal).
//
// A x_A is a two-level block-Toeplitz product.  It is computed through circulant
// embedding on a Px x Py grid (Px >= 2Nx-1, Py >= 2Ny-1) as
//   y_A = crop( IDFT2( Ghat[k] * DFT2(pad(x_A))[k] ) ),
// with Ghat the scaled spectrum of the placed generators built at plan time.
// Channel c = r*b + p (right-hand side r, basis p) is the contiguous axis of
// every grid, so every transform pass reads and writes whole channel runs.
//
// Stages (one kernel each):
//   k_fwd_x   embed + DFT along x, rows iy < Ny only      x      -> [Ny][Px][C]
//   k_fwd_y   DFT along y (inputs iy < Ny)                      -> [Px][Py][C]
//   k_prod    per-frequency b x b block times b x R block        -> [Px][Py][C]
//   k_inv_y   inverse DFT along y, keep iy < Ny                  -> [Ny][Px][C]
//   k_inv_x   inverse DFT along x, keep ix < Nx, add rim term    -> y_A
//   k_rim_main  one pass over B: y_A = B_er x_r, partial B x_A
//   k_rim_finish  y_r = sum of partials + C x_r
#include "tp_fft.h"
#include "tp_internal.h"

namespace tp {

// ------------------------------------------------------------------ helpers
template <typename T>
__device__ __forceinline__ cpx<T> shfl_xor_c(cpx<T> v, int m) {
    return mk<T>(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}
template <typename T>
__device__ __forceinline__ cpx<T> wave_sum(cpx<T> v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + shfl_xor_c(v, m);
    return v;
}

// Column activity: a NULL entry in a column-pointer table marks an idle column
// (the solver masks columns this way).  Without a table every column is live.
__device__ __forceinline__ bool cols_live(const void *const *tab, int r0, int r1) {
    if (!tab) return true;
    for (int r = r0; r <= r1; ++r)
        if (tab[r]) return true;
    return false;
}

template <typename T>
__device__ __forceinline__ void zero_lds(cpx<T> *buf, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) buf[i] = mk<T>(0, 0);
}

// ------------------------------------------------------------ FFT passes
template <typename T, typename In>
__global__ void __launch_bounds__(256) k_fwd_x(Cols<const In> x, int R, int Nx, int b, FFTDesc fx,
                                               int lgCC, cpx<T> *__restrict__ out) {
    extern __shared__ char smem_raw[];
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fx.P;
    const int CC = 1 << lgCC, C = b * R, P = fx.P;
    const int c0 = blockIdx.x * CC, iy = blockIdx.y;
    if (!cols_live((const void *const *)x.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twl, fx);
    zero_lds<T>(buf, P * CC);
    __syncthreads();
    for (int i = threadIdx.x; i < Nx * CC; i += blockDim.x) {
        const int ix = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            const In *xc = x.col(r);
            if (xc) buf[(fx.perm[ix] << lgCC) + cl] = cvt<T>(xc[(long)(iy * Nx + ix) * b + p]);
        }
    }
    __syncthreads();
    lds_fft<T, false>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
        const int k = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) out[((long)iy * P + k) * C + c] = buf[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fwd_y(const cpx<T> *__restrict__ in, int C, int Ny, int Px,
                                               FFTDesc fy, int lgCC, cpx<T> *__restrict__ out,
                                               const void *const *act, int b) {
    extern __shared__ char smem_raw[];
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fy.P;
    const int CC = 1 << lgCC, P = fy.P;
    const int c0 = blockIdx.x * CC, kx = blockIdx.y;
    if (!cols_live(act, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twl, fy);
    zero_lds<T>(buf, P * CC);
    __syncthreads();
    for (int i = threadIdx.x; i < Ny * CC; i += blockDim.x) {
        const int iy = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) buf[(fy.perm[iy] << lgCC) + cl] = in[((long)iy * Px + kx) * C + c];
    }
    __syncthreads();
    lds_fft<T, false>(buf, lgCC, fy, twl);
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
        const int ky = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) out[((long)kx * P + ky) * C + c] = buf[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_inv_y(const cpx<T> *__restrict__ in, int C, int Ny, int Px,
                                               FFTDesc fy, int lgCC, cpx<T> *__restrict__ out,
                                               const void *const *act, int b) {
    extern __shared__ char smem_raw[];
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fy.P;
    const int CC = 1 << lgCC, P = fy.P;
    const int c0 = blockIdx.x * CC, kx = blockIdx.y;
    if (!cols_live(act, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twl, fy);
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
        const int ky = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        buf[(fy.perm[ky] << lgCC) + cl] = (c < C) ? in[((long)kx * P + ky) * C + c] : mk<T>(0, 0);
    }
    __syncthreads();
    lds_fft<T, true>(buf, lgCC, fy, twl);
    for (int i = threadIdx.x; i < Ny * CC; i += blockDim.x) {
        const int iy = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) out[((long)iy * Px + kx) * C + c] = buf[i];
    }
}

template <typename T, typename Out>
__global__ void __launch_bounds__(256) k_inv_x(const cpx<T> *__restrict__ in, int R, int Nx, int b,
                                               FFTDesc fx, int lgCC, Cols<Out> y, int accumulate) {
    extern __shared__ char smem_raw[];
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fx.P;
    const int CC = 1 << lgCC, C = b * R, P = fx.P;
    const int c0 = blockIdx.x * CC, iy = blockIdx.y;
    if (!cols_live((const void *const *)y.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twl, fx);
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
        const int kx = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        buf[(fx.perm[kx] << lgCC) + cl] = (c < C) ? in[((long)iy * P + kx) * C + c] : mk<T>(0, 0);
    }
    __syncthreads();
    lds_fft<T, true>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < Nx * CC; i += blockDim.x) {
        const int ix = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            Out *yc = y.col(r);
            if (!yc) continue;
            Out *dst = yc + (long)(iy * Nx + ix) * b + p;
            cpx<T> v = buf[i];
            if (accumulate) v = v + cvt<T>(*dst);
            *dst = cvt<typename Out::value_type>(v);
        }
    }
}

// ---------------------------------------------------- per-frequency product
// Workgroup = one frequency k, four waves.  Wave w streams rows p = w, w+4, ...
// of the b x b spectrum block: lane l reads G[k][p][q] for q = l, l+64, ...
// (one contiguous row segment per wave instruction), multiplies it with the
// input columns staged in LDS and the wave sums the row.  Rows are unrolled by
// U so that U independent loads are in flight per lane.  RB right-hand sides
// share each spectrum load; blockIdx.y selects the RB-column block.
template <typename T, int RB, int U>
__global__ void __launch_bounds__(256) k_prod(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in,
                                              int b, int R, cpx<T> *__restrict__ out, const void *const *act) {
    extern __shared__ char smem_raw[];
    cpx<T> *xs = reinterpret_cast<cpx<T> *>(smem_raw);   // [RB][b]
    const int C = b * R, rb = blockIdx.y * RB;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const long k = blockIdx.x;
    if (!cols_live(act, rb, min(rb + RB, R) - 1)) return;
    const cpx<T> *Gk = G + k * (long)b * b;
    for (int i = threadIdx.x; i < RB * b; i += blockDim.x) {
        const int c = i / b, q = i - c * b;
        xs[i] = (rb + c < R) ? in[k * C + (long)(rb + c) * b + q] : mk<T>(0, 0);
    }
    __syncthreads();
    for (int p0 = w; p0 < b; p0 += nw * U) {
        cpx<T> acc[U][RB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < RB; ++c) acc[u][c] = mk<T>(0, 0);
        for (int q = lane; q < b; q += 64) {
            cpx<T> g[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + u * nw;
                g[u] = (p < b) ? Gk[(long)p * b + q] : mk<T>(0, 0);
            }
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                const cpx<T> xv = xs[c * b + q];
#pragma unroll
                for (int u = 0; u < U; ++u) acc[u][c] = cmac(acc[u][c], g[u], xv);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * nw;
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                const cpx<T> s = wave_sum(acc[u][c]);
                if (lane == 0 && p < b && rb + c < R) out[k * C + (long)(rb + c) * b + p] = s;
            }
        }
    }
}

// ------------------------------------------------------------------- rim
// Workgroup = one slab of TE = 64*E element columns and all Nr rim rows.  Lane
// l of wave w owns columns e0 + l + 64 i and rows w, w + nw, ...:
//   uA[e]   = sum_row BE[row][e] x_r[row]   (BE = B when reciprocal)  -> y_A
//   part[slab][row] = sum_{e in slab} B[row][e] x_A[e]                -> y_r partials
template <typename T, typename In, typename Out, int E, int RB>
__global__ void __launch_bounds__(256) k_rim_main(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                                  Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                                  cpx<T> *__restrict__ part) {
    extern __shared__ char smem_raw[];
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int TE = 64 * E, slab = blockIdx.x, rb = blockIdx.y * RB;
    const long e0 = (long)slab * TE;
    if (!cols_live((const void *const *)x.tab, rb, min(rb + RB, R) - 1)) return;
    cpx<T> *xr = reinterpret_cast<cpx<T> *>(smem_raw);            // [RB][Nr]
    cpx<T> *ua = xr + RB * Nr;                                       // [nw][TE][RB]
    for (int i = threadIdx.x; i < RB * Nr; i += blockDim.x) {
        const int c = i / Nr, t = i - c * Nr;
        const In *xc = (rb + c < R) ? x.col(rb + c) : nullptr;
        xr[i] = xc ? cvt<T>(xc[N + t]) : mk<T>(0, 0);
    }
    cpx<T> xa[E][RB], acc[E][RB];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const long e = e0 + lane + 64 * i;
#pragma unroll
        for (int c = 0; c < RB; ++c) {
            const In *xc = (rb + c < R) ? x.col(rb + c) : nullptr;
            xa[i][c] = (e < N && xc) ? cvt<T>(xc[e]) : mk<T>(0, 0);
            acc[i][c] = mk<T>(0, 0);
        }
    }
    __syncthreads();
    const cpx<T> *BEm = BE ? BE : B;
    for (int row = w; row < Nr; row += nw) {
        cpx<T> s[RB];
#pragma unroll
        for (int c = 0; c < RB; ++c) s[c] = mk<T>(0, 0);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const long e = e0 + lane + 64 * i;
            if (e < N) {
                const cpx<T> g = B[(long)row * N + e];
                const cpx<T> ge = BE ? BEm[(long)row * N + e] : g;
#pragma unroll
                for (int c = 0; c < RB; ++c) {
                    s[c] = cmac(s[c], g, xa[i][c]);
                    acc[i][c] = cmac(acc[i][c], ge, xr[c * Nr + row]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < RB; ++c) {
            cpx<T> t = wave_sum(s[c]);
            if (lane == 0 && rb + c < R) part[((long)slab * Nr + row) * R + rb + c] = t;
        }
    }
#pragma unroll
    for (int i = 0; i < E; ++i)
#pragma unroll
        for (int c = 0; c < RB; ++c) ua[((long)w * TE + lane + 64 * i) * RB + c] = acc[i][c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < TE * RB; idx += blockDim.x) {
        const int el = idx / RB, c = idx - el * RB;
        const long e = e0 + el;
        Out *yc = (e < N && rb + c < R) ? y.col(rb + c) : nullptr;
        if (yc) {
            cpx<T> s = mk<T>(0, 0);
            for (int v = 0; v < nw; ++v) s = s + ua[(long)v * TE * RB + idx];
            yc[e] = cvt<typename Out::value_type>(s);
        }
    }
}

template <typename T, typename In, typename Out>
__global__ void __launch_bounds__(64) k_rim_finish(const cpx<T> *__restrict__ part, const cpx<T> *__restrict__ Cm,
                                                   Cols<const In> x, Cols<Out> y, int R, long N, int Nr, int nslab) {
    const int row = blockIdx.x, c = blockIdx.y, lane = threadIdx.x;
    const In *xcol = x.col(c);
    Out *ycol = y.col(c);
    if (!xcol || !ycol) return;
    cpx<T> s = mk<T>(0, 0);
    for (int t = lane; t < nslab; t += 64) s = s + part[((long)t * Nr + row) * R + c];
    const In *xc = xcol + N;
    for (int t = lane; t < Nr; t += 64) s = cmac(s, Cm[(long)row * Nr + t], cvt<T>(xc[t]));
    s = wave_sum(s);
    if (lane == 0) ycol[N + row] = cvt<typename Out::value_type>(s);
}

// --------------------------------------------------------------- launcher
static int fft_lgcc(int P, int C, size_t elem) {
    // channels per workgroup: a power of two, at most 64, LDS tile <= 48 KB
    int lg = 6;
    while (lg > 0 && ((size_t)P * ((size_t)1 << lg) + P) * elem > 48 * 1024) --lg;
    while (lg > 0 && (1 << (lg - 1)) >= C) --lg;
    return lg;
}

template <typename T>
struct OpPtrs;
template <>
struct OpPtrs<double> {
    static const c128 *G(tp_plan p) { return p->G64; }
    static const c128 *B(tp_plan p) { return p->B64; }
    static const c128 *BE(tp_plan p) { return p->BE64; }
    static const c128 *C(tp_plan p) { return p->C64; }
};
template <>
struct OpPtrs<float> {
    static const c64 *G(tp_plan p) { return p->G32; }
    static const c64 *B(tp_plan p) { return p->B32; }
    static const c64 *BE(tp_plan p) { return p->BE32; }
    static const c64 *C(tp_plan p) { return p->C32; }
};

template <typename T, typename In, typename Out>
hipError_t matvec_launch(tp_plan pl, Cols<const In> x, Cols<Out> y, int R, hipStream_t st) {
    const int Nx = pl->Nx, Ny = pl->Ny, b = pl->b, Nr = pl->Nr;
    const int Px = pl->Px, Py = pl->Py, C = b * R;
    cpx<T> *gA = reinterpret_cast<cpx<T> *>(pl->gridA);
    cpx<T> *gB = reinterpret_cast<cpx<T> *>(pl->gridB);
    const size_t es = sizeof(cpx<T>);
    const dim3 blk(256);
    const void *const *act = (const void *const *)x.tab;

    if (Nr > 0) {
        constexpr int RB = 1;
        const int E = pl->rim_te / 64;
        const int nw = 4;
        const size_t sh = ((size_t)RB * Nr + (size_t)nw * pl->rim_te * RB) * es;
        dim3 grid(pl->rim_nslab, (R + RB - 1) / RB);
        cpx<T> *part = reinterpret_cast<cpx<T> *>(pl->rim_part);
        if (E == 1)
            hipLaunchKernelGGL((k_rim_main<T, In, Out, 1, RB>), grid, dim3(64 * nw), sh, st, OpPtrs<T>::B(pl),
                               OpPtrs<T>::BE(pl), x, y, R, pl->N, Nr, part);
        else if (E == 2)
            hipLaunchKernelGGL((k_rim_main<T, In, Out, 2, RB>), grid, dim3(64 * nw), sh, st, OpPtrs<T>::B(pl),
                               OpPtrs<T>::BE(pl), x, y, R, pl->N, Nr, part);
        else
            hipLaunchKernelGGL((k_rim_main<T, In, Out, 4, RB>), grid, dim3(64 * nw), sh, st, OpPtrs<T>::B(pl),
                               OpPtrs<T>::BE(pl), x, y, R, pl->N, Nr, part);
    }
    {
        const int lg = fft_lgcc(Px, C, es);
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Ny);
        hipLaunchKernelGGL((k_fwd_x<T, In>), grid, blk, sh, st, x, R, Nx, b, pl->fx, lg, gA);
    }
    {
        const int lg = fft_lgcc(Py, C, es);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_fwd_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    {
        const int RBc = R >= 16 ? 16 : R >= 8 ? 8 : R >= 4 ? 4 : R >= 2 ? 2 : 1;
        const size_t sh = (size_t)RBc * b * es;
        dim3 grid(Px * Py, (R + RBc - 1) / RBc);
        const cpx<T> *G = OpPtrs<T>::G(pl);
        switch (RBc) {
            case 1: hipLaunchKernelGGL((k_prod<T, 1, 4>), grid, blk, sh, st, G, gB, b, R, gA, act); break;
            case 2: hipLaunchKernelGGL((k_prod<T, 2, 4>), grid, blk, sh, st, G, gB, b, R, gA, act); break;
            case 4: hipLaunchKernelGGL((k_prod<T, 4, 2>), grid, blk, sh, st, G, gB, b, R, gA, act); break;
            case 8: hipLaunchKernelGGL((k_prod<T, 8, 1>), grid, blk, sh, st, G, gB, b, R, gA, act); break;
            default: hipLaunchKernelGGL((k_prod<T, 16, 1>), grid, blk, sh, st, G, gB, b, R, gA, act); break;
        }
    }
    {
        const int lg = fft_lgcc(Py, C, es);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_inv_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    {
        const int lg = fft_lgcc(Px, C, es);
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Ny);
        hipLaunchKernelGGL((k_inv_x<T, Out>), grid, blk, sh, st, gB, R, Nx, b, pl->fx, lg, y, Nr > 0 ? 1 : 0);
    }
    if (Nr > 0) {
        hipLaunchKernelGGL((k_rim_finish<T, In, Out>), dim3(Nr, R), dim3(64), 0, st,
                           reinterpret_cast<const cpx<T> *>(pl->rim_part), OpPtrs<T>::C(pl), x, y, R, pl->N, Nr,
                           pl->rim_nslab);
    }
    return hipGetLastError();
}

hipError_t matvec_fp64(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st) {
    return matvec_launch<double, c128, c128>(pl, x, y, R, st);
}
hipError_t matvec_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st) {
    return matvec_launch<float, c64, c64>(pl, x, y, R, st);
}
hipError_t matvec_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st) {
    return matvec_launch<float, c128, c128>(pl, x, y, R, st);
}

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
    for (int i = threadIdx.x; i < W * CC; i += blockDim.x) {
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
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
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
    for (int i = threadIdx.x; i < H * CC; i += blockDim.x) {
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
    for (int i = threadIdx.x; i < P * CC; i += blockDim.x) {
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
    const long bb = (long)pl->b * pl->b;
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
        dim3 grid((unsigned)((bb + (1 << lg) - 1) >> lg), Px);
        hipLaunchKernelGGL(k_gen_fwd_y, grid, dim3(256), sh, st, tmp, Ny, Px, bb, pl->fy, lg,
                           1.0 / ((double)Px * (double)Py), pl->G64, pl->G32);
    }
    return hipGetLastError();
}

hipError_t cast_to_c64(const c128 *in, c64 *out, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_cast_c64, dim3((unsigned)nb), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

}  // namespace tp
