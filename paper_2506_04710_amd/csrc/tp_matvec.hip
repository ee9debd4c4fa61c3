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
// Kernels:
//   k_fwd_x      embed + DFT along x, rows iy < Ny only     x -> [Ny][Px][C]
//   k_fwd_y      DFT along y (inputs iy < Ny)                 -> [Px][Py][C]
//   k_prod       per-frequency b x b block times b x R block  -> [Px][Py][C]
//   k_inv_y      inverse DFT along y, keep iy < Ny            -> [Ny][Px][C]
//   k_rim_main   one pass over B: y_A = B_er x_r, partial B x_A per slab
//   k_inv_x_fin  inverse DFT along x, keep ix < Nx, add the rim term -> y_A;
//                and y_r = sum of the slab partials + C x_r
//   k_spec_rim   single-column path: y transform, product and inverse y
//                transform fused per spectrum column, with the rim pass as
//                extra workgroups of the same launch
// A single column runs k_fwd_x -> k_spec_rim -> k_inv_x_fin; several columns
// run k_rim_main, k_fwd_x, k_fwd_y, k_prod, k_inv_y, k_inv_x_fin.
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

template <typename T>
__device__ __forceinline__ void zero_lds(cpx<T> *buf, int n) {
    for (int i = threadIdx.x; i < n; i += kBlock) buf[i] = mk<T>(0, 0);
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
    for (int i = threadIdx.x; i < Nx * CC; i += kBlock) {
        const int ix = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            const In *xc = x.col(r);
            if (xc) buf[(fx.perm[ix] << lgCC) + cl] = cvt<T>(xc[(long)(iy * Nx + ix) * b + p]);
        }
    }
    __syncthreads();
    lds_fft<T, false>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
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
    for (int i = threadIdx.x; i < Ny * CC; i += kBlock) {
        const int iy = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) buf[(fy.perm[iy] << lgCC) + cl] = in[((long)iy * Px + kx) * C + c];
    }
    __syncthreads();
    lds_fft<T, false>(buf, lgCC, fy, twl);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
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
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
        const int ky = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        buf[(fy.perm[ky] << lgCC) + cl] = (c < C) ? in[((long)kx * P + ky) * C + c] : mk<T>(0, 0);
    }
    __syncthreads();
    lds_fft<T, true>(buf, lgCC, fy, twl);
    for (int i = threadIdx.x; i < Ny * CC; i += kBlock) {
        const int iy = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) out[((long)iy * Px + kx) * C + c] = buf[i];
    }
}

// ---------------------------------------------------- per-frequency product
// Several columns.  Workgroup = one frequency k and a block of RC columns.
// The RC input columns xhat[k][r][0..b) sit in LDS; the b x b spectrum block
// is streamed in 8-row panels with 8 lanes per row (lane l: row l >> 3 of the
// panel, values q in [(l & 7) VPL, (l & 7) VPL + VPL)), each lane forms its
// part of the RC row products and the 8 lanes of a row add them up.  Wave w
// takes panels w, w + 4, ... with the next panel's loads issued first.
template <typename T, int VPL, int RC>
__global__ void __launch_bounds__(256) k_prod(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in,
                                              int b, int R, cpx<T> *__restrict__ out, const void *const *act) {
    extern __shared__ char smem_raw[];
    cpx<T> *xs = reinterpret_cast<cpx<T> *>(smem_raw);   // [RC][b]
    const int C = b * R, r0 = blockIdx.y * RC;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kBlock >> 6;
    const long k = blockIdx.x;
    const int rn = min(RC, R - r0);
    if (!cols_live(act, r0, r0 + rn - 1)) return;
    const int pl = lane >> 3, qs = (lane & 7) * VPL;
    const cpx<T> *Gk = G + k * (long)b * b;
    const int npanel = (b + 7) >> 3;
    cpx<T> gc[VPL], gn[VPL];
    auto load = [&](cpx<T>(&g)[VPL], int panel) {
        const int p = panel * 8 + pl;
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const int q = qs + v;
            g[v] = (panel < npanel && p < b && q < b) ? Gk[(long)p * b + q] : mk<T>(0, 0);
        }
    };
    load(gc, w);
    for (int i = threadIdx.x; i < RC * b; i += kBlock) {
        const int c = i / b, q = i - c * b;
        xs[i] = (c < rn) ? in[k * C + (long)(r0 + c) * b + q] : mk<T>(0, 0);
    }
    __syncthreads();
    for (int panel = w; panel < npanel; panel += nw) {
        const int nxt = panel + nw;
        if (nxt < npanel) load(gn, nxt);
        const int p = panel * 8 + pl;
        cpx<T> acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = mk<T>(0, 0);
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            if (qs + v < b) {
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[c] = cmac(acc[c], gc[v], xs[c * b + qs + v]);
            }
        }
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            acc[c] = acc[c] + shfl_xor_c(acc[c], 1);
            acc[c] = acc[c] + shfl_xor_c(acc[c], 2);
            acc[c] = acc[c] + shfl_xor_c(acc[c], 4);
        }
        if ((lane & 7) == 0 && p < b) {
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (c < rn) out[k * C + (long)(r0 + c) * b + p] = acc[c];
        }
        if (nxt < npanel) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) gc[v] = gn[v];
        }
    }
}

// ------------------------------------------------------------------- rim
// One slab = TE = 64*E element columns x all Nr rim rows.  Lane l of wave w
// owns columns e0 + l + 64 i; wave w takes rows in groups of UR consecutive
// rows (w*UR, w*UR + nw*UR, ...), issuing all UR*E loads of a group before
// using any, so UR*E independent loads are in flight per lane:
//   uA[e]            = sum_row BE[row][e] x_r[row]   (BE = B when reciprocal) -> y_A
//   part[slab][row]  = sum_{e in slab} B[row][e] x_A[e]                      -> y_r partials
template <typename T, typename In, typename Out, int E, int RB, int UR, bool NBE>
__device__ __forceinline__ void rim_block(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                          Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                          cpx<T> *__restrict__ part, int slab, int rbk, char *smem) {
    const int nw = kBlock >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int TE = 64 * E, rb = rbk * RB;
    const long e0 = (long)slab * TE;
    if (!cols_live((const void *const *)x.tab, rb, min(rb + RB, R) - 1)) return;
    cpx<T> *xr = reinterpret_cast<cpx<T> *>(smem);   // [RB][Nr]
    cpx<T> *ua = xr + RB * Nr;                          // [nw][TE][RB]
    for (int i = threadIdx.x; i < RB * Nr; i += kBlock) {
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
    for (int r0 = w * UR; r0 < Nr; r0 += nw * UR) {
        cpx<T> g[UR][E], ge[NBE ? UR : 1][E];
#pragma unroll
        for (int u = 0; u < UR; ++u)
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const long e = e0 + lane + 64 * i;
                const int row = r0 + u;
                const bool ok = row < Nr && e < N;
                g[u][i] = ok ? B[(long)row * N + e] : mk<T>(0, 0);
                if constexpr (NBE) ge[u][i] = ok ? BE[(long)row * N + e] : mk<T>(0, 0);
            }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int row = r0 + u;
            cpx<T> sr[RB];
#pragma unroll
            for (int c = 0; c < RB; ++c) sr[c] = mk<T>(0, 0);
#pragma unroll
            for (int i = 0; i < E; ++i)
#pragma unroll
                for (int c = 0; c < RB; ++c) {
                    sr[c] = cmac(sr[c], g[u][i], xa[i][c]);
                    if (row < Nr) acc[i][c] = cmac(acc[i][c], NBE ? ge[NBE ? u : 0][i] : g[u][i], xr[c * Nr + row]);
                }
#pragma unroll
            for (int c = 0; c < RB; ++c) {
                const cpx<T> t = wave_sum(sr[c]);
                if (lane == 0 && row < Nr && rb + c < R) part[((long)slab * Nr + row) * R + rb + c] = t;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < E; ++i)
#pragma unroll
        for (int c = 0; c < RB; ++c) ua[((long)w * TE + lane + 64 * i) * RB + c] = acc[i][c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < TE * RB; idx += kBlock) {
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

template <typename T, typename In, typename Out, int E, int RB, int UR, bool NBE>
__global__ void __launch_bounds__(256) k_rim_main(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                                  Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                                  cpx<T> *__restrict__ part) {
    extern __shared__ char smem_raw[];
    rim_block<T, In, Out, E, RB, UR, NBE>(B, BE, x, y, R, N, Nr, part, blockIdx.x, blockIdx.y, smem_raw);
}

// y_r = sum over slabs of the partials + C x_r; one wave per (rim row, column).
template <typename T, typename In, typename Out>
__device__ __forceinline__ void rim_finish_wave(const cpx<T> *__restrict__ part, const cpx<T> *__restrict__ Cm,
                                                Cols<const In> x, Cols<Out> y, int R, long N, int Nr, int nslab,
                                                int row, int c) {
    const int lane = threadIdx.x & 63;
    if (row >= Nr) return;
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

// Preconditioner rim entries: y_r = base_r + D x_r (D = 1 / diag(C)); one wave
// per (rim row block of 64, column).
template <typename T, typename In, typename Out>
__device__ __forceinline__ void diag_finish_wave(const cpx<T> *__restrict__ D, Cols<const In> x, Cols<Out> y,
                                                 Cols<const Out> acc, int accumulate, long N, int Nr, int row,
                                                 int c) {
    const int lane = threadIdx.x & 63;
    if (row >= Nr) return;
    const In *xcol = x.col(c);
    Out *ycol = y.col(c);
    if (!xcol || !ycol) return;
    const Out *ac = accumulate ? acc.col(c) : nullptr;
    if (lane == 0) {
        Out v = cvt<typename Out::value_type>(D[row] * cvt<T>(xcol[N + row]));
        if (ac) v = v + ac[N + row];
        ycol[N + row] = v;
    }
}

// ------------------------------------------------ fused single-column path
// Workgroup = (frequency column kx, 8 spectrum rows p0..p0+7).  It
//   1. loads the x-transformed column X1[iy][kx][0..b) (iy < Ny) into LDS and
//      transforms it along y (all Py frequencies, all b channels);
//   2. streams the 8 x b row panels of the Py spectrum blocks G[kx][ky]
//      (one contiguous 8*b run per ky): lane l takes row l >> 3 and the VPL
//      values q in [(l & 7) VPL, (l & 7) VPL + VPL), multiplies them with
//      xhat[ky][q] and the 8 lanes of the row add up their parts; wave w takes
//      ky = w, w + 4, ... and keeps the loads of the next U frequencies in
//      flight while it reduces the current ones (the first group is issued
//      before the y transform);
//   3. inverse-transforms the 8 output channels along y in LDS and writes the
//      rows iy < Ny of Y1.
// The y transform of the input column is repeated by the b / 8 workgroups of
// a column; it is small next to the spectrum stream.
template <typename T>
__device__ __forceinline__ cpx<T> sum8(cpx<T> v) {
    v = v + shfl_xor_c(v, 1);
    v = v + shfl_xor_c(v, 2);
    return v + shfl_xor_c(v, 4);
}

template <typename T, int VPL, int U>
__device__ __forceinline__ void spec_block(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ X1,
                                           cpx<T> *__restrict__ Y1, int b, int Ny, int Px, const FFTDesc &fy,
                                           int lgCC, int blk, char *smem) {
    constexpr int TP = 8;
    const int P = fy.P, CC = 1 << lgCC;
    const int nchunk = (b + TP - 1) / TP;
    const int kx = blk / nchunk, p0 = (blk - kx * nchunk) * TP;
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem);
    cpx<T> *xs = twl + P;          // [Py][CC]
    cpx<T> *ys = xs + P * CC;      // [Py][TP]
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kBlock >> 6;
    const int pl = lane >> 3, qs = (lane & 7) * VPL, p = p0 + pl;
    const bool prow = p < b;
    const long kstride = (long)b * b;
    const cpx<T> *Grow = G + (long)kx * P * kstride + (long)min(p, b - 1) * b;
    int *perm = reinterpret_cast<int *>(ys + P * TP);   // [Py] digit reversal, in LDS
    // Spectrum loads use clamped addresses and are masked only where used, so
    // no branch forms around them and the waits stay exact: the next U panels
    // stay in flight while the current ones are reduced.
    cpx<T> gc[U][VPL], gn[U][VPL];
    auto load = [&](cpx<T>(&g)[U][VPL], int ky0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long ky = min(ky0 + u * nw, P - 1);
#pragma unroll
            for (int v = 0; v < VPL; ++v) g[u][v] = Grow[ky * kstride + min(qs + v, b - 1)];
        }
    };
    load(gc, w);
    load_twiddles<T>(twl, fy);
    for (int i = threadIdx.x; i < P; i += kBlock) perm[i] = fy.perm[i];
    zero_lds<T>(xs, P * CC);
    __syncthreads();
    batched<8, cpx<T>>(
        Ny * CC, [&](int i) { return X1[((long)(i >> lgCC) * Px + kx) * b + min(i & (CC - 1), b - 1)]; },
        [&](int i, cpx<T> v) {
            const int iy = i >> lgCC, c = i & (CC - 1);
            if (c < b) xs[(perm[iy] << lgCC) + c] = v;
        });
    __syncthreads();
    lds_fft<T, false>(xs, lgCC, fy, twl);
    // values past the row (q >= b) are masked to zero; their LDS index is
    // clamped into the row so that no other row's (or uninitialised) value
    // enters the sum
    bool qok[VPL];
    int qi[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        qok[v] = prow && qs + v < b;
        qi[v] = min(qs + v, CC - 1);
    }
    auto reduce = [&](const cpx<T>(&g)[U][VPL], int ky0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ky = ky0 + u * nw;
            const cpx<T> *xk = xs + (min(ky, P - 1) << lgCC);
            cpx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int v = 0; v < VPL; ++v) acc = cmac(acc, keep(g[u][v], qok[v]), xk[qi[v]]);
            acc = sum8(acc);
            // the inverse transform takes its input in digit-reversed slots
            if ((lane & 7) == 0 && ky < P) ys[(perm[ky] << 3) + pl] = acc;
        }
    };
    // two register buffers in turn (no copies between them, so the compiler
    // never has to wait for a buffer's loads before the other one is used)
    // The loads are unconditional (clamped past the end): a load under a
    // branch would make the wait before the other buffer's use cover it too.
    const int step = nw * U;
    for (int ky0 = w; ky0 < P; ky0 += 2 * step) {
        load(gn, ky0 + step);
        reduce(gc, ky0);
        load(gc, ky0 + 2 * step);
        if (ky0 + step < P) reduce(gn, ky0 + step);
    }
    __syncthreads();
    lds_fft<T, true>(ys, 3, fy, twl);
    for (int i = threadIdx.x; i < Ny * TP; i += kBlock) {
        const int iy = i >> 3, pr = i & 7, pp = p0 + pr;
        if (pp < b) Y1[((long)iy * Px + kx) * b + pp] = ys[i];
    }
}

// Rim pass for a single column.  Slab = TE = 64 E element columns x all Nr
// rows; 16 lanes per row: lane l takes row offset l >> 4 of each group of 4
// rows and the VE = 4 E columns [(l & 15) VE, (l & 15) VE + VE) of the slab,
// so a group of 4 rows is 4 contiguous TE-column runs.  Per row the 16 lanes
// add up sum_e B[row][e] x_A[e] (-> slab partial of y_r); every lane keeps
// sum_row BE[row][e] x_r[row] for its columns, and those are summed over the
// row lanes and the waves at the end (-> y_A).  The next group's loads are
// issued before the current group is used.
template <typename T, typename In, typename Out, int E, bool NBE>
__device__ __forceinline__ void rim_block1(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                           Cols<const In> x, Cols<Out> y, long N, int Nr,
                                           cpx<T> *__restrict__ part, int slab, char *smem) {
    constexpr int VE = 4 * E, TE = 64 * E;
    const int nw = kBlock >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ro = lane >> 4, cs = (lane & 15) * VE;
    const long e0 = (long)slab * TE;
    const In *xc = x.col(0);
    Out *yc = y.col(0);
    if (!xc || !yc) return;
    cpx<T> *xr = reinterpret_cast<cpx<T> *>(smem);   // [Nr]
    cpx<T> *ua = xr + Nr;                               // [nw][TE]
    for (int i = threadIdx.x; i < Nr; i += kBlock) xr[i] = cvt<T>(xc[N + i]);
    cpx<T> xa[VE], acc[VE];
#pragma unroll
    for (int v = 0; v < VE; ++v) {
        const long e = e0 + cs + v;
        xa[v] = e < N ? cvt<T>(xc[e]) : mk<T>(0, 0);
        acc[v] = mk<T>(0, 0);
    }
    __syncthreads();
    // rim loads: clamped addresses, masked where used (no branches, exact waits)
    bool eok[VE];
    long ei[VE];
#pragma unroll
    for (int v = 0; v < VE; ++v) {
        eok[v] = e0 + cs + v < N;
        ei[v] = min(e0 + cs + v, N - 1);
    }
    cpx<T> gc[VE], gn[VE], ec[NBE ? VE : 1], en[NBE ? VE : 1];
    auto load = [&](cpx<T>(&g)[VE], cpx<T>(&ge)[NBE ? VE : 1], int row) {
        const long rr = (long)min(row, Nr - 1) * N;
#pragma unroll
        for (int v = 0; v < VE; ++v) {
            g[v] = B[rr + ei[v]];
            if constexpr (NBE) ge[v] = BE[rr + ei[v]];
        }
    };
    auto rows = [&](const cpx<T>(&g)[VE], const cpx<T>(&ge)[NBE ? VE : 1], int row) {
        cpx<T> sr = mk<T>(0, 0);
        const bool rok = row < Nr;
        const cpx<T> xrow = xr[min(row, Nr - 1)];
#pragma unroll
        for (int v = 0; v < VE; ++v) {
            const cpx<T> gv = keep(g[v], rok && eok[v]);
            sr = cmac(sr, gv, xa[v]);
            acc[v] = cmac(acc[v], NBE ? keep(ge[NBE ? v : 0], rok && eok[v]) : gv, xrow);
        }
        sr = sr + shfl_xor_c(sr, 8);
        sr = sum8(sr);
        if ((lane & 15) == 0 && rok) part[(long)slab * Nr + row] = sr;
    };
    // groups of 4 rows; two register buffers in turn
    const int r0 = w * 4 + ro, step = nw * 4;
    load(gc, ec, r0);
    for (int g0 = w * 4; g0 < Nr; g0 += 2 * step) {
        const int row = r0 + (g0 - w * 4);
        load(gn, en, row + step);          // unconditional: see the spectrum stream
        rows(gc, ec, row);
        load(gc, ec, row + 2 * step);
        if (g0 + step < Nr) rows(gn, en, row + step);
    }
    // sum the four row lanes of each column, then the waves
#pragma unroll
    for (int v = 0; v < VE; ++v) {
        acc[v] = acc[v] + shfl_xor_c(acc[v], 16);
        acc[v] = acc[v] + shfl_xor_c(acc[v], 32);
    }
    if (ro == 0)
#pragma unroll
        for (int v = 0; v < VE; ++v) ua[w * TE + cs + v] = acc[v];
    __syncthreads();
    for (int el = threadIdx.x; el < TE; el += kBlock) {
        const long e = e0 + el;
        if (e < N) {
            cpx<T> t = mk<T>(0, 0);
            for (int v = 0; v < nw; ++v) t = t + ua[v * TE + el];
            yc[e] = cvt<typename Out::value_type>(t);
        }
    }
}

// Spectrum workgroups and rim workgroups share one launch so that both HBM
// streams (the spectrum and the dense rim) run together; the two kinds are
// interleaved in block order.
template <typename T, typename In, typename Out, int VPL, int U, int E, bool NBE>
__global__ void __launch_bounds__(256) k_spec_rim(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ X1,
                                                  cpx<T> *__restrict__ Y1, int b, int Ny, int Px, FFTDesc fy,
                                                  int lgCC, int nspec, const cpx<T> *__restrict__ B,
                                                  const cpx<T> *__restrict__ BE, Cols<const In> x, Cols<Out> y,
                                                  long N, int Nr, cpx<T> *__restrict__ part, int nrim) {
    extern __shared__ char smem_raw[];
    const int i = blockIdx.x, both = 2 * min(nspec, nrim);
    int spec_id, rim_id;
    if (i < both) {
        spec_id = (i & 1) ? -1 : (i >> 1);
        rim_id = (i & 1) ? (i >> 1) : -1;
    } else if (nspec > nrim) {
        spec_id = i - both + nrim;
        rim_id = -1;
    } else {
        spec_id = -1;
        rim_id = i - both + nspec;
    }
    if (spec_id >= 0) {
        if (!cols_live((const void *const *)x.tab, 0, 0)) return;
        spec_block<T, VPL, U>(G, X1, Y1, b, Ny, Px, fy, lgCC, spec_id, smem_raw);
    } else if constexpr (E > 0) {
        rim_block1<T, In, Out, E, NBE>(B, BE, x, y, N, Nr, part, rim_id, smem_raw);
    }
}

// Inverse x transform + crop (+ rim term already in y), and the rim finish
// waves, in one launch: blocks [0, ninv) transform, the rest finish rim rows.
template <typename T, typename In, typename Out>
__global__ void __launch_bounds__(256) k_inv_x_fin(const cpx<T> *__restrict__ in, int R, int Nx, int b, FFTDesc fx,
                                                   int lgCC, int nchunk, Cols<Out> y, int accumulate,
                                                   Cols<const Out> acc, int ninv, const cpx<T> *__restrict__ part,
                                                   const cpx<T> *__restrict__ Cm, const cpx<T> *__restrict__ D,
                                                   Cols<const In> x, long N, int Nr, int nslab) {
    extern __shared__ char smem_raw[];
    const int blk = blockIdx.x;
    if (blk >= ninv) {
        const int f = blk - ninv, w = threadIdx.x >> 6;
        const int nrowblk = (Nr + 3) >> 2;
        const int c = f / nrowblk, row = (f - c * nrowblk) * 4 + w;
        if (D)
            diag_finish_wave<T, In, Out>(D, x, y, acc, accumulate, N, Nr, row, c);
        else
            rim_finish_wave<T, In, Out>(part, Cm, x, y, R, N, Nr, nslab, row, c);
        return;
    }
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fx.P;
    const int CC = 1 << lgCC, C = b * R, P = fx.P;
    const int iy = blk / nchunk, c0 = (blk - iy * nchunk) * CC;
    if (!cols_live((const void *const *)y.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twl, fx);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
        const int kx = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        buf[(fx.perm[kx] << lgCC) + cl] = (c < C) ? in[((long)iy * P + kx) * C + c] : mk<T>(0, 0);
    }
    __syncthreads();
    lds_fft<T, true>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < Nx * CC; i += kBlock) {
        const int ix = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            Out *yc = y.col(r);
            if (!yc) continue;
            const long e = (long)(iy * Nx + ix) * b + p;
            // the added term keeps the output's precision (an FP64 solution
            // vector updated by an FP32 preconditioner stays FP64)
            Out v = cvt<typename Out::value_type>(buf[i]);
            if (accumulate) {
                const Out *ac = acc.col(r);
                if (ac) v = v + ac[e];
            }
            yc[e] = v;
        }
    }
}

// ------------------------------------------------- small grids: 2-D tiles
// When the whole Px x Py grid of CC channels fits in LDS, one workgroup does
// both transform directions: the forward kernel embeds x_A (rows and columns
// in digit-reversed slots), transforms along y and then x, and writes the
// channel block of every frequency; the inverse kernel loads the frequencies,
// transforms along y and then x (x only for the Ny rows kept), crops to the
// elements, adds the rim term and, in extra workgroups, finishes y_r.
// Tile layout: value (x, y, channel) at (x Py + y) CC + channel.
template <typename T, typename In>
__global__ void __launch_bounds__(256) k_fft2_fwd(Cols<const In> x, int R, int Nx, int Ny, int b, FFTDesc fx,
                                                  FFTDesc fy, int lgCC, int XS, cpx<T> *__restrict__ out) {
    extern __shared__ char smem_raw[];
    cpx<T> *twx = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *twy = twx + fx.P;
    cpx<T> *buf = twy + fy.P;
    int *px = reinterpret_cast<int *>(buf + fx.P * XS);   // digit-reversal tables
    int *py = px + fx.P;
    const int CC = 1 << lgCC, C = b * R, Px = fx.P, Py = fy.P;
    const int c0 = blockIdx.x * CC;
    if (!cols_live((const void *const *)x.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twx, fx);
    load_twiddles<T>(twy, fy);
    for (int i = threadIdx.x; i < Px + Py; i += kBlock) px[i] = i < Px ? fx.perm[i] : fy.perm[i - Px];
    zero_lds<T>(buf, Px * XS);
    // kBlock is a multiple of CC, so a thread keeps one channel (and one
    // column pointer) for the whole loop and walks the elements
    {
        const int cl = threadIdx.x & (CC - 1), c = c0 + cl;
        const In *xc = c < C ? x.col(c / b) : nullptr;
        __syncthreads();
        if (xc) {
            xc += c % b;
            const int es = kBlock >> lgCC, ne = Nx * Ny;
            for (int eb = threadIdx.x >> lgCC; eb < ne; eb += 8 * es) {
                In v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = ldg(xc + (long)min(eb + u * es, ne - 1) * b);
#pragma unroll
                for (int u = 0; u < 8; ++u) pin(v[u]);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = eb + u * es;
                    if (e < ne) {
                        const int iy = e / Nx, ix = e - iy * Nx;
                        buf[px[ix] * XS + (py[iy] << lgCC) + cl] = cvt<T>(v[u]);
                    }
                }
            }
        }
    }
    __syncthreads();
    lds_fft_axis<T, false>(buf, lgCC, fy, CC, Px, XS, twy);
    lds_fft_axis<T, false>(buf, lgCC, fx, XS, Py, CC, twx);
    for (int i = threadIdx.x; i < Px * Py * CC; i += kBlock) {
        const int k = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        const int kx = k / Py, ky = k - kx * Py;
        if (c < C) out[(long)k * C + c] = buf[kx * XS + (ky << lgCC) + cl];
    }
}

template <typename T, typename In, typename Out>
__global__ void __launch_bounds__(256) k_fft2_inv_fin(const cpx<T> *__restrict__ in, int R, int Nx, int Ny, int b,
                                                      FFTDesc fx, FFTDesc fy, int lgCC, int XS, Cols<Out> y,
                                                      int accumulate, Cols<const Out> acc, int ninv,
                                                      const cpx<T> *__restrict__ part,
                                                      const cpx<T> *__restrict__ Cm, const cpx<T> *__restrict__ D,
                                                      Cols<const In> x, long N, int Nr, int nslab) {
    extern __shared__ char smem_raw[];
    const int blk = blockIdx.x;
    if (blk >= ninv) {
        const int f = blk - ninv, w = threadIdx.x >> 6;
        const int nrowblk = (Nr + 3) >> 2;
        const int c = f / nrowblk, row = (f - c * nrowblk) * 4 + w;
        if (D)
            diag_finish_wave<T, In, Out>(D, x, y, acc, accumulate, N, Nr, row, c);
        else
            rim_finish_wave<T, In, Out>(part, Cm, x, y, R, N, Nr, nslab, row, c);
        return;
    }
    cpx<T> *twx = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *twy = twx + fx.P;
    cpx<T> *buf = twy + fy.P;
    int *px = reinterpret_cast<int *>(buf + fx.P * XS);
    int *py = px + fx.P;
    const int CC = 1 << lgCC, C = b * R, Px = fx.P, Py = fy.P;
    const int c0 = blk * CC;
    if (!cols_live((const void *const *)y.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    load_twiddles<T>(twx, fx);
    load_twiddles<T>(twy, fy);
    for (int i = threadIdx.x; i < Px + Py; i += kBlock) px[i] = i < Px ? fx.perm[i] : fy.perm[i - Px];
    __syncthreads();
    batched<8, cpx<T>>(
        Px * Py * CC, [&](int i) { return in[(long)(i >> lgCC) * C + min(c0 + (i & (CC - 1)), C - 1)]; },
        [&](int i, cpx<T> v) {
            const int k = i >> lgCC, cl = i & (CC - 1);
            const int kx = k / Py, ky = k - kx * Py;
            buf[px[kx] * XS + (py[ky] << lgCC) + cl] = c0 + cl < C ? v : mk<T>(0, 0);
        });
    __syncthreads();
    lds_fft_axis<T, true>(buf, lgCC, fy, CC, Px, XS, twy);
    lds_fft_axis<T, true>(buf, lgCC, fx, XS, Ny, CC, twx);
    const int cl = threadIdx.x & (CC - 1), c = c0 + cl;
    Out *yc = c < C ? y.col(c / b) : nullptr;
    if (!yc) return;
    yc += c % b;
    const Out *ac = accumulate ? acc.col(c / b) : nullptr;
    if (ac) ac += c % b;
    const int es = kBlock >> lgCC, ne = Nx * Ny;
    for (int eb = threadIdx.x >> lgCC; eb < ne; eb += 8 * es) {
        Out old[8];
        if (ac) {
#pragma unroll
            for (int u = 0; u < 8; ++u) old[u] = ldg(ac + (long)min(eb + u * es, ne - 1) * b);
#pragma unroll
            for (int u = 0; u < 8; ++u) pin(old[u]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = eb + u * es;
            if (e < ne) {
                const int iy = e / Nx, ix = e - iy * Nx;
                Out v = cvt<typename Out::value_type>(buf[ix * XS + (iy << lgCC) + cl]);
                if (ac) v = v + old[u];
                stg(yc + (long)e * b, v);
            }
        }
    }
}

// --------------------------------------------------------------- launcher
static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Values between consecutive x rows of a 2-D tile: Py CC, padded so that the
// row stride in bytes is an odd multiple of 128; the channel runs of a wave's
// x-direction butterflies then fall in alternate halves of the 64 LDS banks.
static int fft2_xstride(int Py, int lgCC, size_t elem) {
    int xs = Py << lgCC;
    while ((xs * elem) % 256 != 128) ++xs;
    return xs;
}

// Channels per workgroup of the 2-D tile kernels (log2), or -1 when a tile of
// at least 4 channels does not fit in 48 KB of LDS.
#ifndef TP_FFT2_MAXLG
#define TP_FFT2_MAXLG 4
#endif
static int fft2_lgcc(int Px, int Py, int C, size_t elem) {
    auto bytes = [&](int lg) {
        return ((size_t)Px * fft2_xstride(Py, lg, elem) + Px + Py) * elem + (size_t)(Px + Py) * sizeof(int);
    };
    int lg = TP_FFT2_MAXLG;
    while (lg >= 2 && bytes(lg) > 48 * 1024) --lg;
    if (lg < 2) return -1;
    while (lg > 2 && (1 << (lg - 1)) >= C) --lg;
    return lg;
}

static int fft_lgcc(int P, int C, size_t elem, int max_cc = 64) {
    // channels per workgroup: a power of two, at most max_cc, LDS tile <= 48 KB
    int lg = ilog2(max_cc);
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
    static const c128 *S(tp_plan p) { return p->S64; }
    static const c128 *D(tp_plan p) { return p->D64; }
};
template <>
struct OpPtrs<float> {
    static const c64 *G(tp_plan p) { return p->G32; }
    static const c64 *B(tp_plan p) { return p->B32; }
    static const c64 *BE(tp_plan p) { return p->BE32; }
    static const c64 *C(tp_plan p) { return p->C32; }
    static const c64 *S(tp_plan p) { return p->S32; }
    static const c64 *D(tp_plan p) { return p->D32; }
};

static int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Fused single-column path: LDS bytes.
static size_t spec_lds(tp_plan pl, size_t es) {
    const int P = pl->Py, CC = next_pow2(pl->b);
    return ((size_t)P + (size_t)P * CC + (size_t)P * 8) * es + (size_t)P * sizeof(int);
}
static size_t rim_lds(tp_plan pl, int RB, size_t es) { return ((size_t)RB * pl->Nr + 4 * (size_t)pl->rim_te * RB) * es; }
constexpr size_t kLdsLimit = 160 * 1024;
// From this many columns on, the per-frequency product and the rim pass use
// the MFMA kernels (a column block of 16 or 32 fills the matrix-core tiles).
#ifndef TP_MFMA_MIN_R
#define TP_MFMA_MIN_R 16
#endif
constexpr int kMfmaMinR = TP_MFMA_MIN_R;

template <typename T, typename In, typename Out, int VPL, int E, bool NBE>
static void launch_spec_rim(tp_plan pl, const cpx<T> *G, Cols<const In> x, Cols<Out> y, cpx<T> *gA, cpx<T> *gB,
                            size_t sh, hipStream_t st) {
    // rounds kept in flight per wave: fewer for wide rows and for FP64
#ifndef TP_SPEC_U32
#define TP_SPEC_U32 2
#endif
#ifndef TP_SPEC_U32_NORIM
#define TP_SPEC_U32_NORIM TP_SPEC_U32
#endif
#ifndef TP_SPEC_U64
#define TP_SPEC_U64 2
#endif
    constexpr int U = sizeof(T) == 8 ? TP_SPEC_U64 : VPL > 8 ? 1 : (E == 0 ? TP_SPEC_U32_NORIM : TP_SPEC_U32);
    const int nchunk = (pl->b + 7) / 8, nspec = pl->Px * nchunk;
    const int nrim = E > 0 ? pl->rim_nslab : 0;
    const int lgCC = ilog2(next_pow2(pl->b));
    hipLaunchKernelGGL((k_spec_rim<T, In, Out, VPL, U, E, NBE>), dim3(nspec + nrim), dim3(256), sh, st, G, gA, gB,
                       pl->b, pl->Ny, pl->Px, pl->fy, lgCC, nspec, OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl), x, y, pl->N,
                       pl->Nr, reinterpret_cast<cpx<T> *>(pl->rim_part), nrim);
}

// rim: whether the launch carries the rim pass (the operator with Nr > 0)
template <typename T, typename In, typename Out, int VPL>
static void launch_spec_rim_e(tp_plan pl, const cpx<T> *G, bool rim, Cols<const In> x, Cols<Out> y, cpx<T> *gA,
                              cpx<T> *gB, size_t sh, hipStream_t st) {
    if (!rim) {
        launch_spec_rim<T, In, Out, VPL, 0, false>(pl, G, x, y, gA, gB, sh, st);
        return;
    }
    const bool nbe = OpPtrs<T>::BE(pl) != nullptr;
    switch ((pl->rim_te / 64) * 2 + (nbe ? 1 : 0)) {
        case 2: launch_spec_rim<T, In, Out, VPL, 1, false>(pl, G, x, y, gA, gB, sh, st); break;
        case 3: launch_spec_rim<T, In, Out, VPL, 1, true>(pl, G, x, y, gA, gB, sh, st); break;
        case 4: launch_spec_rim<T, In, Out, VPL, 2, false>(pl, G, x, y, gA, gB, sh, st); break;
        case 5: launch_spec_rim<T, In, Out, VPL, 2, true>(pl, G, x, y, gA, gB, sh, st); break;
        case 8: launch_spec_rim<T, In, Out, VPL, 4, false>(pl, G, x, y, gA, gB, sh, st); break;
        default: launch_spec_rim<T, In, Out, VPL, 4, true>(pl, G, x, y, gA, gB, sh, st); break;
    }
}

template <typename T, int VPL>
static void launch_prod_v(int RC, dim3 grid, size_t sh, hipStream_t st, const cpx<T> *G, const cpx<T> *in, int b,
                          int R, cpx<T> *out, const void *const *act) {
    switch (RC) {
        case 2: hipLaunchKernelGGL((k_prod<T, VPL, 2>), grid, dim3(256), sh, st, G, in, b, R, out, act); break;
        case 4: hipLaunchKernelGGL((k_prod<T, VPL, 4>), grid, dim3(256), sh, st, G, in, b, R, out, act); break;
        case 8: hipLaunchKernelGGL((k_prod<T, VPL, 8>), grid, dim3(256), sh, st, G, in, b, R, out, act); break;
        default: hipLaunchKernelGGL((k_prod<T, VPL, 16>), grid, dim3(256), sh, st, G, in, b, R, out, act); break;
    }
}
template <typename T>
static void launch_prod(int vpl, int RC, dim3 grid, size_t sh, hipStream_t st, const cpx<T> *G, const cpx<T> *in,
                        int b, int R, cpx<T> *out, const void *const *act) {
    if (vpl <= 2) launch_prod_v<T, 2>(RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 4) launch_prod_v<T, 4>(RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 6) launch_prod_v<T, 6>(RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 8) launch_prod_v<T, 8>(RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 12) launch_prod_v<T, 12>(RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 16) launch_prod_v<T, 16>(RC, grid, sh, st, G, in, b, R, out, act);
    else launch_prod_v<T, 32>(RC, grid, sh, st, G, in, b, R, out, act);
}

// Rows per group (UR) depend only on the slab width, in the fused and the
// general path alike: which rows a wave sums, and in which order, must not
// depend on the number of columns, so a column's result is the same alone or
// in a batch, bit for bit.
template <typename T, typename In, typename Out>
static void launch_rim_general(tp_plan pl, Cols<const In> x, Cols<Out> y, int R, hipStream_t st) {
    const size_t es = sizeof(cpx<T>);
    cpx<T> *part = reinterpret_cast<cpx<T> *>(pl->rim_part);
    const int E = pl->rim_te / 64;
    const int RB = 8 / E;
    dim3 grid(pl->rim_nslab, (R + RB - 1) / RB);
    const size_t sh = rim_lds(pl, RB, es);
    const cpx<T> *B = OpPtrs<T>::B(pl), *BE = OpPtrs<T>::BE(pl);
    switch (E * 2 + (BE ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((k_rim_main<T, In, Out, 1, 8, 8, false>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                   pl->N, pl->Nr, part); break;
        case 3: hipLaunchKernelGGL((k_rim_main<T, In, Out, 1, 8, 8, true>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                   pl->N, pl->Nr, part); break;
        case 4: hipLaunchKernelGGL((k_rim_main<T, In, Out, 2, 4, 4, false>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                   pl->N, pl->Nr, part); break;
        case 5: hipLaunchKernelGGL((k_rim_main<T, In, Out, 2, 4, 4, true>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                   pl->N, pl->Nr, part); break;
        case 8: hipLaunchKernelGGL((k_rim_main<T, In, Out, 4, 2, 2, false>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                   pl->N, pl->Nr, part); break;
        default: hipLaunchKernelGGL((k_rim_main<T, In, Out, 4, 2, 2, true>), grid, dim3(256), sh, st, B, BE, x, y, R,
                                    pl->N, pl->Nr, part); break;
    }
}

// ev (optional, kMatvecStages + 1 events): ev[0] before the first stage and
// ev[i + 1] after stage i, for per-stage timing.  Stages that a path merges
// into another are recorded as empty intervals.
// PRE: apply the block-circulant preconditioner instead of the operator:
// spectrum S, no rim pass, rim entries D x_r, and y = base + M^-1 x for the
// columns whose base pointer is set (base.tab or base.base).
template <typename T, typename In, typename Out, bool PRE = false>
hipError_t matvec_launch(tp_plan pl, Cols<const In> x, Cols<Out> y, int R, hipStream_t st,
                         hipEvent_t *ev = nullptr, Cols<const Out> base = Cols<const Out>{nullptr, 0, nullptr}) {
    const int Nx = pl->Nx, Ny = pl->Ny, b = pl->b, Nr = pl->Nr;
    const int Px = pl->Px, Py = pl->Py, C = b * R;
    cpx<T> *gA = reinterpret_cast<cpx<T> *>(pl->gridA);
    cpx<T> *gB = reinterpret_cast<cpx<T> *>(pl->gridB);
    const size_t es = sizeof(cpx<T>);
    const dim3 blk(256);
    const void *const *act = (const void *const *)x.tab;
    auto mark = [&](int i) {
        if (ev) hipEventRecord(ev[i], st);
    };
    const cpx<T> *G = PRE ? OpPtrs<T>::S(pl) : OpPtrs<T>::G(pl);
    const bool rim = !PRE && Nr > 0;         // dense rim pass
    const size_t sh_fused = std::max(spec_lds(pl, es), rim ? rim_lds(pl, 1, es) : (size_t)0);
    const bool fused = R == 1 && sh_fused <= kLdsLimit;

    // many columns: the product and the rim run on the matrix cores
    const bool mfma = !fused && R >= kMfmaMinR;
    const bool rim_mma =
        mfma && rim && pl->rim_te == 64 && rim_mfma_lds<T>(OpPtrs<T>::BE(pl) != nullptr) <= kLdsLimit;

    mark(0);
    if (rim && !fused) {
        if (rim_mma)
            rim_mfma<T, In, Out>(OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl), x, y, R, pl->N, Nr, pl->rim_nslab,
                                 reinterpret_cast<cpx<T> *>(pl->rim_part), st);
        else
            launch_rim_general<T, In, Out>(pl, x, y, R, st);
    }
    mark(1);
    // small grids with several columns: both transform directions per launch
    const int lg2 = fused ? -1 : fft2_lgcc(Px, Py, C, es);
    const int xs2 = lg2 >= 0 ? fft2_xstride(Py, lg2, es) : 0;
    const size_t sh2 = ((size_t)Px * xs2 + Px + Py) * es + (size_t)(Px + Py) * sizeof(int);
    if (lg2 >= 0) {
        hipLaunchKernelGGL((k_fft2_fwd<T, In>), dim3((C + (1 << lg2) - 1) >> lg2), blk, sh2, st, x, R, Nx, Ny, b,
                           pl->fx, pl->fy, lg2, xs2, gB);
    } else {
        const int lg = fft_lgcc(Px, C, es, 8);
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Ny);
        hipLaunchKernelGGL((k_fwd_x<T, In>), grid, blk, sh, st, x, R, Nx, b, pl->fx, lg, gA);
    }
    mark(2);
    if (!fused && lg2 < 0) {
        const int lg = fft_lgcc(Py, C, es, 16);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_fwd_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    mark(3);
    if (fused) {
        const int vpl = (b + 7) / 8;
        if (vpl <= 2) launch_spec_rim_e<T, In, Out, 2>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 4) launch_spec_rim_e<T, In, Out, 4>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 6) launch_spec_rim_e<T, In, Out, 6>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 8) launch_spec_rim_e<T, In, Out, 8>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 12) launch_spec_rim_e<T, In, Out, 12>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 16) launch_spec_rim_e<T, In, Out, 16>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else launch_spec_rim_e<T, In, Out, 32>(pl, G, rim, x, y, gA, gB, sh_fused, st);
    } else if (mfma) {
        prod_mfma<T>(G, gB, b, R, (long)Px * Py, gA, act, st);
    } else {
        // columns per workgroup: up to 16 (the spectrum block is re-read from
        // cache by each column block of a frequency)
        const int RC = R >= 16 ? 16 : R >= 8 ? 8 : R >= 4 ? 4 : 2;
        const size_t sh = (size_t)RC * b * es;
        dim3 grid(Px * Py, (R + RC - 1) / RC);
        const int vpl = (b + 7) / 8;
        launch_prod<T>(vpl, RC, grid, sh, st, G, gB, b, R, gA, act);
    }
    mark(4);
    if (!fused && lg2 < 0) {
        const int lg = fft_lgcc(Py, C, es, 16);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_inv_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    mark(5);
    // the operator adds its rim term (already in y); the preconditioner adds
    // the caller's base columns, if any
    const Cols<const Out> acc = PRE ? base : Cols<const Out>{y.base, y.ld, y.tab};
    const int accumulate = PRE ? (base.base || base.tab ? 1 : 0) : (rim ? 1 : 0);
    const cpx<T> *D = PRE ? OpPtrs<T>::D(pl) : nullptr;
    const int nfin = Nr > 0 ? ((Nr + 3) / 4) * R : 0;
    if (lg2 >= 0) {
        const int ninv = (C + (1 << lg2) - 1) >> lg2;
        hipLaunchKernelGGL((k_fft2_inv_fin<T, In, Out>), dim3(ninv + nfin), blk, sh2, st, gA, R, Nx, Ny, b, pl->fx,
                           pl->fy, lg2, xs2, y, accumulate, acc, ninv,
                           reinterpret_cast<const cpx<T> *>(pl->rim_part), OpPtrs<T>::C(pl), D, x, pl->N, Nr,
                           pl->rim_nslab);
    } else {
        // the fused path leaves Y1 in gB with channel count b (R = 1), the
        // general path in gB with b * R channels: the same layout
        const int lg = fft_lgcc(Px, C, es, 8);
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        const int nchunk = (C + (1 << lg) - 1) >> lg;
        const int ninv = nchunk * Ny;
        hipLaunchKernelGGL((k_inv_x_fin<T, In, Out>), dim3(ninv + nfin), blk, sh, st, gB, R, Nx, b, pl->fx, lg,
                           nchunk, y, accumulate, acc, ninv, reinterpret_cast<const cpx<T> *>(pl->rim_part),
                           OpPtrs<T>::C(pl), D, x, pl->N, Nr, pl->rim_nslab);
    }
    mark(6);
    mark(7);
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
hipError_t matvec_fp64_timed(tp_plan pl, Cols<const c128> x, Cols<c128> y, int R, hipStream_t st, hipEvent_t *ev) {
    return matvec_launch<double, c128, c128>(pl, x, y, R, st, ev);
}
hipError_t matvec_fp32_timed(tp_plan pl, Cols<const c64> x, Cols<c64> y, int R, hipStream_t st, hipEvent_t *ev) {
    return matvec_launch<float, c64, c64>(pl, x, y, R, st, ev);
}
hipError_t precond_fp64(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R, hipStream_t st) {
    return matvec_launch<double, c128, c128, true>(pl, x, y, R, st, nullptr, base);
}
hipError_t precond_fp32(tp_plan pl, Cols<const c64> x, Cols<c64> y, Cols<const c64> base, int R, hipStream_t st) {
    return matvec_launch<float, c64, c64, true>(pl, x, y, R, st, nullptr, base);
}
hipError_t precond_fp32_wide(tp_plan pl, Cols<const c128> x, Cols<c128> y, Cols<const c128> base, int R,
                             hipStream_t st) {
    return matvec_launch<float, c128, c128, true>(pl, x, y, R, st, nullptr, base);
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

hipError_t precond_build(tp_plan pl, c128 *S, int *flag, hipStream_t st) {
    const long P = (long)pl->Px * pl->Py;
    const double scl = 1.0 / ((double)P * (double)P);
    const size_t sh = (size_t)pl->b * (sizeof(c128) + sizeof(int));
    hipLaunchKernelGGL(k_block_inv, dim3((unsigned)P), dim3(256), sh, st, S, pl->b, scl, flag);
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

}  // namespace tp
