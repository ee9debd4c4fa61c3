#pragma once
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
//
// Symmetric generators (Z_{-m,-n} = Z_{m,n}^T) give Ghat(-k) = Ghat(k)^T, and
// the plan then stores the spectrum columns kx <= Px/2 only: the products read
// a mirrored frequency's block transposed, and the fused single-column path
// applies each stored block to both of its frequencies (spec_block_half).
#include "tp_fft.h"
#include "tp_mfma.h"
#include "tp_internal.h"

namespace tp {

// ------------------------------------------------------------------ helpers
template <typename T>
__device__ __forceinline__ cpx<T> wave_sum(cpx<T> v) {
    return wave_allsum(v);
}

template <typename T>
__device__ __forceinline__ void zero_lds(cpx<T> *buf, int n, int nt = kBlock) {
    for (int i = threadIdx.x; i < n; i += nt) buf[i] = mk<T>(0, 0);
}

// ------------------------------------------------------------ FFT passes
template <typename T, typename In>
__device__ __forceinline__ void fwd_x_body(Cols<const In> x, int R, int Nx, int b, const FFTDesc &fx, int lgCC,
                                           cpx<T> *__restrict__ out, const RimMap &rm, int bx, int by,
                                           char *smem_raw) {
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fx.P;
    const int CC = 1 << lgCC, C = b * R, P = fx.P;
    const int c0 = bx * CC, iy = by;
    if (!cols_live((const void *const *)x.tab, c0 / b, (min(c0 + CC, C) - 1) / b)) return;
    auto fetch = [&](int i, bool &ok) {
        const int ix = i >> lgCC, c = c0 + (i & (CC - 1));
        ok = false;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            const In *xc = x.col(r);
            const long j = xc ? cell_unknown(rm, iy * Nx + ix, p) : -1;
            if (j >= 0) {
                ok = true;
                return cvt<T>(xc[j]);
            }
        }
        return mk<T>(0, 0);
    };
    // the first value per thread is fetched before the twiddles and the
    // zero fill, so its round trip overlaps theirs
    bool ok0;
    const cpx<T> v0 = threadIdx.x < Nx * CC ? fetch(threadIdx.x, ok0) : (ok0 = false, mk<T>(0, 0));
    load_twiddles<T>(twl, fx);
    zero_lds<T>(buf, P * CC);
    __syncthreads();
    if (ok0) buf[(fx.perm[threadIdx.x >> lgCC] << lgCC) + (threadIdx.x & (CC - 1))] = v0;
    for (int i = threadIdx.x + kBlock; i < Nx * CC; i += kBlock) {
        bool ok;
        const cpx<T> v = fetch(i, ok);
        if (ok) buf[(fx.perm[i >> lgCC] << lgCC) + (i & (CC - 1))] = v;
    }
    __syncthreads();
    lds_fft<T, false>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < P * CC; i += kBlock) {
        const int k = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) out[((long)iy * P + k) * C + c] = buf[i];
    }
}

template <typename T, typename In>
__global__ void __launch_bounds__(256) k_fwd_x(Cols<const In> x, int R, int Nx, int b, FFTDesc fx,
                                               int lgCC, cpx<T> *__restrict__ out, RimMap rm) {
    extern __shared__ char smem_raw[];
    fwd_x_body<T, In>(x, R, Nx, b, fx, lgCC, out, rm, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T>
__device__ __forceinline__ void fwd_y_body(const cpx<T> *__restrict__ in, int C, int Ny, int Px, const FFTDesc &fy,
                                           int lgCC, cpx<T> *__restrict__ out, const void *const *act, int b,
                                           int bx, int by, char *smem_raw) {
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fy.P;
    const int CC = 1 << lgCC, P = fy.P;
    const int c0 = bx * CC, kx = by;
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
__global__ void __launch_bounds__(256) k_fwd_y(const cpx<T> *__restrict__ in, int C, int Ny, int Px,
                                               FFTDesc fy, int lgCC, cpx<T> *__restrict__ out,
                                               const void *const *act, int b) {
    extern __shared__ char smem_raw[];
    fwd_y_body<T>(in, C, Ny, Px, fy, lgCC, out, act, b, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T>
__device__ __forceinline__ void inv_y_body(const cpx<T> *__restrict__ in, int C, int Ny, int Px, const FFTDesc &fy,
                                           int lgCC, cpx<T> *__restrict__ out, const void *const *act, int b,
                                           int bx, int by, char *smem_raw) {
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = twl + fy.P;
    const int CC = 1 << lgCC, P = fy.P;
    const int c0 = bx * CC, kx = by;
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

template <typename T>
__global__ void __launch_bounds__(256) k_inv_y(const cpx<T> *__restrict__ in, int C, int Ny, int Px,
                                               FFTDesc fy, int lgCC, cpx<T> *__restrict__ out,
                                               const void *const *act, int b) {
    extern __shared__ char smem_raw[];
    inv_y_body<T>(in, C, Ny, Px, fy, lgCC, out, act, b, blockIdx.x, blockIdx.y, smem_raw);
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
                                              int b, int R, cpx<T> *__restrict__ out, const void *const *act,
                                              int Px, int Py, int kxh) {
    extern __shared__ char smem_raw[];
    cpx<T> *xs = reinterpret_cast<cpx<T> *>(smem_raw);   // [RC][b]
    const int C = b * R, r0 = blockIdx.y * RC;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kBlock >> 6;
    const long k = blockIdx.x;
    const int rn = min(RC, R - r0);
    if (!cols_live(act, r0, r0 + rn - 1)) return;
    const int pl = lane >> 3, qs = (lane & 7) * VPL;
    // a mirrored frequency reads its stored block transposed
    bool tr;
    const cpx<T> *Gk = G + spec_src(k, Px, Py, kxh, tr) * (long)b * b;
    const long sp = tr ? 1 : b, sq = tr ? b : 1;
    const int npanel = (b + 7) >> 3;
    cpx<T> gc[VPL], gn[VPL];
    auto load = [&](cpx<T>(&g)[VPL], int panel) {
        const int p = panel * 8 + pl;
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            const int q = qs + v;
            g[v] = (panel < npanel && p < b && q < b) ? Gk[p * sp + q * sq] : mk<T>(0, 0);
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
            acc[c] = sum8(acc[c]);
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
    // The prologue's own loads (tables, the first 8 input values per thread)
    // all issue together; the first panels follow the transform (issued
    // earlier, they hold the waves at the load queue until the memory system
    // has served the panels of every workgroup).
    const int t = threadIdx.x, nx = Ny * CC;
    const cpx<T> *tw = tw_of<T>(fy);
    const cpx<T> tw0 = tw[min(t, P - 1)], tw1 = tw[min(t + kBlock, P - 1)];
    const int pm0 = fy.perm[min(t, P - 1)], pm1 = fy.perm[min(t + kBlock, P - 1)];
    auto xload = [&](int i) { return X1[((long)(i >> lgCC) * Px + kx) * b + min(i & (CC - 1), b - 1)]; };
    cpx<T> xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = xload(min(t + u * kBlock, nx - 1));
    zero_lds<T>(xs, P * CC);
    if (t < P) {
        twl[t] = tw0;
        perm[t] = pm0;
    }
    if (t + kBlock < P) {
        twl[t + kBlock] = tw1;
        perm[t + kBlock] = pm1;
    }
    __syncthreads();
    auto xstore = [&](int i, cpx<T> v) {
        const int iy = i >> lgCC, c = i & (CC - 1);
        if (c < b) xs[(perm[iy] << lgCC) + c] = v;
    };
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (t + u * kBlock < nx) xstore(t + u * kBlock, xv[u]);
    if (nx > 8 * kBlock)
        batched<8, cpx<T>>(
            nx - 8 * kBlock, [&](int i) { return xload(i + 8 * kBlock); },
            [&](int i, cpx<T> v) { xstore(i + 8 * kBlock, v); });
    __syncthreads();
    lds_fft<T, false>(xs, lgCC, fy, twl);
    load(gc, w);
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

// Sum v[0..V) (V a power of two) over the 8 lanes that share lane & 7 (lane
// bits 3..5), leaving each lane a share of the totals.  While more than one
// value is left, a step on lane bit 5, 4, 3 keeps the half of the values that
// the lane's bit selects and adds the partner's copy of that half; remaining
// bits take plain sums.  With S = min(3, log2 V) halving steps and
// g = (lane >> 3) >> (3 - S), v[i] (i < max(V / 8, 1)) ends up holding the
// total of value i + (V >> S) g; for V < 8 the lanes with (lane >> 3) not a
// multiple of 2^(3 - S) hold copies.
template <int V>
struct RS8 {
    static constexpr int S = V >= 8 ? 3 : V >= 4 ? 2 : V >= 2 ? 1 : 0;
    static constexpr int NV = V >= 8 ? V / 8 : 1;
};
template <typename T, int V, int STEP = 0>
__device__ __forceinline__ void rs8(cpx<T> (&v)[V], int lane) {
    constexpr int bit = 32 >> STEP;
    if constexpr (STEP < RS8<V>::S) {
        constexpr int h = V >> (STEP + 1);
#pragma unroll
        for (int i = 0; i < h; ++i) {
            if constexpr (bit == 8) {
                const bool hi = (lane & bit) != 0;
                const cpx<T> send = hi ? v[i] : v[i + h];
                const cpx<T> kept = hi ? v[i + h] : v[i];
                v[i] = kept + dpp<kDppRor8>(send);
            } else {
                v[i] = half_sum<bit>(v[i], v[i + h]);   // permlane swap of the two halves
            }
        }
    } else {
        v[0] = xor_sum<bit>(v[0]);
    }
    if constexpr (STEP < 2) rs8<T, V, STEP + 1>(v, lane);
}

constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// ------------------------------------ one column, half spectrum: pair stream
// The per-frequency product of one column over a half spectrum with the y
// transforms in passes of their own (no transform work inside): workgroup =
// one stored block s = (kx, ky), kx < kxh.  The block is read once and applied
// to its own frequency, yhat(kx, ky) = G xhat(kx, ky), and, when its mirror
// frequency (Px - kx, -ky) is not stored, transposed to it: yhat(-k) =
// G^T xhat(-k).  Wave w takes rows p = 8 w .. 8 w + 7 with 8 lanes per row;
// lane l holds G[p][q] for q = (l & 7) + 8 v, v < VPL, so that each load
// instruction of a wave reads 8 contiguous runs of 8 values (whole cache
// lines for FP64, half lines for FP32).  Row sums add the 8 lanes of a row
// (DPP); column sums add the 8 rows of a wave (rs8) and then the waves, in
// wave order, in LDS.  One workgroup per stored block
// keeps the stream balanced over the compute units whatever the block width;
// every block's loads issue before anything else.
template <typename T, int VPL>
__device__ __forceinline__ void pair_prod_body(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in, int b,
                                               int Px, int Py, int kxh, cpx<T> *__restrict__ out,
                                               const void *const *act, int bx, char *smem_raw) {
    constexpr int VP = pow2_at_least(VPL), S = RS8<VP>::S, NV = RS8<VP>::NV;
    if (!cols_live(act, 0, 0)) return;                 // an idle column (solver phases)
    const int nw = blockDim.x >> 6;
    cpx<T> *xk = reinterpret_cast<cpx<T> *>(smem_raw);   // [b] xhat(k)
    cpx<T> *xm = xk + b;                                   // [b] xhat(-k)
    cpx<T> *zp = xm + b;                                   // [nw][b] column sums per wave
    const int s = bx;
    const int kx = s / Py, ky = s - kx * Py;
    const bool mir = kx > 0 && Px - kx >= kxh;
    const long k = (long)kx * Py + ky;
    const long km = (long)(Px - kx) * Py + (ky == 0 ? 0 : Py - ky);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pl = lane >> 3, qj = lane & 7, p = w * 8 + pl;
    const bool prow = p < b;
    const cpx<T> *Grow = G + (long)s * b * b + (long)min(p, b - 1) * b;
    cpx<T> g[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) g[v] = Grow[min(qj + 8 * v, b - 1)];
    for (int i = threadIdx.x; i < b; i += blockDim.x) {
        xk[i] = in[k * b + i];
        if (mir) xm[i] = in[km * b + i];
    }
    __syncthreads();
    bool qok[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) qok[v] = prow && qj + 8 * v < b;
    cpx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc = cmac(acc, keep(g[v], qok[v]), xk[min(qj + 8 * v, b - 1)]);
    acc = sum8(acc);
    if ((lane & 7) == 0 && prow) out[k * b + p] = acc;
    if (!mir) return;                                  // uniform over the workgroup
    const cpx<T> xv = xm[min(p, b - 1)];
    cpx<T> m[VP];
#pragma unroll
    for (int v = 0; v < VP; ++v) m[v] = v < VPL ? keep(g[v], qok[v]) * xv : mk<T>(0, 0);
    rs8<T, VP>(m, lane);
    const int grp = pl >> (3 - S);
    const bool writer = (pl & ((1 << (3 - S)) - 1)) == 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int v = i + (VP >> S) * grp;
        if (writer && v < VPL && qj + 8 * v < b) zp[w * b + qj + 8 * v] = m[i];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < b; q += blockDim.x) {
        cpx<T> t = zp[q];
        for (int u = 1; u < nw; ++u) t = t + zp[u * b + q];
        out[km * b + q] = t;
    }
}

template <typename T, int VPL>
__global__ void __launch_bounds__(1024) k_pair_prod(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in,
                                                    int b, int Px, int Py, int kxh, cpx<T> *__restrict__ out,
                                                    const void *const *act) {
    extern __shared__ char smem_raw[];
    pair_prod_body<T, VPL>(G, in, b, Px, Py, kxh, out, act, blockIdx.x, smem_raw);
}


// Fused single-column path over half the spectrum.  A symmetric operator
// (Z_{-m,-n} = Z_{m,n}^T, Sec. II-B) has Ghat(-k) = Ghat(k)^T, and the plan
// stores the columns kx < kxh = Px / 2 + 1 only.  Workgroup = stored column kx
// and 8 rows p0..p0+7:
//   * rows p0..p0+7 of yhat(kx, .) as in spec_block;
//   * for the mirror column kxm = Px - kx (when it differs from kx), the part
//     of yhat(kxm, -ky) = Ghat(kx, ky)^T xhat(kxm, -ky) that the 8 rows give,
//     for every channel q: lanes form G[p][q] xhat(kxm, -ky)[p] and the 8
//     lanes of a channel sum them (rs8).  The part is inverse-transformed
//     along y here; the inverse x pass adds the nchunk parts.
// The forward y transforms run in decimation-in-frequency order, so xhat(ky)
// sits in LDS row perm[ky], the slot the inverse transform reads ky from.
// Wave w takes the frequency pairs {j, -j}, j = w, w + 4, ... (j <= Py / 2), so
// the mirror outputs of a pair go to the pair's own two rows, which no other
// wave touches: they overwrite xhat(kx, .) there once both forward products
// have read it.
template <typename T, int VPL, int UP, int NT>
__device__ __forceinline__ void spec_block_half(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ X1,
                                                cpx<T> *__restrict__ Y1, cpx<T> *__restrict__ Yp, int b, int Ny,
                                                int Px, int kxh, const FFTDesc &fy, int lgCC, int blk, char *smem) {
    constexpr int TP = 8, VP = pow2_at_least(VPL), S = RS8<VP>::S, NV = RS8<VP>::NV;
    const int P = fy.P, CC = 1 << lgCC;
    const int nchunk = (b + TP - 1) / TP;
    const int kx = blk / nchunk, ch = blk - kx * nchunk, p0 = ch * TP;
    const int kxm = kx == 0 ? 0 : Px - kx;
    const bool mir = kxm != kx;
    cpx<T> *twl = reinterpret_cast<cpx<T> *>(smem);
    cpx<T> *xs = twl + P;          // [Py][CC] xhat(kx, .), then the mirror part
    cpx<T> *ys = xs + P * CC;      // [Py][TP] rows p0.. of yhat(kx, .)
    cpx<T> *xm = ys + P * TP;      // [Py][TP] channels p0.. of xhat(kxm, .)
    int *perm = reinterpret_cast<int *>(xm + P * TP);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = NT >> 6;
    const int pl = lane >> 3, qs = (lane & 7) * VPL, p = p0 + pl;
    const bool prow = p < b;
    const long kstride = (long)b * b;
    const cpx<T> *Grow = G + (long)kx * P * kstride + (long)min(p, b - 1) * b;
    const int npair = P / 2 + 1;
    // a register buffer holds the two panels of each of UP pairs (the wave's
    // pairs j, j + 4, ...); clamped addresses (no branches around the loads)
    cpx<T> gc[2 * UP][VPL], gn[2 * UP][VPL];
    auto load = [&](cpx<T>(&g)[2 * UP][VPL], int j0) {
#pragma unroll
        for (int up = 0; up < UP; ++up) {
            const int ja = min(j0 + up * nw, npair - 1), jb = ja == 0 ? 0 : P - ja;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                g[2 * up][v] = Grow[ja * kstride + min(qs + v, b - 1)];
                g[2 * up + 1][v] = Grow[jb * kstride + min(qs + v, b - 1)];
            }
        }
    };
    // The prologue's own loads (tables, the first input values of both
    // columns) all issue together; the first panels follow the transforms
    // (issued earlier, they hold the waves at the load queue until the
    // memory system has served the panels of every workgroup).  Inputs go in
    // natural order: rows iy < Ny of column kx (all channels) and of column
    // kxm (channels p0..p0+7).
    const int t = threadIdx.x, nx = Ny * CC, nxm = mir ? Ny * TP : 0;
    const cpx<T> *tw = tw_of<T>(fy);
    const cpx<T> tw0 = tw[min(t, P - 1)], tw1 = tw[min(t + NT, P - 1)];
    const int pm0 = fy.perm[min(t, P - 1)], pm1 = fy.perm[min(t + NT, P - 1)];
    auto xload = [&](int i) { return X1[((long)(i >> lgCC) * Px + kx) * b + min(i & (CC - 1), b - 1)]; };
    auto mload = [&](int i) { return X1[((long)(i >> 3) * Px + kxm) * b + min(p0 + (i & (TP - 1)), b - 1)]; };
    constexpr int XU = NT >= 2048 ? 1 : 2048 / NT;   // first-round input values per thread
    cpx<T> xv[XU];
#pragma unroll
    for (int u = 0; u < XU; ++u) xv[u] = xload(min(t + u * NT, nx - 1));
    const cpx<T> mv = mload(min(t, Ny * TP - 1));
    zero_lds<T>(xs, P * CC, NT);
    if (mir) zero_lds<T>(xm, P * TP, NT);
    if (t < P) {
        twl[t] = tw0;
        perm[t] = pm0;
    }
    if (t + NT < P) {
        twl[t + NT] = tw1;
        perm[t + NT] = pm1;
    }
    __syncthreads();
    auto xstore = [&](int i, cpx<T> v) {
        if ((i & (CC - 1)) < b) xs[i] = v;
    };
    auto mstore = [&](int i, cpx<T> v) {
        if (p0 + (i & (TP - 1)) < b) xm[i] = v;
    };
#pragma unroll
    for (int u = 0; u < XU; ++u)
        if (t + u * NT < nx) xstore(t + u * NT, xv[u]);
    if (t < nxm) mstore(t, mv);
    if (nx > XU * NT)
        batched<8, cpx<T>>(
            nx - XU * NT, [&](int i) { return xload(i + XU * NT); },
            [&](int i, cpx<T> v) { xstore(i + XU * NT, v); }, NT);
    if (nxm > NT)
        batched<8, cpx<T>>(
            nxm - NT, [&](int i) { return mload(i + NT); }, [&](int i, cpx<T> v) { mstore(i + NT, v); }, NT);
    __syncthreads();
    // (only the b real channels of the CC-wide rows are transformed)
    lds_fft2<T, false, true, NT>(xs, lgCC, b, mir ? xm : nullptr, 3, TP, fy, twl);
    load(gc, w);
    bool qok[VPL];
    int qi[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        qok[v] = prow && qs + v < b;
        qi[v] = min(qs + v, CC - 1);
    }
    const int grp = pl >> (3 - S);
    const bool writer = (pl & ((1 << (3 - S)) - 1)) == 0;
    auto reduce_pair = [&](const cpx<T>(&g)[2 * UP][VPL], int up, int j) {
        const bool aok = j < npair;
        const int ja = min(j, npair - 1), jb = ja == 0 ? 0 : P - ja;
        const bool bok = aok && jb != ja;
        const int ra = perm[ja], rb = perm[jb];
        cpx<T> acc[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const cpx<T> *xk = xs + ((u ? rb : ra) << lgCC);
            cpx<T> a = mk<T>(0, 0);
#pragma unroll
            for (int v = 0; v < VPL; ++v) a = cmac(a, keep(g[2 * up + u][v], qok[v]), xk[qi[v]]);
            acc[u] = sum8(a);
        }
        cpx<T> mo[2][NV];
        if (mir) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                // panel u's mirror frequency is the other member of the pair
                const cpx<T> xv = xm[((u ? ra : rb) << 3) + pl];
                cpx<T> m[VP];
#pragma unroll
                for (int v = 0; v < VP; ++v) m[v] = v < VPL ? keep(g[2 * up + u][v], qok[v]) * xv : mk<T>(0, 0);
                rs8<T, VP>(m, lane);
#pragma unroll
                for (int i = 0; i < NV; ++i) mo[u][i] = m[i];
            }
        }
        // rows ra and rb have been read above; from here on they are written
        if ((lane & 7) == 0) {
            if (aok) ys[(ra << 3) + pl] = acc[0];
            if (bok) ys[(rb << 3) + pl] = acc[1];
        }
        if (mir) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const bool ok = (u ? bok : aok) && writer;
                cpx<T> *row = xs + ((u ? ra : rb) << lgCC);
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    const int v = i + (VP >> S) * grp;
                    if (ok && v < VPL && qs + v < b) row[qs + v] = mo[u][i];
                }
            }
        }
    };
    auto reduce = [&](const cpx<T>(&g)[2 * UP][VPL], int j0) {
#pragma unroll
        for (int up = 0; up < UP; ++up) reduce_pair(g, up, j0 + up * nw);
    };
    // two register buffers in turn, loads unconditional (see spec_block)
    // Buffer tb of this wave holds its pairs j = w + tb UP nw + up nw.  The
    // steady loop issues no load past the wave's last buffer; the one or two
    // buffers left are reduced after it (a uniform branch with nothing
    // pending behind it).
    const int bstep = UP * nw;
    const int nbuf = npair > w ? (npair - w + bstep - 1) / bstep : 0;
    int tb = 0;
    for (; tb + 2 < nbuf; tb += 2) {
        load(gn, w + (tb + 1) * bstep);
        reduce(gc, w + tb * bstep);
        load(gc, w + (tb + 2) * bstep);
        reduce(gn, w + (tb + 1) * bstep);
    }
    if (nbuf - tb == 2) {
        load(gn, w + (tb + 1) * bstep);
        reduce(gc, w + tb * bstep);
        reduce(gn, w + (tb + 1) * bstep);
    } else if (nbuf - tb == 1) {
        reduce(gc, w + tb * bstep);
    }
    __syncthreads();
    lds_fft2<T, true, false, NT>(ys, 3, TP, mir ? xs : nullptr, lgCC, b, fy, twl);
    for (int i = threadIdx.x; i < Ny * TP; i += NT) {
        const int iy = i >> 3, pr = i & 7, pp = p0 + pr;
        if (pp < b) Y1[((long)iy * Px + kx) * b + pp] = ys[i];
    }
    if (mir) {
        const int nmir = Px - kxh;
        cpx<T> *yp = Yp + ((long)ch * Ny * nmir + (kxm - kxh)) * b;
        for (int i = threadIdx.x; i < Ny * CC; i += NT) {
            const int iy = i >> lgCC, q = i & (CC - 1);
            if (q < b) yp[(long)iy * nmir * b + q] = xs[i];
        }
    }
}

// Rim pass for a single column.  Slab = TE = 64 E element columns x all Nr
// rows; 16 lanes per row: lane l takes row offset l >> 4 of each group of 4
// rows and the VE = 4 E columns [(l & 15) VE, (l & 15) VE + VE) of the slab,
// so a group of 4 rows is 4 contiguous TE-column runs.  Per row the 16 lanes
// add up sum_e B[row][e] x_A[e] (-> slab partial of y_r); every lane keeps
// sum_row BE[row][e] x_r[row] for its columns, and those are summed over the
// row lanes and the waves at the end (-> y_A).  A register buffer holds UR
// groups (the wave's next UR groups); the next buffer's loads are issued
// before the current one is used.
template <typename T, typename In, typename Out, int E, bool NBE, int UR>
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
    constexpr int NE = NBE ? VE : 1;
    const int step = nw * 4, bstep = UR * step;   // rows between a wave's groups, between buffers
    cpx<T> gc[UR][VE], gn[UR][VE], ec[UR][NE], en[UR][NE];
    auto load = [&](cpx<T>(&g)[UR][VE], cpx<T>(&ge)[UR][NE], int row) {
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const long rr = (long)min(row + u * step, Nr - 1) * N;
#pragma unroll
            for (int v = 0; v < VE; ++v) {
                g[u][v] = B[rr + ei[v]];
                if constexpr (NBE) ge[u][v] = BE[rr + ei[v]];
            }
        }
    };
    auto rows = [&](const cpx<T>(&g)[UR][VE], const cpx<T>(&ge)[UR][NE], int row0) {
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int row = row0 + u * step;
            cpx<T> sr = mk<T>(0, 0);
            const bool rok = row < Nr;
            const cpx<T> xrow = xr[min(row, Nr - 1)];
#pragma unroll
            for (int v = 0; v < VE; ++v) {
                const cpx<T> gv = keep(g[u][v], rok && eok[v]);
                sr = cmac(sr, gv, xa[v]);
                acc[v] = cmac(acc[v], NBE ? keep(ge[u][NBE ? v : 0], rok && eok[v]) : gv, xrow);
            }
            sr = xor_sum<8>(sr);
            sr = sum8(sr);
            if ((lane & 15) == 0 && rok) part[(long)slab * Nr + row] = sr;
        }
    };
    // groups of 4 rows; two register buffers in turn, loads unconditional
    // (see the spectrum stream)
    const int r0 = w * 4 + ro;
    load(gc, ec, r0);
    for (int g0 = w * 4; g0 < Nr; g0 += 2 * bstep) {
        const int row = r0 + (g0 - w * 4);
        load(gn, en, row + bstep);
        rows(gc, ec, row);
        load(gc, ec, row + 2 * bstep);
        if (g0 + bstep < Nr) rows(gn, en, row + bstep);
    }
    // sum the four row lanes of each column, then the waves
#pragma unroll
    for (int v = 0; v < VE; ++v) {
        acc[v] = xor_sum<16>(acc[v]);
        acc[v] = xor_sum<32>(acc[v]);
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

// Which task a workgroup of the fused launch takes.  Workgroups are dealt to
// the 8 XCDs in turn (XCD x runs blocks x, x + 8, ...), and each XCD has its
// own share of the memory bandwidth, so every XCD gets the same mix: XCD x
// takes s_x of the nspec spectrum tasks, spread evenly over its sequence of
// blocks, and rim tasks in between.  Then the rim streams of an XCD keep its
// bandwidth busy while its spectrum workgroups transform.  The spectrum tasks
// of an XCD are consecutive (the row chunks of one column share its input).
__device__ __forceinline__ void block_task(int i, int nspec, int nrim, int &spec_id, int &rim_id) {
    const int ntot = nspec + nrim, x = i & 7, q = i >> 3;
    const int nq = (ntot - x + 7) >> 3;                       // blocks on XCD x
    int c0 = 0;                                               // blocks on the XCDs before x
    for (int xx = 0; xx < x; ++xx) c0 += (ntot - xx + 7) >> 3;
    // spectrum tasks in proportion to the blocks: s0 before XCD x, sx on it
    auto share = [&](int c) { return (int)((long)nspec * c / ntot); };
    const int s0 = share(c0), sx = share(c0 + nq) - s0;
    auto specs = [&](int qq) { return (int)((long)qq * sx / nq); };   // among its first qq blocks
    const int before = specs(q), upto = specs(q + 1);
    if (upto > before) {
        spec_id = s0 + before;
        rim_id = -1;
    } else {
        spec_id = -1;
        rim_id = (c0 - s0) + (q - before);
    }
}

// Spectrum workgroups and rim workgroups share one launch so that both HBM
// streams (the spectrum and the dense rim) run together; the two kinds are
// interleaved in block order.
template <typename T, typename In, typename Out, int VPL, int U, int E, bool NBE, bool HALF, int NT = kBlock>
__global__ void __launch_bounds__(NT) k_spec_rim(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ X1,
                                                  cpx<T> *__restrict__ Y1, int b, int Ny, int Px, FFTDesc fy,
                                                  int lgCC, int nspec, const cpx<T> *__restrict__ B,
                                                  const cpx<T> *__restrict__ BE, Cols<const In> x, Cols<Out> y,
                                                  long N, int Nr, cpx<T> *__restrict__ part, int nrim,
                                                  cpx<T> *__restrict__ Yp, int kxh) {
    extern __shared__ char smem_raw[];
    int spec_id, rim_id;
    if constexpr (sizeof(T) == 4) {
        block_task(blockIdx.x, nspec, nrim, spec_id, rim_id);
    } else {
        // FP64 (two waves per SIMD, not every workgroup resident at once):
        // spectrum and rim tasks alternate in block order
        const int i = blockIdx.x, both = 2 * min(nspec, nrim);
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
    }
    if (spec_id >= 0) {
        if (!cols_live((const void *const *)x.tab, 0, 0)) return;
        // without the rim pass the spectrum stream alone must keep HBM busy:
        // two pairs per register buffer (FP32, 8-wave workgroups)
        if constexpr (HALF)
            spec_block_half<T, VPL, (E == 0 && sizeof(T) == 4 && NT == 512) ? 2 : 1, NT>(
                G, X1, Y1, Yp, b, Ny, Px, kxh, fy, lgCC, spec_id, smem_raw);
        else
            spec_block<T, VPL, U>(G, X1, Y1, b, Ny, Px, fy, lgCC, spec_id, smem_raw);
    } else if constexpr (E > 0) {
        // two groups per buffer for FP32 slabs of up to 128 columns (the
        // register budget of wider slabs and of FP64 holds one)
        rim_block1<T, In, Out, E, NBE, (sizeof(T) == 4 && E <= 2) ? 2 : 1>(B, BE, x, y, N, Nr, part, rim_id,
                                                                          smem_raw);
    }
}

// Inverse x transform + crop (+ rim term already in y), and the rim finish
// waves, in one launch: blocks [0, ninv) transform, the rest finish rim rows.
// Mirror parts of the half-spectrum single-column path: columns kx >= kxh of
// the y-transformed grid are the sum over nch parts, part h of (iy, kx, c) at
// yp[h * hstride + (iy * nmir + kx - kxh) * b + c].
template <typename T>
struct MirrorParts {
    const cpx<T> *yp;
    int kxh, nmir, nch;
    long hstride;
};

template <typename T, typename In, typename Out>
__device__ __forceinline__ void inv_x_fin_body(const cpx<T> *__restrict__ in, int R, int Nx, int b,
                                               const FFTDesc &fx, int lgCC, int nchunk, Cols<Out> y, int accumulate,
                                               Cols<const Out> acc, int ninv, const cpx<T> *__restrict__ part,
                                               const cpx<T> *__restrict__ Cm, const cpx<T> *__restrict__ D,
                                               Cols<const In> x, long N, int Nr, int nslab, const MirrorParts<T> &mp,
                                               const RimMap &rm, int blk, char *smem_raw) {
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
    auto gather = [&](int i) {
        const int kx = i >> lgCC, c = c0 + (i & (CC - 1));
        cpx<T> v = mk<T>(0, 0);
        if (c < C) {
            if (mp.yp && kx >= mp.kxh) {
                // all parts in flight at once (nch <= 12: rows of at most 96),
                // then added in part order
                const cpx<T> *src = mp.yp + ((long)iy * mp.nmir + (kx - mp.kxh)) * b + c;
                cpx<T> pv[12];
#pragma unroll
                for (int h = 0; h < 12; ++h) pv[h] = h < mp.nch ? src[h * mp.hstride] : mk<T>(0, 0);
#pragma unroll
                for (int h = 0; h < 12; ++h)
                    if (h < mp.nch) v = v + pv[h];
            } else {
                v = in[((long)iy * P + kx) * C + c];
            }
        }
        return v;
    };
    // the first two values per thread are fetched before the twiddles, so
    // both round trips overlap
    cpx<T> pre[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = threadIdx.x + j * kBlock;
        pre[j] = i < P * CC ? gather(i) : mk<T>(0, 0);
    }
    load_twiddles<T>(twl, fx);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = threadIdx.x + j * kBlock;
        if (i < P * CC) buf[(fx.perm[i >> lgCC] << lgCC) + (i & (CC - 1))] = pre[j];
    }
    for (int i = threadIdx.x + 2 * kBlock; i < P * CC; i += kBlock)
        buf[(fx.perm[i >> lgCC] << lgCC) + (i & (CC - 1))] = gather(i);
    __syncthreads();
    lds_fft<T, true>(buf, lgCC, fx, twl);
    for (int i = threadIdx.x; i < Nx * CC; i += kBlock) {
        const int ix = i >> lgCC, cl = i & (CC - 1), c = c0 + cl;
        if (c < C) {
            const int r = c / b, p = c - r * b;
            Out *yc = y.col(r);
            if (!yc) continue;
            const long e = cell_unknown(rm, iy * Nx + ix, p);
            if (e < 0) continue;
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

template <typename T, typename In, typename Out>
__global__ void __launch_bounds__(256) k_inv_x_fin(const cpx<T> *__restrict__ in, int R, int Nx, int b, FFTDesc fx,
                                                   int lgCC, int nchunk, Cols<Out> y, int accumulate,
                                                   Cols<const Out> acc, int ninv, const cpx<T> *__restrict__ part,
                                                   const cpx<T> *__restrict__ Cm, const cpx<T> *__restrict__ D,
                                                   Cols<const In> x, long N, int Nr, int nslab, MirrorParts<T> mp,
                                                   RimMap rm) {
    extern __shared__ char smem_raw[];
    inv_x_fin_body<T, In, Out>(in, R, Nx, b, fx, lgCC, nchunk, y, accumulate, acc, ninv, part, Cm, D, x, N, Nr,
                               nslab, mp, rm, blockIdx.x, smem_raw);
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
__device__ __forceinline__ void fft2_fwd_tile(Cols<const In> x, int R, int Nx, int Ny, int b, const FFTDesc &fx,
                                              const FFTDesc &fy, int lgCC, int XS, cpx<T> *__restrict__ out,
                                              const RimMap &rm, int blk, char *smem_raw) {
    cpx<T> *twx = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *twy = twx + fx.P;
    cpx<T> *buf = twy + fy.P;
    int *px = reinterpret_cast<int *>(buf + fx.P * XS);   // digit-reversal tables
    int *py = px + fx.P;
    const int CC = 1 << lgCC, C = b * R, Px = fx.P, Py = fy.P;
    const int c0 = blk * CC;
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
        const int p = c % b;
        if (xc && p >= rm.be) {
            // a rim channel: the rim functions placed at this channel's cells
            const int es = kBlock >> lgCC, ne = Nx * Ny;
            const float rNx = 1.0f / (float)Nx;
            for (int e = threadIdx.x >> lgCC; e < ne; e += es) {
                const long j = cell_unknown(rm, e, p);
                if (j >= 0) {
                    int ix;
                    const int iy = small_divmod(e, Nx, rNx, ix);
                    buf[px[ix] * XS + (py[iy] << lgCC) + cl] = cvt<T>(ldg(xc + j));
                }
            }
        } else if (xc) {
            xc += p;
            const int es = kBlock >> lgCC, ne = Nx * Ny;
            const float rNx = 1.0f / (float)Nx;
            for (int eb = threadIdx.x >> lgCC; eb < ne; eb += 8 * es) {
                In v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = ldg(xc + (long)min(eb + u * es, ne - 1) * rm.be);
#pragma unroll
                for (int u = 0; u < 8; ++u) pin(v[u]);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = eb + u * es;
                    if (e < ne) {
                        int ix;
                    const int iy = small_divmod(e, Nx, rNx, ix);
                        buf[px[ix] * XS + (py[iy] << lgCC) + cl] = cvt<T>(v[u]);
                    }
                }
            }
        }
    }
    __syncthreads();
    // x first, on the Ny rows that hold data (at their digit-reversed y
    // positions), then y on every column
    lds_fft_axis<T, false>(buf, lgCC, fx, XS, Ny, CC, twx, py);
    lds_fft_axis<T, false>(buf, lgCC, fy, CC, Px, XS, twy);
    // frequency k = kx Py + ky of item i, stepped without a division per item
    const int kst = kBlock >> lgCC, cl = threadIdx.x & (CC - 1), c = c0 + cl;
    int kx = (threadIdx.x >> lgCC) / Py, ky = (threadIdx.x >> lgCC) - kx * Py;
    for (int i = threadIdx.x; i < Px * Py * CC; i += kBlock) {
        const int k = i >> lgCC;
        if (c < C) out[(long)k * C + c] = buf[kx * XS + (ky << lgCC) + cl];
        ky += kst;
        while (ky >= Py) {
            ky -= Py;
            ++kx;
        }
    }
}

template <typename T, typename In>
__global__ void __launch_bounds__(256) k_fft2_fwd(Cols<const In> x, int R, int Nx, int Ny, int b, FFTDesc fx,
                                                  FFTDesc fy, int lgCC, int XS, cpx<T> *__restrict__ out,
                                                  RimMap rm) {
    extern __shared__ char smem_raw[];
    fft2_fwd_tile<T, In>(x, R, Nx, Ny, b, fx, fy, lgCC, XS, out, rm, blockIdx.x, smem_raw);
}

template <typename T, typename In, typename Out>
__device__ __forceinline__ void fft2_inv_tile(const cpx<T> *__restrict__ in, int R, int Nx, int Ny, int b,
                                              const FFTDesc &fx, const FFTDesc &fy, int lgCC, int XS, Cols<Out> y,
                                              int accumulate, Cols<const Out> acc, int ninv,
                                              const cpx<T> *__restrict__ part, const cpx<T> *__restrict__ Cm,
                                              const cpx<T> *__restrict__ D, Cols<const In> x, long N, int Nr,
                                              int nslab, const RimMap &rm, int blk, char *smem_raw) {
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
    const float rPy = 1.0f / (float)Py;
    batched<8, cpx<T>>(
        Px * Py * CC, [&](int i) { return in[(long)(i >> lgCC) * C + min(c0 + (i & (CC - 1)), C - 1)]; },
        [&](int i, cpx<T> v) {
            const int k = i >> lgCC, cl = i & (CC - 1);
            int ky;
            const int kx = small_divmod(k, Py, rPy, ky);
            buf[px[kx] * XS + (py[ky] << lgCC) + cl] = c0 + cl < C ? v : mk<T>(0, 0);
        });
    __syncthreads();
    lds_fft_axis<T, true>(buf, lgCC, fy, CC, Px, XS, twy);
    lds_fft_axis<T, true>(buf, lgCC, fx, XS, Ny, CC, twx);
    const int cl = threadIdx.x & (CC - 1), c = c0 + cl;
    Out *yc = c < C ? y.col(c / b) : nullptr;
    if (!yc) return;
    const int p = c % b;
    const Out *ac = accumulate ? acc.col(c / b) : nullptr;
    const int es = kBlock >> lgCC, ne = Nx * Ny;
            const float rNx = 1.0f / (float)Nx;
    if (p >= rm.be) {
        // a rim channel: results of the rim functions placed at its cells
        for (int e = threadIdx.x >> lgCC; e < ne; e += es) {
            const long j = cell_unknown(rm, e, p);
            if (j >= 0) {
                int ix;
                    const int iy = small_divmod(e, Nx, rNx, ix);
                Out v = cvt<typename Out::value_type>(buf[ix * XS + (iy << lgCC) + cl]);
                if (ac) v = v + ldg(ac + j);
                stg(yc + j, v);
            }
        }
        return;
    }
    yc += p;
    if (ac) ac += p;
    for (int eb = threadIdx.x >> lgCC; eb < ne; eb += 8 * es) {
        Out old[8];
        if (ac) {
#pragma unroll
            for (int u = 0; u < 8; ++u) old[u] = ldg(ac + (long)min(eb + u * es, ne - 1) * rm.be);
#pragma unroll
            for (int u = 0; u < 8; ++u) pin(old[u]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = eb + u * es;
            if (e < ne) {
                int ix;
                    const int iy = small_divmod(e, Nx, rNx, ix);
                Out v = cvt<typename Out::value_type>(buf[ix * XS + (iy << lgCC) + cl]);
                if (ac) v = v + old[u];
                stg(yc + (long)e * rm.be, v);
            }
        }
    }
}

template <typename T, typename In, typename Out>
__global__ void __launch_bounds__(256) k_fft2_inv_fin(const cpx<T> *__restrict__ in, int R, int Nx, int Ny, int b,
                                                      FFTDesc fx, FFTDesc fy, int lgCC, int XS, Cols<Out> y,
                                                      int accumulate, Cols<const Out> acc, int ninv,
                                                      const cpx<T> *__restrict__ part,
                                                      const cpx<T> *__restrict__ Cm, const cpx<T> *__restrict__ D,
                                                      Cols<const In> x, long N, int Nr, int nslab, RimMap rm) {
    extern __shared__ char smem_raw[];
    fft2_inv_tile<T, In, Out>(in, R, Nx, Ny, b, fx, fy, lgCC, XS, y, accumulate, acc, ninv, part, Cm, D, x, N, Nr,
                              nslab, rm, blockIdx.x, smem_raw);
}

// ------------------------------------ many columns: one persistent launch
// The operator (or preconditioner) on 16+ columns of a grid small enough for
// the 2-D transform tiles, in one persistent launch: every workgroup takes
// tasks from a queue, in dependency order: the dense rim's matrix-core slabs,
// the forward 2-D tiles, the per-frequency products (after every forward
// tile), the inverse tiles (after every product and rim slab) and the rim
// finish (after every rim slab).  A task is taken only by a running workgroup
// and waits only on tasks earlier in the queue, which wait on nothing later,
// so every wait ends whatever the number of resident workgroups.  A task
// signals completion by its writes, a device-scope fence by every thread, a
// barrier and one atomic increment; a waiter spins on an acquire load of the
// counter and then fences before it reads (another XCD's L2 may hold stale
// lines of the previous application's buffers).  Each task runs the same body
// as its separate launch, so the results are the same bits.
// Counters: [0] queue head, [1] rim slabs done, [2] forward tiles done,
// [3] products done, [4] set when a wait gave up (it cannot happen unless
// the device stops running the workgroups that hold earlier tasks).
constexpr int kFusedCounters = 5;

// The dense rim's slabs (matrix cores) and the forward 2-D tiles in one
// launch: both only read x and they write disjoint buffers (the rim: y's
// element rows and the slab partials; the tiles: the transform grid), so no
// ordering is needed between them, and the rim's matrix-core work overlaps
// the latency-bound transforms.  Rim workgroups come first.
template <typename T, typename In, typename Out, bool NBE>
__global__ void __launch_bounds__(256) k_rim_fft2_fwd(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                                      Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                                      cpx<T> *__restrict__ part, int nslab, int nrim, int Nx, int Ny,
                                                      int b, FFTDesc fx, FFTDesc fy, int lgCC, int XS,
                                                      cpx<T> *__restrict__ out, RimMap rm) {
    extern __shared__ char smem_raw[];
    const int blk = blockIdx.x;
    if (blk < nrim)
        rim_mfma_tile<T, In, Out, rim_nt<T>(), rim_rch<T>(), NBE>(B, BE, x, y, R, N, Nr, part, blk % nslab,
                                                                  blk / nslab, smem_raw);
    else
        fft2_fwd_tile<T, In>(x, R, Nx, Ny, b, fx, fy, lgCC, XS, out, rm, blk - nrim, smem_raw);
}

static __global__ void k_zero_ints(int *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Completion counters of the persistent launch.  The wait spins on relaxed
// loads and takes one agent-scope acquire after the count is reached: an
// acquire load in the loop would invalidate the caches on every spin.  The
// signal makes each wave's writes visible at agent scope, then one thread
// adds to the counter with release order.
__device__ __forceinline__ void fused_wait(int *c, int target, int *err) {
    if (threadIdx.x == 0) {
        long spins = 0;
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1L << 22)) {    // seconds, far beyond any real wait: give up rather than hang
                atomicOr(err, 1);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__device__ __forceinline__ void fused_signal(int *c) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(c, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

struct FusedDims {
    int nslab, ncb_rim, nrim;     // rim slabs x column blocks
    int nfwd;                     // forward 2-D tiles
    int ncb, nprod;               // product column blocks, items (frequencies x column blocks)
    int ninv, nfin;               // inverse tiles, rim finish blocks
};

// Every stage of a many-column application in one persistent launch.  The
// workgroups take tasks from a queue in this order: dense rim slabs (slab x
// column block), forward 2-D tiles, matrix-core products (frequency x column
// block), inverse tiles, rim-row finish blocks.  A task depends only on tasks
// earlier in the queue (products on every forward tile, inverse tiles on
// every product and rim slab, finish blocks on the rim slabs), and a task is
// taken only by a running workgroup, so every wait ends.  Each task body is
// the device function of the separate launch, so results match it bit for
// bit.  Counters: [0] queue, [1] rim slabs, [2] forward tiles, [3] products,
// [4] set if a wait gave up (it never should).
template <typename T, typename In, typename Out, bool RIM>
__global__ void __launch_bounds__(256) k_fused_multi(
    Cols<const In> x, Cols<Out> y, int R, int Nx, int Ny, int b, FFTDesc fx, FFTDesc fy, int lgCC, int XS,
    cpx<T> *__restrict__ gA, cpx<T> *__restrict__ gB, const cpx<T> *__restrict__ G, int kxh,
    const cpx<T> *__restrict__ B, cpx<T> *__restrict__ part, const cpx<T> *__restrict__ Cm,
    const cpx<T> *__restrict__ D, int accumulate, Cols<const Out> acc, long N, int Nr, RimMap rm, FusedDims fd,
    int *ctr) {
    extern __shared__ char smem_raw[];
    __shared__ int task;
    constexpr int NTP = sizeof(T) == 4 ? 2 : 1;          // product column tiles (the default)
    const int Px = fx.P, Py = fy.P;
    const int e_rim = fd.nrim, e_fwd = e_rim + fd.nfwd, e_prod = e_fwd + fd.nprod,
              e_all = e_prod + fd.ninv + fd.nfin;
    const void *const *act = (const void *const *)x.tab;
    for (;;) {
        __syncthreads();                                  // LDS and `task` free again
        if (threadIdx.x == 0) task = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int t = task;
        if (t >= e_all) break;
        if (t < e_rim) {
            if constexpr (RIM) {
                rim_mfma_tile<T, In, Out, rim_nt<T>(), rim_rch<T>(), false>(B, B, x, y, R, N, Nr, part,
                                                                             t % fd.nslab, t / fd.nslab, smem_raw);
                fused_signal(&ctr[1]);
            }
        } else if (t < e_fwd) {
            fft2_fwd_tile<T, In>(x, R, Nx, Ny, b, fx, fy, lgCC, XS, gB, rm, t - e_rim, smem_raw);
            fused_signal(&ctr[2]);
        } else if (t < e_prod) {
            fused_wait(&ctr[2], fd.nfwd, &ctr[4]);
            const int item = t - e_fwd;
            const long k = item / fd.ncb;
            prod_mfma_item<T, NTP, 4, true>(G, gB, b, R, Px, Py, kxh, gA, act, k, (int)(item - k * fd.ncb),
                                            smem_raw);
            fused_signal(&ctr[3]);
        } else {
            const int blk = t - e_prod;
            if (blk < fd.ninv) fused_wait(&ctr[3], fd.nprod, &ctr[4]);
            if (RIM) fused_wait(&ctr[1], fd.nrim, &ctr[4]);
            fft2_inv_tile<T, In, Out>(gA, R, Nx, Ny, b, fx, fy, lgCC, XS, y, accumulate, acc, fd.ninv, part, Cm, D, x,
                                      N, Nr, fd.nslab, rm, blk, smem_raw);
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
static int fft2_lgcc(int Px, int Py, int C, size_t elem, size_t lds_cap = 48 * 1024) {
    constexpr int minlg = 2;   // tiles of 1 or 2 channels lose to the separate passes (63 x 63: 54 vs 39 us)
    auto bytes = [&](int lg) {
        return ((size_t)Px * fft2_xstride(Py, lg, elem) + Px + Py) * elem + (size_t)(Px + Py) * sizeof(int);
    };
    int lg = TP_FFT2_MAXLG;
    while (lg >= minlg && bytes(lg) > lds_cap) --lg;
    if (lg < minlg) return -1;
    while (lg > minlg && (1 << (lg - 1)) >= C) --lg;
    return lg;
}

// channels per workgroup (at most) of the separate x and y transform passes:
// the x pass takes 16 where that still leaves 1024 or more workgroups (longer
// contiguous runs per row; measured 10-25 % faster on 384-1024 channels),
// else 8 (a single column on the 63 x 63 grid loses with 16: fewer workgroups)
#define TP_FFTY_MAXCC 16
static int fftx_maxcc(int C, int Ny) { return ((C + 15) / 16) * Ny >= 1024 ? 16 : 8; }
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

// LDS of the persistent multi-column launch: the largest task's
template <typename T>
static size_t fused_multi_lds(int b, size_t sh2, bool rim) {
    constexpr int NTP = sizeof(T) == 4 ? 2 : 1;
    const int KP = (b + 7) >> 3;
    const size_t shp = (size_t)16 * NTP * (8 * KP + 2) * sizeof(cpx<T>);
    return std::max(std::max(sh2, shp), rim ? rim_mfma_lds<T>(false) : (size_t)0);
}

template <typename T, typename In, typename Out>
static void launch_fused_multi(tp_plan pl, Cols<const In> x, Cols<Out> y, int R, const cpx<T> *G, bool rim, int lg2,
                               int xs2, size_t sh2, int accumulate, Cols<const Out> acc, const cpx<T> *D, int nfin,
                               const RimMap &rm, hipStream_t st) {
    constexpr int NTP = sizeof(T) == 4 ? 2 : 1, NTR = rim_nt<T>();
    const int b = pl->bc, C = b * R;
    FusedDims fd;
    fd.nslab = pl->rim_nslab;
    fd.ncb_rim = (R + 16 * NTR - 1) / (16 * NTR);
    fd.nrim = rim ? fd.nslab * fd.ncb_rim : 0;
    fd.nfwd = (C + (1 << lg2) - 1) >> lg2;
    fd.ncb = (R + 16 * NTP - 1) / (16 * NTP);
    fd.nprod = pl->Px * pl->Py * fd.ncb;
    fd.ninv = fd.nfwd;
    fd.nfin = nfin;
    const size_t sh = fused_multi_lds<T>(b, sh2, rim);
    const int total = fd.nrim + fd.nfwd + fd.nprod + fd.ninv + fd.nfin;
    const int grid = std::min(total, 512);
    cpx<T> *gA = reinterpret_cast<cpx<T> *>(pl->gridA);
    cpx<T> *gB = reinterpret_cast<cpx<T> *>(pl->gridB);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, pl->fctr, kFusedCounters);
    if (rim)
        hipLaunchKernelGGL((k_fused_multi<T, In, Out, true>), dim3(grid), dim3(256), sh, st, x, y, R, pl->Nx, pl->Ny,
                           b, pl->fx, pl->fy, lg2, xs2, gA, gB, G, pl->kxh, OpPtrs<T>::B(pl),
                           reinterpret_cast<cpx<T> *>(pl->rim_part), OpPtrs<T>::C(pl), D, accumulate, acc, pl->N,
                           pl->Nr, rm, fd, pl->fctr);
    else
        hipLaunchKernelGGL((k_fused_multi<T, In, Out, false>), dim3(grid), dim3(256), sh, st, x, y, R, pl->Nx, pl->Ny,
                           b, pl->fx, pl->fy, lg2, xs2, gA, gB, G, pl->kxh, OpPtrs<T>::B(pl),
                           reinterpret_cast<cpx<T> *>(pl->rim_part), OpPtrs<T>::C(pl), D, accumulate, acc, pl->N,
                           pl->Nr, rm, fd, pl->fctr);
}


static int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Fused single-column path: LDS bytes.
static size_t spec_lds(tp_plan pl, size_t es) {
    const int P = pl->Py, CC = next_pow2(pl->bc);
    const size_t xm = pl->half ? (size_t)P * 8 : 0;   // mirror column channels
    return ((size_t)P + (size_t)P * CC + (size_t)P * 8 + xm) * es + (size_t)P * sizeof(int);
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
    // half spectrum: one workgroup per stored column and row chunk
    const int nchunk = (pl->bc + 7) / 8, nspec = pl->kxh * nchunk;
    const int nrim = E > 0 ? pl->rim_nslab : 0;
    const int lgCC = ilog2(next_pow2(pl->bc));
    cpx<T> *yp = reinterpret_cast<cpx<T> *>(pl->ypart);
    // (the half-spectrum form holds two panels per register buffer: rows of at
    // most 96 values, VPL <= 12)
    // Without the rim pass (E = 0) the spectrum workgroups have the GPU to
    // themselves: 8 waves each (FP32), so a column's stream and transforms
    // use a whole compute unit.
    // With more spectrum tasks than compute units (rows of more than 64
    // values), 8-wave workgroups (one per CU) would run in two rounds; 4-wave
    // ones fit two per CU, so every task is resident at once.
    if constexpr (VPL <= 12)
        if (pl->half) {
            if constexpr (E == 0 && sizeof(T) == 4) {
                if (nspec <= 256) {
                    hipLaunchKernelGGL((k_spec_rim<T, In, Out, VPL, U, E, NBE, true, 512>), dim3(nspec + nrim),
                                       dim3(512), sh, st, G, gA, gB, pl->bc, pl->Ny, pl->Px, pl->fy, lgCC, nspec,
                                       OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl), x, y, pl->N, pl->Nr,
                                       reinterpret_cast<cpx<T> *>(pl->rim_part), nrim, yp, pl->kxh);
                    return;
                }
            }
            {
                hipLaunchKernelGGL((k_spec_rim<T, In, Out, VPL, U, E, NBE, true, kBlock>), dim3(nspec + nrim),
                                   dim3(kBlock), sh, st, G, gA, gB, pl->bc, pl->Ny, pl->Px, pl->fy, lgCC, nspec,
                                   OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl), x, y, pl->N, pl->Nr,
                                   reinterpret_cast<cpx<T> *>(pl->rim_part), nrim, yp, pl->kxh);
            }
            return;
        }
        hipLaunchKernelGGL((k_spec_rim<T, In, Out, VPL, U, E, NBE, false>), dim3(nspec + nrim), dim3(256), sh, st, G,
                           gA, gB, pl->bc, pl->Ny, pl->Px, pl->fy, lgCC, nspec, OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl),
                           x, y, pl->N, pl->Nr, reinterpret_cast<cpx<T> *>(pl->rim_part), nrim, yp, pl->kxh);
}

// Pair stream over the stored half spectrum, one column (gB -> gA).
template <typename T>
static void launch_pair_prod(tp_plan pl, const cpx<T> *G, const cpx<T> *in, cpx<T> *out, const void *const *act,
                             hipStream_t st) {
    const int b = pl->bc, nw = (b + 7) / 8, vpl = (b + 7) / 8;
    const size_t sh = (size_t)(2 + nw) * b * sizeof(cpx<T>);
    const dim3 grid((unsigned)(pl->kxh * pl->Py)), blk((unsigned)(64 * nw));
    const int Px = pl->Px, Py = pl->Py, kxh = pl->kxh;
    if (vpl <= 2) hipLaunchKernelGGL((k_pair_prod<T, 2>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else if (vpl <= 4) hipLaunchKernelGGL((k_pair_prod<T, 4>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else if (vpl <= 6) hipLaunchKernelGGL((k_pair_prod<T, 6>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else if (vpl <= 8) hipLaunchKernelGGL((k_pair_prod<T, 8>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else if (vpl <= 9) hipLaunchKernelGGL((k_pair_prod<T, 9>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else if (vpl <= 12) hipLaunchKernelGGL((k_pair_prod<T, 12>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
    else hipLaunchKernelGGL((k_pair_prod<T, 16>), grid, blk, sh, st, G, in, b, Px, Py, kxh, out, act);
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
static void launch_prod_v(tp_plan pl, int RC, dim3 grid, size_t sh, hipStream_t st, const cpx<T> *G,
                          const cpx<T> *in, int b, int R, cpx<T> *out, const void *const *act) {
    const int Px = pl->Px, Py = pl->Py, kxh = pl->kxh;
    switch (RC) {
        case 2: hipLaunchKernelGGL((k_prod<T, VPL, 2>), grid, dim3(256), sh, st, G, in, b, R, out, act, Px, Py, kxh);
                break;
        case 4: hipLaunchKernelGGL((k_prod<T, VPL, 4>), grid, dim3(256), sh, st, G, in, b, R, out, act, Px, Py, kxh);
                break;
        case 8: hipLaunchKernelGGL((k_prod<T, VPL, 8>), grid, dim3(256), sh, st, G, in, b, R, out, act, Px, Py, kxh);
                break;
        default: hipLaunchKernelGGL((k_prod<T, VPL, 16>), grid, dim3(256), sh, st, G, in, b, R, out, act, Px, Py,
                                    kxh);
                 break;
    }
}
template <typename T>
static void launch_prod(tp_plan pl, int vpl, int RC, dim3 grid, size_t sh, hipStream_t st, const cpx<T> *G,
                        const cpx<T> *in, int b, int R, cpx<T> *out, const void *const *act) {
    if (vpl <= 2) launch_prod_v<T, 2>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 4) launch_prod_v<T, 4>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 6) launch_prod_v<T, 6>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 8) launch_prod_v<T, 8>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 12) launch_prod_v<T, 12>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else if (vpl <= 16) launch_prod_v<T, 16>(pl, RC, grid, sh, st, G, in, b, R, out, act);
    else launch_prod_v<T, 32>(pl, RC, grid, sh, st, G, in, b, R, out, act);
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
// The FP32 product with the block in LDS, when the plan's option asks for it
// and the block and the workgroup fit
template <typename T>
static bool prod_lds_ok(tp_plan pl, int b) {
    if (sizeof(T) != 4 || pl->opt_prod_lds == 0 || b > 128 || prod_lds_bytes(b) > kLdsLimit) return false;
    const int CG = (pl->opt_prod_lds >> 4) & 15, RT = pl->opt_prod_lds & 15, nrt = (b + 15) >> 4;
    const int rt = RT <= 2 ? 2 : RT <= 3 ? 3 : 6;
    return CG >= 1 && CG * ((nrt + rt - 1) / rt) <= 16;
}

// The launches an application takes at R columns (one choice for the
// operator and its preconditioner alike; PRE picks the preconditioner).
struct Path {
    bool rim;          // dense rim pass (slabs; finished with the rim rows)
    bool pairs;        // one column, pair-stream spectrum pass
    bool fused;        // one column, fused spectrum pass
    bool mfma;         // products (and a dense rim) on the matrix cores
    bool rim_mma;      // the dense rim on the matrix cores
    bool fusedm;       // every stage in one persistent launch
    bool rimfwd;       // the dense rim's slabs and the forward 2-D tiles in one launch
    int lg2, xs2;      // 2-D tiles: log2 channels per tile (-1: separate x and y passes), row stride
    size_t sh_fused, sh2;
};

template <typename T, bool PRE>
static Path choose_path(tp_plan pl, int R) {
    Path P;
    const int b = pl->bc, Nr = pl->Nr, Px = pl->Px, Py = pl->Py, C = b * R;
    const size_t es = sizeof(cpx<T>);
    P.rim = !PRE && Nr > 0 && pl->nrc == 0;
    P.sh_fused = std::max(spec_lds(pl, es), P.rim ? rim_lds(pl, 1, es) : (size_t)0);
    // one column without a rim pass over a half spectrum: the fused path or the
    // pair stream (y transforms in passes of their own), as the plan's option
    // says (the tuner picks it; without a choice the fused path)
    P.pairs = R == 1 && !P.rim && pl->half && b <= 128 && pl->opt_spectrum_pass == TP_PASS_PAIRS;
    // one column: the fused path (for a half spectrum, rows of at most 96)
    P.fused = !P.pairs && R == 1 && P.sh_fused <= kLdsLimit && !(pl->half && b > 96);
    // many columns: the product and the rim run on the matrix cores (from the
    // plan's threshold, else kMfmaMinR columns)
    P.mfma = !P.fused && !P.pairs && R >= (pl->opt_mfma_min_r ? pl->opt_mfma_min_r : kMfmaMinR);
    P.rim_mma = P.mfma && P.rim && pl->rim_te == 64 && rim_mfma_lds<T>(OpPtrs<T>::BE(pl) != nullptr) <= kLdsLimit;
    // small grids with several columns: both transform directions per launch
    // (the plan's option may let the 2-D tiles take more LDS: larger grids
    // then run both transform directions in one launch, on fewer workgroups)
    P.lg2 = P.fused ? -1 : fft2_lgcc(Px, Py, C, es, pl->opt_fft2_lds ? (size_t)pl->opt_fft2_lds : 48 * 1024);
    P.xs2 = P.lg2 >= 0 ? fft2_xstride(Py, P.lg2, es) : 0;
    P.sh2 = ((size_t)Px * P.xs2 + Px + Py) * es + (size_t)(Px + Py) * sizeof(int);
    // many columns on the 2-D tiles and the matrix cores: optionally every
    // stage in one persistent launch (default column tile, even b, a dense
    // rim only when reciprocal)
    P.fusedm = pl->opt_multi_fused == 1 && pl->opt_prod_lds == 0 && P.mfma && P.lg2 >= 0 && pl->fctr && b % 2 == 0 &&
               (!P.rim || (P.rim_mma && OpPtrs<T>::BE(pl) == nullptr)) &&
               (pl->opt_mfma_cols == 0 || pl->opt_mfma_cols == (sizeof(T) == 4 ? 32 : 16)) &&
               fused_multi_lds<T>(b, P.sh2, P.rim) + 1024 <= kLdsLimit;
    P.rimfwd = !P.fusedm && pl->opt_rim_overlap == 1 && P.rim_mma && P.lg2 >= 0 &&
               std::max(P.sh2, rim_mfma_lds<T>(OpPtrs<T>::BE(pl) != nullptr)) + 1024 <= kLdsLimit;
    return P;
}

template <typename T, typename In, typename Out, bool PRE = false>
hipError_t matvec_launch(tp_plan pl, Cols<const In> x, Cols<Out> y, int R, hipStream_t st,
                         hipEvent_t *ev = nullptr, Cols<const Out> base = Cols<const Out>{nullptr, 0, nullptr},
                         int last_stage = 7) {
    // b: channels per cell (element basis functions, plus the rim channels of
    // a placed rim); the embedding and crop map channels to unknowns
    const int Nx = pl->Nx, Ny = pl->Ny, b = pl->bc, Nr = pl->Nr;
    const int Px = pl->Px, Py = pl->Py, C = b * R;
    const RimMap rm{pl->rim_map, pl->b, pl->nrc, pl->N};
    cpx<T> *gA = reinterpret_cast<cpx<T> *>(pl->gridA);
    cpx<T> *gB = reinterpret_cast<cpx<T> *>(pl->gridB);
    const size_t es = sizeof(cpx<T>);
    const dim3 blk(256);
    const void *const *act = (const void *const *)x.tab;
    auto mark = [&](int i) {
        if (ev) hipEventRecord(ev[i], st);
    };
    // instrumentation (a copy of the plan record with only_stage set): launch
    // one stage alone, on the workspace a full application left behind
    // (last_stage < 7: the stages after it are left to the caller)
    auto on = [&](int stage) { return stage <= last_stage && (pl->only_stage < 0 || pl->only_stage == stage); };
    const cpx<T> *G = PRE ? OpPtrs<T>::S(pl) : OpPtrs<T>::G(pl);
    const Path P = choose_path<T, PRE>(pl, R);
    const bool rim = P.rim, pairs = P.pairs, fused = P.fused, mfma = P.mfma, rim_mma = P.rim_mma;
    const int lg2 = P.lg2, xs2 = P.xs2;
    const size_t sh_fused = P.sh_fused, sh2 = P.sh2;
    // the operator adds its rim term (already in y); the preconditioner adds
    // the caller's base columns, if any
    const Cols<const Out> acc = PRE ? base : Cols<const Out>{y.base, y.ld, y.tab};
    const int accumulate = PRE ? (base.base || base.tab ? 1 : 0) : (rim ? 1 : 0);
    const cpx<T> *D = PRE ? OpPtrs<T>::D(pl) : nullptr;
    // rim rows of a dense rim (C x_r and the slab partials, or D x_r) are
    // finished by extra waves; a placed rim's rows come out of the crop
    const int nfin = (Nr > 0 && pl->nrc == 0) ? ((Nr + 3) / 4) * R : 0;
    if (P.fusedm) {
        mark(0);
        mark(1);
        mark(2);
        mark(3);
        if (on(3))
            launch_fused_multi<T, In, Out>(pl, x, y, R, G, rim, lg2, xs2, sh2, accumulate, acc, D, nfin, rm, st);
        mark(4);
        mark(5);
        mark(6);
        mark(7);
        return hipGetLastError();
    }

    // the dense rim and the forward 2-D tiles in one launch (plan option; a
    // timing of one stage launches them apart)
    const bool rimfwd = P.rimfwd && pl->only_stage < 0;
    mark(0);
    if (rimfwd) {
        const cpx<T> *Bp = OpPtrs<T>::B(pl), *BEp = OpPtrs<T>::BE(pl);
        const int nrim = pl->rim_nslab * ((R + 16 * rim_nt<T>() - 1) / (16 * rim_nt<T>()));
        const int nfwd = (C + (1 << lg2) - 1) >> lg2;
        const size_t sh = std::max(sh2, rim_mfma_lds<T>(BEp != nullptr));
        cpx<T> *partp = reinterpret_cast<cpx<T> *>(pl->rim_part);
        if (BEp)
            hipLaunchKernelGGL((k_rim_fft2_fwd<T, In, Out, true>), dim3(nrim + nfwd), blk, sh, st, Bp, BEp, x, y, R,
                               pl->N, Nr, partp, pl->rim_nslab, nrim, Nx, Ny, b, pl->fx, pl->fy, lg2, xs2, gB, rm);
        else
            hipLaunchKernelGGL((k_rim_fft2_fwd<T, In, Out, false>), dim3(nrim + nfwd), blk, sh, st, Bp, Bp, x, y,
                               R, pl->N, Nr, partp, pl->rim_nslab, nrim, Nx, Ny, b, pl->fx, pl->fy, lg2, xs2, gB,
                               rm);
    } else if (rim && !fused && on(0)) {
        if (rim_mma)
            rim_mfma<T, In, Out>(OpPtrs<T>::B(pl), OpPtrs<T>::BE(pl), x, y, R, pl->N, Nr, pl->rim_nslab,
                                 reinterpret_cast<cpx<T> *>(pl->rim_part), st);
        else
            launch_rim_general<T, In, Out>(pl, x, y, R, st);
    }
    mark(1);
    if (!on(1) || rimfwd) {
    } else if (lg2 >= 0) {
        hipLaunchKernelGGL((k_fft2_fwd<T, In>), dim3((C + (1 << lg2) - 1) >> lg2), blk, sh2, st, x, R, Nx, Ny, b,
                           pl->fx, pl->fy, lg2, xs2, gB, rm);
    } else {
        const int lg = fft_lgcc(Px, C, es, fftx_maxcc(C, Ny));
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Ny);
        hipLaunchKernelGGL((k_fwd_x<T, In>), grid, blk, sh, st, x, R, Nx, b, pl->fx, lg, gA, rm);
    }
    mark(2);
    if (!fused && lg2 < 0 && on(2)) {
        const int lg = fft_lgcc(Py, C, es, TP_FFTY_MAXCC);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_fwd_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    mark(3);
    if (!on(3)) {
    } else if (fused) {
        const int vpl = (b + 7) / 8;
        if (vpl <= 2) launch_spec_rim_e<T, In, Out, 2>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 4) launch_spec_rim_e<T, In, Out, 4>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 6) launch_spec_rim_e<T, In, Out, 6>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 8) launch_spec_rim_e<T, In, Out, 8>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 9) launch_spec_rim_e<T, In, Out, 9>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 12) launch_spec_rim_e<T, In, Out, 12>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else if (vpl <= 16) launch_spec_rim_e<T, In, Out, 16>(pl, G, rim, x, y, gA, gB, sh_fused, st);
        else launch_spec_rim_e<T, In, Out, 32>(pl, G, rim, x, y, gA, gB, sh_fused, st);
    } else if (pairs) {
        launch_pair_prod<T>(pl, G, gB, gA, act, st);
    } else if (mfma && prod_lds_ok<T>(pl, b)) {
        prod_lds(reinterpret_cast<const c64 *>(G), reinterpret_cast<const c64 *>(gB), b, R, Px, Py, pl->kxh,
                 reinterpret_cast<c64 *>(gA), act, st, (pl->opt_prod_lds >> 4) & 15, pl->opt_prod_lds & 15,
                 (pl->opt_prod_lds & 256) != 0 && pl->half);
    } else if (mfma) {
        prod_mfma<T>(G, gB, b, R, Px, Py, pl->kxh, gA, act, st, pl->opt_mfma_cols);
    } else {
        // columns per workgroup: up to 16 (the spectrum block is re-read from
        // cache by each column block of a frequency)
        const int RC = R >= 16 ? 16 : R >= 8 ? 8 : R >= 4 ? 4 : 2;
        const size_t sh = (size_t)RC * b * es;
        dim3 grid(Px * Py, (R + RC - 1) / RC);
        const int vpl = (b + 7) / 8;
        launch_prod<T>(pl, vpl, RC, grid, sh, st, G, gB, b, R, gA, act);
    }
    mark(4);
    if (!fused && lg2 < 0 && on(4)) {
        const int lg = fft_lgcc(Py, C, es, TP_FFTY_MAXCC);
        const size_t sh = ((size_t)Py * (1 << lg) + Py) * es;
        dim3 grid((C + (1 << lg) - 1) >> lg, Px);
        hipLaunchKernelGGL((k_inv_y<T>), grid, blk, sh, st, gA, C, Ny, Px, pl->fy, lg, gB, act, b);
    }
    mark(5);
    if (!on(5)) {
    } else if (lg2 >= 0) {
        const int ninv = (C + (1 << lg2) - 1) >> lg2;
        hipLaunchKernelGGL((k_fft2_inv_fin<T, In, Out>), dim3(ninv + nfin), blk, sh2, st, gA, R, Nx, Ny, b, pl->fx,
                           pl->fy, lg2, xs2, y, accumulate, acc, ninv,
                           reinterpret_cast<const cpx<T> *>(pl->rim_part), OpPtrs<T>::C(pl), D, x, pl->N, Nr,
                           pl->rim_nslab, rm);
    } else {
        // the fused path leaves Y1 in gB with channel count b (R = 1), the
        // general path in gB with b * R channels: the same layout
        const int lg = fft_lgcc(Px, C, es, fftx_maxcc(C, Ny));
        const size_t sh = ((size_t)Px * (1 << lg) + Px) * es;
        const int nchunk = (C + (1 << lg) - 1) >> lg;
        const int ninv = nchunk * Ny;
        // the half-spectrum fused path leaves the mirror columns as parts
        MirrorParts<T> mp{nullptr, Px, 0, 0, 0};
        if (fused && pl->half) {
            mp.yp = reinterpret_cast<const cpx<T> *>(pl->ypart);
            mp.kxh = pl->kxh;
            mp.nmir = Px - pl->kxh;
            mp.nch = (b + 7) / 8;
            mp.hstride = (long)Ny * mp.nmir * b;
        }
        hipLaunchKernelGGL((k_inv_x_fin<T, In, Out>), dim3(ninv + nfin), blk, sh, st, gB, R, Nx, b, pl->fx, lg,
                           nchunk, y, accumulate, acc, ninv, reinterpret_cast<const cpx<T> *>(pl->rim_part),
                           OpPtrs<T>::C(pl), D, x, pl->N, Nr, pl->rim_nslab, mp, rm);
    }
    mark(6);
    mark(7);
    return hipGetLastError();
}

// --------------------------------------------- both precisions per launch
// The mixed solver applies, in every super-step, the FP32 operator to the
// columns in an Arnoldi step and the FP64 operator to the columns in a
// residual step; one of the two usually has no live column (one right-hand
// side: always).  Here each stage of the one-column pair-stream path runs once
// for both: workgroups with blockIdx.z = 0 take the FP32 instance, z = 1 the
// FP64 one (each with its own grids), and an instance without live columns
// exits at once, so the idle instance costs no launch of its own.
template <typename In>
__global__ void __launch_bounds__(256) k_fwd_x_dual(Cols<const In> x32, Cols<const In> x64, int R, int Nx, int b,
                                                    FFTDesc fx, int lg32, int lg64, int g32, int g64, c64 *o32,
                                                    c128 *o64, RimMap rm) {
    extern __shared__ char smem_raw[];
    if (blockIdx.z == 0) {
        if ((int)blockIdx.x < g32)
            fwd_x_body<float, In>(x32, R, Nx, b, fx, lg32, o32, rm, blockIdx.x, blockIdx.y, smem_raw);
    } else if ((int)blockIdx.x < g64) {
        fwd_x_body<double, In>(x64, R, Nx, b, fx, lg64, o64, rm, blockIdx.x, blockIdx.y, smem_raw);
    }
}

template <bool INV>
__global__ void __launch_bounds__(256) k_y_dual(const c64 *i32, const c128 *i64, int C, int Ny, int Px, FFTDesc fy,
                                                int lg32, int lg64, int g32, int g64, c64 *o32, c128 *o64,
                                                const void *const *a32, const void *const *a64, int b) {
    extern __shared__ char smem_raw[];
    if (blockIdx.z == 0) {
        if ((int)blockIdx.x >= g32) return;
        if (INV) inv_y_body<float>(i32, C, Ny, Px, fy, lg32, o32, a32, b, blockIdx.x, blockIdx.y, smem_raw);
        else fwd_y_body<float>(i32, C, Ny, Px, fy, lg32, o32, a32, b, blockIdx.x, blockIdx.y, smem_raw);
    } else {
        if ((int)blockIdx.x >= g64) return;
        if (INV) inv_y_body<double>(i64, C, Ny, Px, fy, lg64, o64, a64, b, blockIdx.x, blockIdx.y, smem_raw);
        else fwd_y_body<double>(i64, C, Ny, Px, fy, lg64, o64, a64, b, blockIdx.x, blockIdx.y, smem_raw);
    }
}

template <int VPL>
__global__ void __launch_bounds__(1024) k_pair_prod_dual(const c64 *G32, const c128 *G64, const c64 *i32,
                                                         const c128 *i64, int b, int Px, int Py, int kxh, c64 *o32,
                                                         c128 *o64, const void *const *a32,
                                                         const void *const *a64) {
    extern __shared__ char smem_raw[];
    if (blockIdx.z == 0) pair_prod_body<float, VPL>(G32, i32, b, Px, Py, kxh, o32, a32, blockIdx.x, smem_raw);
    else pair_prod_body<double, VPL>(G64, i64, b, Px, Py, kxh, o64, a64, blockIdx.x, smem_raw);
}

template <typename In, typename Out>
__global__ void __launch_bounds__(256) k_inv_x_dual(const c64 *i32, const c128 *i64, int R, int Nx, int b, FFTDesc fx,
                                                    int lg32, int lg64, int nc32, int nc64, Cols<Out> y32,
                                                    Cols<Out> y64, int g32, int g64, long N, int Nr, RimMap rm) {
    extern __shared__ char smem_raw[];
    // the operator of a plan without a dense rim pass: no accumulation, no
    // rim rows to finish (a placed rim's rows come out of the crop)
    if (blockIdx.z == 0) {
        if ((int)blockIdx.x >= g32) return;
        inv_x_fin_body<float, In, Out>(i32, R, Nx, b, fx, lg32, nc32, y32, 0, Cols<const Out>{y32.base, y32.ld, y32.tab},
                                       g32, nullptr, nullptr, nullptr, Cols<const In>{nullptr, 0, nullptr}, N, Nr, 0,
                                       MirrorParts<float>{nullptr, 0, 0, 0, 0}, rm, blockIdx.x, smem_raw);
    } else {
        if ((int)blockIdx.x >= g64) return;
        inv_x_fin_body<double, In, Out>(i64, R, Nx, b, fx, lg64, nc64, y64, 0,
                                        Cols<const Out>{y64.base, y64.ld, y64.tab}, g64, nullptr, nullptr, nullptr,
                                        Cols<const In>{nullptr, 0, nullptr}, N, Nr, 0,
                                        MirrorParts<double>{nullptr, 0, 0, 0, 0}, rm, blockIdx.x, smem_raw);
    }
}

// Many columns: the matrix-core product of both instances in one launch
// (default column tiles: NT32 for FP32, one tile of 16 for FP64).  Each
// instance deals its own items to the XCDs as k_prod_mfma does (a contiguous
// range per XCD, sized from the instance's own item count, so an instance
// with fewer items than the launch still spreads over all eight).
template <int NT32, bool EVEN>
__global__ void __launch_bounds__(1024) k_prod_mfma_dual(const c64 *G32, const c128 *G64, const c64 *i32,
                                                         const c128 *i64, int b, int R, int Px, int Py, int kxh,
                                                         c64 *o32, c128 *o64, const void *const *a32,
                                                         const void *const *a64) {
    extern __shared__ char smem_raw[];
    const long P = (long)Px * Py;
    const int ncb = blockIdx.z == 0 ? (R + 16 * NT32 - 1) / (16 * NT32) : (R + 15) / 16;
    const long nitem = P * ncb, per = (nitem + 7) >> 3;
    if ((long)(blockIdx.x >> 3) >= per) return;
    const long item = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (item >= nitem) return;
    const long k = item / ncb;
    if (blockIdx.z == 0)
        prod_mfma_item<float, NT32, TP_PROD_KC, EVEN>(G32, i32, b, R, Px, Py, kxh, o32, a32, k,
                                                      (int)(item - k * ncb), smem_raw);
    else
        prod_mfma_item<double, 1, TP_PROD_KC, EVEN>(G64, i64, b, R, Px, Py, kxh, o64, a64, k, (int)(item - k * ncb),
                                                    smem_raw);
}

// Many columns on small grids: the 2-D tiles of both instances per launch
// (no rim: the operator of a plan without a dense rim pass).
template <typename In>
__global__ void __launch_bounds__(256) k_fft2_fwd_dual(Cols<const In> x32, Cols<const In> x64, int R, int Nx, int Ny,
                                                       int b, FFTDesc fx, FFTDesc fy, int lg32, int lg64, int xs32,
                                                       int xs64, int g32, int g64, c64 *o32, c128 *o64, RimMap rm) {
    extern __shared__ char smem_raw[];
    if (blockIdx.z == 0) {
        if ((int)blockIdx.x < g32)
            fft2_fwd_tile<float, In>(x32, R, Nx, Ny, b, fx, fy, lg32, xs32, o32, rm, blockIdx.x, smem_raw);
    } else if ((int)blockIdx.x < g64) {
        fft2_fwd_tile<double, In>(x64, R, Nx, Ny, b, fx, fy, lg64, xs64, o64, rm, blockIdx.x, smem_raw);
    }
}

template <typename In, typename Out>
__global__ void __launch_bounds__(256) k_fft2_inv_dual(const c64 *i32, const c128 *i64, int R, int Nx, int Ny, int b,
                                                       FFTDesc fx, FFTDesc fy, int lg32, int lg64, int xs32, int xs64,
                                                       int g32, int g64, Cols<Out> y32, Cols<Out> y64, long N,
                                                       int Nr, RimMap rm) {
    extern __shared__ char smem_raw[];
    const Cols<const In> nox{nullptr, 0, nullptr};
    if (blockIdx.z == 0) {
        if ((int)blockIdx.x < g32)
            fft2_inv_tile<float, In, Out>(i32, R, Nx, Ny, b, fx, fy, lg32, xs32, y32, 0,
                                          Cols<const Out>{y32.base, y32.ld, y32.tab}, g32, nullptr, nullptr, nullptr,
                                          nox, N, Nr, 0, rm, blockIdx.x, smem_raw);
    } else if ((int)blockIdx.x < g64) {
        fft2_inv_tile<double, In, Out>(i64, R, Nx, Ny, b, fx, fy, lg64, xs64, y64, 0,
                                       Cols<const Out>{y64.base, y64.ld, y64.tab}, g64, nullptr, nullptr, nullptr,
                                       nox, N, Nr, 0, rm, blockIdx.x, smem_raw);
    }
}

// The FP32 operator on (x32 -> y32) and the FP64 operator on (x64 -> y64) in
// one launch per stage, where both precisions take the same launch shape and
// the plan has FP32 grids of its own: one column on the pair-stream path with
// separate x and y passes, or many columns (up to the plan's max_rhs) with the
// matrix-core product at its default column tiles, on separate passes or on
// 2-D tiles, without a dense rim pass.  Otherwise returns false and launches
// nothing.
template <typename In, typename Out>
bool matvec_dual_launch(tp_plan pl, Cols<const In> x32, Cols<Out> y32, Cols<const In> x64, Cols<Out> y64, int R,
                        hipStream_t st, bool skip_fwd_x = false) {
    if (!pl->gridA32 || !pl->G32 || !pl->G64) return false;
    const Path p32 = choose_path<float, false>(pl, R), p64 = choose_path<double, false>(pl, R);
    if (p32.rim || p64.rim || p32.fused || p64.fused || p32.fusedm || p64.fusedm) return false;
    const bool pairs = p32.pairs && p64.pairs;
    const bool mfma = p32.mfma && p64.mfma && pl->opt_mfma_cols == 0 && pl->opt_prod_lds == 0;
    if (!pairs && !mfma) return false;
    const bool tiles = p32.lg2 >= 0 && p64.lg2 >= 0;
    if (!tiles && (p32.lg2 >= 0 || p64.lg2 >= 0)) return false;
    if (pairs && tiles) return false;
    if (skip_fwd_x && (tiles || !pairs)) return false;
    const int Nx = pl->Nx, Ny = pl->Ny, b = pl->bc, Px = pl->Px, Py = pl->Py, C = b * R;
    const RimMap rm{pl->rim_map, pl->b, pl->nrc, pl->N};
    c64 *A32 = reinterpret_cast<c64 *>(pl->gridA32), *B32 = reinterpret_cast<c64 *>(pl->gridB32);
    c128 *A64 = reinterpret_cast<c128 *>(pl->gridA), *B64 = reinterpret_cast<c128 *>(pl->gridB);
    const void *const *a32 = (const void *const *)x32.tab;
    const void *const *a64 = (const void *const *)x64.tab;
    const dim3 blk(256);
    if (tiles) {
        // 2-D tiles: forward (-> B), products (B -> A), inverse (A -> y)
        const int g32 = (C + (1 << p32.lg2) - 1) >> p32.lg2, g64 = (C + (1 << p64.lg2) - 1) >> p64.lg2;
        const size_t sh = std::max(p32.sh2, p64.sh2);
        hipLaunchKernelGGL((k_fft2_fwd_dual<In>), dim3(std::max(g32, g64), 1, 2), blk, sh, st, x32, x64, R, Nx, Ny, b,
                           pl->fx, pl->fy, p32.lg2, p64.lg2, p32.xs2, p64.xs2, g32, g64, B32, B64, rm);
    } else {
        // x passes (-> A)
        const int lx32 = fft_lgcc(Px, C, 8, fftx_maxcc(C, Ny)), lx64 = fft_lgcc(Px, C, 16, fftx_maxcc(C, Ny));
        const int gx32 = (C + (1 << lx32) - 1) >> lx32, gx64 = (C + (1 << lx64) - 1) >> lx64;
        const size_t shx = std::max(((size_t)Px * (1 << lx32) + Px) * 8, ((size_t)Px * (1 << lx64) + Px) * 16);
        if (!skip_fwd_x)
            hipLaunchKernelGGL((k_fwd_x_dual<In>), dim3(std::max(gx32, gx64), Ny, 2), blk, shx, st, x32, x64, R, Nx,
                               b, pl->fx, lx32, lx64, gx32, gx64, A32, A64, rm);
        // y passes (A -> B)
        const int ly32 = fft_lgcc(Py, C, 8, TP_FFTY_MAXCC), ly64 = fft_lgcc(Py, C, 16, TP_FFTY_MAXCC);
        const int gy32 = (C + (1 << ly32) - 1) >> ly32, gy64 = (C + (1 << ly64) - 1) >> ly64;
        const size_t shy = std::max(((size_t)Py * (1 << ly32) + Py) * 8, ((size_t)Py * (1 << ly64) + Py) * 16);
        hipLaunchKernelGGL((k_y_dual<false>), dim3(std::max(gy32, gy64), Px, 2), blk, shy, st, A32, A64, C, Ny, Px,
                           pl->fy, ly32, ly64, gy32, gy64, B32, B64, a32, a64, b);
    }
    // products (B -> A)
    if (pairs) {
        const int nw = (b + 7) / 8, vpl = (b + 7) / 8;
        const size_t sh = (size_t)(2 + nw) * b * sizeof(c128);
        const dim3 grid((unsigned)(pl->kxh * Py), 1, 2), pblk((unsigned)(64 * nw));
        const int kxh = pl->kxh;
#define TP_PAIR_DUAL(V)                                                                                         \
    hipLaunchKernelGGL((k_pair_prod_dual<V>), grid, pblk, sh, st, pl->G32, pl->G64, B32, B64, b, Px, Py, kxh, A32, \
                       A64, a32, a64)
        if (vpl <= 2) TP_PAIR_DUAL(2);
        else if (vpl <= 4) TP_PAIR_DUAL(4);
        else if (vpl <= 6) TP_PAIR_DUAL(6);
        else if (vpl <= 8) TP_PAIR_DUAL(8);
        else if (vpl <= 9) TP_PAIR_DUAL(9);
        else if (vpl <= 12) TP_PAIR_DUAL(12);
        else TP_PAIR_DUAL(16);
#undef TP_PAIR_DUAL
    } else {
        // default column tiles: FP32 16 up to 16 columns, else 32; FP64 16
        const int nt32 = R > 16 ? 2 : 1, KP = (b + 7) >> 3;
        const size_t sh = std::max((size_t)16 * nt32 * (8 * KP + 2) * 8, (size_t)16 * (8 * KP + 2) * 16);
        const long P = (long)Px * Py;
        const long n32 = P * ((R + 16 * nt32 - 1) / (16 * nt32)), n64 = P * ((R + 15) / 16);
        const long nitem = std::max(n32, n64);
        const dim3 grid((unsigned)(((nitem + 7) / 8) * 8), 1, 2), mblk((unsigned)(64 * ((b + 15) / 16)));
        const int kxh = pl->kxh;
        if (b % 2 == 0) {
            if (nt32 == 2)
                hipLaunchKernelGGL((k_prod_mfma_dual<2, true>), grid, mblk, sh, st, pl->G32, pl->G64, B32, B64, b, R,
                                   Px, Py, kxh, A32, A64, a32, a64);
            else
                hipLaunchKernelGGL((k_prod_mfma_dual<1, true>), grid, mblk, sh, st, pl->G32, pl->G64, B32, B64, b, R,
                                   Px, Py, kxh, A32, A64, a32, a64);
        } else {
            if (nt32 == 2)
                hipLaunchKernelGGL((k_prod_mfma_dual<2, false>), grid, mblk, sh, st, pl->G32, pl->G64, B32, B64, b,
                                   R, Px, Py, kxh, A32, A64, a32, a64);
            else
                hipLaunchKernelGGL((k_prod_mfma_dual<1, false>), grid, mblk, sh, st, pl->G32, pl->G64, B32, B64, b,
                                   R, Px, Py, kxh, A32, A64, a32, a64);
        }
    }
    if (tiles) {
        const int g32 = (C + (1 << p32.lg2) - 1) >> p32.lg2, g64 = (C + (1 << p64.lg2) - 1) >> p64.lg2;
        const size_t sh = std::max(p32.sh2, p64.sh2);
        hipLaunchKernelGGL((k_fft2_inv_dual<In, Out>), dim3(std::max(g32, g64), 1, 2), blk, sh, st, A32, A64, R, Nx,
                           Ny, b, pl->fx, pl->fy, p32.lg2, p64.lg2, p32.xs2, p64.xs2, g32, g64, y32, y64, pl->N,
                           pl->Nr, rm);
        return true;
    }
    // inverse y passes (A -> B), inverse x passes and crop (B -> y)
    const int ly32 = fft_lgcc(Py, C, 8, TP_FFTY_MAXCC), ly64 = fft_lgcc(Py, C, 16, TP_FFTY_MAXCC);
    const int gy32 = (C + (1 << ly32) - 1) >> ly32, gy64 = (C + (1 << ly64) - 1) >> ly64;
    const size_t shy = std::max(((size_t)Py * (1 << ly32) + Py) * 8, ((size_t)Py * (1 << ly64) + Py) * 16);
    hipLaunchKernelGGL((k_y_dual<true>), dim3(std::max(gy32, gy64), Px, 2), blk, shy, st, A32, A64, C, Ny, Px,
                       pl->fy, ly32, ly64, gy32, gy64, B32, B64, a32, a64, b);
    const int lx32 = fft_lgcc(Px, C, 8, fftx_maxcc(C, Ny)), lx64 = fft_lgcc(Px, C, 16, fftx_maxcc(C, Ny));
    const int nc32 = (C + (1 << lx32) - 1) >> lx32, nc64 = (C + (1 << lx64) - 1) >> lx64;
    const size_t shx = std::max(((size_t)Px * (1 << lx32) + Px) * 8, ((size_t)Px * (1 << lx64) + Px) * 16);
    hipLaunchKernelGGL((k_inv_x_dual<In, Out>), dim3(std::max(nc32, nc64) * Ny, 1, 2), blk, shx, st, B32, B64, R,
                       Nx, b, pl->fx, lx32, lx64, nc32, nc64, y32, y64, nc32 * Ny, nc64 * Ny, pl->N, pl->Nr, rm);
    return true;
}

}  // namespace tp
