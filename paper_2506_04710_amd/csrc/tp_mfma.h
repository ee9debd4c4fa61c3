#pragma once
// Matrix-core (MFMA) kernels for many right-hand sides, where the operator's
// per-frequency product and its rim blocks become dense complex contractions.
//
// Both kernels are built from the 16 x 16 x 4 real MFMA (f32 or f64): lane l of
// a wave supplies A[l % 16][l / 16] and B[l / 16][l % 16] and, after the
// instruction, holds D[row(l / 16, v)][l % 16] for v = 0..3, with
// row(g, v) = 4 g + v for f32 and g + 4 v for f64 (checked on gfx950 with
// single-lane unit inputs).  A complex product takes four of them:
//   D_re += A_re B_re + (-A_im) B_im,   D_im += A_re B_im + A_im B_re.
// The contraction index k is free to be permuted, as long as A and B use the
// same permutation; the kernels pick one that gives each lane a contiguous
// run of memory.
#include "tp_internal.h"

// pairs of contraction steps per prefetched chunk of the product
#ifndef TP_PROD_KC
#define TP_PROD_KC 4
#endif

namespace tp {


template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// Stage n values into LDS with U loads in flight per thread: every load of a
// round issues (addresses clamped by `ld`) before any value is stored, so the
// round costs one memory latency rather than U.  Indices past the end are
// clamped to n - 1 for the store as well: such a thread writes the same value
// to the same slot as the thread that owns it, and no branch forms.
template <int U, typename V, typename Load, typename Store>
__device__ __forceinline__ void stage(int n, Load ld, Store st, int nt = kBlock) {
    for (int base = threadIdx.x; base < n; base += U * nt) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(min(base + u * nt, n - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) st(min(base + u * nt, n - 1), v[u]);
    }
}

template <typename T>
struct CAcc {
    typename Mfma<T>::v4 re, im;
    __device__ __forceinline__ void zero() {
        for (int v = 0; v < 4; ++v) re[v] = im[v] = 0;
    }
    __device__ __forceinline__ void mac(cpx<T> a, cpx<T> b) {
        mac_a(a, b);
        mac_b(a, b);
    }
    // the two halves of mac, each two independent instructions: callers with
    // several accumulators issue the first half of every one before the
    // second, so no instruction waits on the one just before it (each
    // accumulator still sums in the order of mac)
    __device__ __forceinline__ void mac_a(cpx<T> a, cpx<T> b) {
        re = Mfma<T>::mac(a.x, b.x, re);
        im = Mfma<T>::mac(a.x, b.y, im);
    }
    __device__ __forceinline__ void mac_b(cpx<T> a, cpx<T> b) {
        re = Mfma<T>::mac(-a.y, b.y, re);
        im = Mfma<T>::mac(a.y, b.x, im);
    }
    __device__ __forceinline__ cpx<T> get(int v) const { return mk<T>(re[v], im[v]); }
};

// ------------------------------------------------ per-frequency product
// Two consecutive values of a row, fetched with one load.
template <typename T>
struct alignas(4 * sizeof(T)) cpair {
    cpx<T> a, b;
};

// One item (frequency k, column block cb of 16 NT columns) by the workgroup's
// waves: wave w takes the 16-row output tiles w, w + nw, ... (one each when
// the launch has a wave per tile, several in the fused persistent launch).
// The arithmetic of an output value does not depend on which wave computes
// it, so both launches give the same bits.
template <typename T, int NT, int KC, bool EVEN>
__device__ __forceinline__ void prod_mfma_item(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in, int b,
                                               int R, int Px, int Py, int kxh, cpx<T> *__restrict__ out,
                                               const void *const *act, long k, int cb, char *smem) {
    cpx<T> *xs = reinterpret_cast<cpx<T> *>(smem);
    const int KP = (b + 7) >> 3, W = 8 * KP, bs = W + 2;
    const long C = (long)b * R;
    const int r0 = cb * 16 * NT, rn = min(16 * NT, R - r0);
    if (!cols_live(act, r0, r0 + rn - 1)) return;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    const int nthr = blockDim.x, nw = nthr >> 6, nrt = (b + 15) >> 4;
    stage<4, cpx<T>>(
        16 * NT * W,
        [&](int idx) {
            const int j = idx / W, q = idx - j * W;
            return in[k * C + (long)(r0 + min(j, rn - 1)) * b + min(q, b - 1)];
        },
        [&](int idx, cpx<T> v) {
            const int j = idx / W, q = idx - j * W;
            xs[j * bs + q] = keep(v, j < rn && q < b);
        },
        nthr);
    // a mirrored frequency (half spectrum) reads its stored block transposed
    bool tr;
    const cpx<T> *Gk = G + spec_src(k, Px, Py, kxh, tr) * (long)b * b;
    // loads use clamped addresses, so they issue without branches; values
    // outside the row are masked to zero only when they are used
    int rt = w, p = 16 * rt + i;
    bool prow = p < b;
    const cpx<T> *arow = Gk + (long)min(p, b - 1) * b;
    const cpx<T> *acol = Gk + min(p, b - 1);
    auto tile = [&](int t) {
        rt = t;
        p = 16 * rt + i;
        prow = p < b;
        arow = Gk + (long)min(p, b - 1) * b;
        acol = Gk + min(p, b - 1);
    };
    auto load = [&](cpair<T>(&a)[KC], int t0) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int q = 8 * (t0 + u) + 2 * g;
            if constexpr (EVEN) {
                a[u] = *reinterpret_cast<const cpair<T> *>(arow + min(q, b - 2));
            } else {
                a[u].a = arow[min(q, b - 1)];
                a[u].b = arow[min(q + 1, b - 1)];
            }
        }
    };
    // transposed: A[p][q] = stored[q][p], a column walk (16 lanes of a group
    // read 16 consecutive values of one stored row)
    auto load_tr = [&](cpair<T>(&a)[KC], int t0) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int q = 8 * (t0 + u) + 2 * g;
            a[u].a = acol[(long)min(q, b - 1) * b];
            a[u].b = acol[(long)min(q + 1, b - 1) * b];
        }
    };
    CAcc<T> acc[NT];
    auto compute = [&](const cpair<T>(&a)[KC], int t0) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int t = t0 + u, q = 8 * t + 2 * g;
            if (t < KP) {
                // with b even and q clamped to b - 2, a pair past the row end
                // holds the row's last two values: masked off here
                const cpx<T> a0 = keep(a[u].a, prow && q < b), a1 = keep(a[u].b, prow && q + 1 < b);
                cpair<T> bx[NT];
#pragma unroll
                for (int n = 0; n < NT; ++n) bx[n] = *reinterpret_cast<const cpair<T> *>(xs + (n * 16 + i) * bs + q);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[n].mac_a(a0, bx[n].a);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[n].mac_b(a0, bx[n].a);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[n].mac_a(a1, bx[n].b);
#pragma unroll
                for (int n = 0; n < NT; ++n) acc[n].mac_b(a1, bx[n].b);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int j = n * 16 + i;
            if (j < rn) {
                cpx<T> *o = out + k * C + (long)(r0 + j) * b + 16 * rt;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = Mfma<T>::row(g, v);
                    if (16 * rt + rr < b) o[rr] = acc[n].get(v);
                }
            }
        }
    };
    // loads unconditional (clamped addresses): a load under a branch would
    // make the wait before the other buffer's use cover it too.  The two
    // orientations are two copies of the loop (tr is uniform).  The first
    // chunk of the wave's first tile is issued before the staging barrier.
    auto run = [&](auto ld) {
        cpair<T> a0[KC], a1[KC];
        if (rt < nrt) ld(a0, 0);
        __syncthreads();
        for (int t = w; t < nrt; t += nw) {
            if (t != w) {
                tile(t);
                ld(a0, 0);
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[n].zero();
            for (int t0 = 0; t0 < KP; t0 += 2 * KC) {
                ld(a1, t0 + KC);
                compute(a0, t0);
                ld(a0, t0 + 2 * KC);
                if (t0 + KC < KP) compute(a1, t0 + KC);
            }
            store();
        }
    };
    if (tr)
        run(load_tr);
    else
        run(load);
}

// yhat[k] = G[k] xhat[k] for every frequency k: (b x b) times (b x R).
// Workgroup = frequency k and a block of 16 NT columns, one wave per 16-row
// output tile.  The contraction runs in pairs of k-steps: at pair t, lane
// group g = l / 16 takes q = 8 t + 2 g + h for the two steps h = 0, 1, so one
// load gives a lane the two consecutive values G[k][p][8t + 2g .. +1] and a
// wave's load covers 16 rows x 64 contiguous bytes (f32).  Pairs are loaded
// in chunks of KC, the next chunk's loads issued before the current chunk's
// MFMAs.  The column block of xhat[k] is staged in LDS, row stride 8 KP + 2.
// EVEN: b is even, so a value pair never straddles the end of a row and is
// fetched with one aligned load.
template <typename T, int NT, int KC, bool EVEN>
__global__ void __launch_bounds__(1024) k_prod_mfma(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in,
                                                    int b, int R, int Px, int Py, int kxh,
                                                    cpx<T> *__restrict__ out, const void *const *act) {
    extern __shared__ char smem_raw[];
    // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so XCD x
    // receives ids x, x + 8, ...; it is given one contiguous range of
    // (frequency, column block) items, and the column blocks of a frequency
    // run back to back on the XCD whose L2 holds that frequency's G block
    const int ncb = (R + 16 * NT - 1) / (16 * NT);
    const long P = (long)Px * Py;
    const long nitem = P * ncb, per = (long)gridDim.x >> 3;
    const long item = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (item >= nitem) return;
    const long k = item / ncb;
    prod_mfma_item<T, NT, KC, EVEN>(G, in, b, R, Px, Py, kxh, out, act, k, (int)(item - k * ncb), smem_raw);
}

// The same product with the frequency's spectrum block in LDS.  Workgroup =
// frequency k and a group of CG column tiles of 16; wave w takes column tile
// w % CG and the RT row tiles of group w / CG.  The block is staged once
// (transposed as it is written when the frequency is a mirrored one, zero past
// column b), each wave holds its column tile of xhat[k] in registers for the
// whole contraction (loaded before the staging barrier), and the contraction
// then reads only LDS and registers.  The contraction order (pairs t, lane
// group g, step h) is that of k_prod_mfma, so both give the same bits.
// LDS row stride 8 KP + 2 values: the 16 rows a 16-lane phase reads fall in
// distinct 16-byte bank groups.  KPM: pairs held in registers (KP <= KPM).
// PAIR (half spectrum): workgroup = stored block s = kx Py + ky (kx < kxh);
// the staged block serves its own frequency and, when the mirror frequency
// (Px - kx, -ky) is not itself stored, the mirror too, with the block read
// from LDS by columns (the transpose): each stored block is read from memory
// once per column group instead of twice.
template <typename T, int RT, int KPM, bool EVEN, bool PAIR>
__global__ void __launch_bounds__(1024) k_prod_lds(const cpx<T> *__restrict__ G, const cpx<T> *__restrict__ in,
                                                   int b, int R, int Px, int Py, int kxh, int CG,
                                                   cpx<T> *__restrict__ out, const void *const *act) {
    extern __shared__ char smem_raw[];
    cpx<T> *gs = reinterpret_cast<cpx<T> *>(smem_raw);
    const int KP = (b + 7) >> 3, W = 8 * KP, S = W + 2;
    const int ntc = (R + 15) >> 4, ncg = (ntc + CG - 1) / CG;
    const long P = PAIR ? (long)kxh * Py : (long)Px * Py, nitem = P * ncg, per = (long)gridDim.x >> 3;
    const long item = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (item >= nitem) return;
    const long k = item / ncg;
    const int cg = (int)(item - k * ncg);
    const int cfirst = cg * CG * 16, clast = min(R, cfirst + CG * 16) - 1;
    if (!cols_live(act, cfirst, clast)) return;
    const long C = (long)b * R;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    const int ct = w % CG, rg = w / CG;
    const int c0 = cfirst + ct * 16;
    const bool wlive = c0 <= clast && cols_live(act, c0, min(c0 + 15, clast));
    // the mirror frequency of a stored block (PAIR), when it is not stored
    const int kxs = (int)(k / Py), kys = (int)(k - (long)kxs * Py);
    const bool mir = PAIR && kxs > 0 && Px - kxs >= kxh;
    const long km = (long)(Px - kxs) * Py + (kys == 0 ? 0 : Py - kys);
    // this lane's column of the tile, its xhat values for every pair (zero
    // past row b and past column R)
    auto load_x = [&](long kk, cpair<T>(&xr)[KPM]) {
        const int col = min(c0 + i, R - 1);
        const bool cok = c0 + i < R;
        const cpx<T> *xc = in + kk * C + (long)col * b;
#pragma unroll
        for (int t = 0; t < KPM; ++t) {
            if (t < KP) {
                const int q = 8 * t + 2 * g;
                if constexpr (EVEN) {
                    xr[t] = *reinterpret_cast<const cpair<T> *>(xc + min(q, b - 2));
                } else {
                    xr[t].a = xc[min(q, b - 1)];
                    xr[t].b = xc[min(q + 1, b - 1)];
                }
                xr[t].a = keep(xr[t].a, cok && q < b);
                xr[t].b = keep(xr[t].b, cok && q + 1 < b);
            }
        }
    };
    cpair<T> xr[KPM], xm[PAIR ? KPM : 1];
    load_x(k, xr);
    if constexpr (PAIR) {
        if (mir) load_x(km, xm);
    }
    // the spectrum block, transposed for a mirrored frequency
    bool tr;
    const cpx<T> *Gk = G + (PAIR ? (tr = false, k) : spec_src(k, Px, Py, kxh, tr)) * (long)b * b;
    const int nthr = blockDim.x;
    if (tr) {
        // LDS[p][q] = stored[q][p]: read stored rows (contiguous in p)
        stage<4, cpx<T>>(
            W * b,
            [&](int idx) {
                const int q = idx / b, p = idx - q * b;
                return Gk[(long)min(q, b - 1) * b + p];
            },
            [&](int idx, cpx<T> v) {
                const int q = idx / b, p = idx - q * b;
                gs[p * S + q] = keep(v, q < b);
            },
            nthr);
    } else {
        stage<4, cpx<T>>(
            W * b,
            [&](int idx) {
                const int p = idx / W, q = idx - p * W;
                return Gk[(long)p * b + min(q, b - 1)];
            },
            [&](int idx, cpx<T> v) {
                const int p = idx / W, q = idx - p * W;
                gs[p * S + q] = keep(v, q < b);
            },
            nthr);
    }
    __syncthreads();
    if (!wlive) return;
    const int nrt = (b + 15) >> 4;
    const int j = c0 + i;
    CAcc<T> acc[RT];
    auto store = [&](long kk) {
        if (j <= clast) {
            cpx<T> *o = out + kk * C + (long)j * b;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int rt = rg * RT + r;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rt + Mfma<T>::row(g, v);
                    if (rt < nrt && row < b) o[row] = acc[r].get(v);
                }
            }
        }
    };
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r].zero();
    // rows past b read the last row (results not stored)
    const cpx<T> *arow[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) arow[r] = gs + min(16 * (rg * RT + r) + i, b - 1) * S + 2 * g;
#pragma unroll
    for (int t = 0; t < KPM; ++t) {
        if (t < KP) {
            // row tiles past the last are computed on the clamped rows and
            // not stored (no branch between the instructions)
            cpair<T> a[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) a[r] = *reinterpret_cast<const cpair<T> *>(arow[r] + 8 * t);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r].mac_a(a[r].a, xr[t].a);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r].mac_b(a[r].a, xr[t].a);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r].mac_a(a[r].b, xr[t].b);
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r].mac_b(a[r].b, xr[t].b);
        }
    }
    store(k);
    if constexpr (PAIR) {
        if (!mir) return;
        // the mirror: A[p][q] = block[q][p], LDS rows q (clamped to the last
        // row; its xhat values are zero there) at column p
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r].zero();
        const cpx<T> *acol[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) acol[r] = gs + min(16 * (rg * RT + r) + i, b - 1);
#pragma unroll
        for (int t = 0; t < KPM; ++t) {
            if (t < KP) {
                const int q = 8 * t + 2 * g;
                cpair<T> a[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    a[r].a = acol[r][min(q, b - 1) * S];
                    a[r].b = acol[r][min(q + 1, b - 1) * S];
                }
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r].mac_a(a[r].a, xm[t].a);
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r].mac_b(a[r].a, xm[t].a);
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r].mac_a(a[r].b, xm[t].b);
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r].mac_b(a[r].b, xm[t].b);
            }
        }
        store(km);
    }
}

// ---------------------------------------------------------------- rim
// One slab of 64 element columns e0 .. e0 + 63 and a block of 16 NT
// right-hand sides, 4 waves:
//   uA[e][j]   = sum_row BE[row][e] x_r[row][j]      (y_A, wave w: e in [16 w, 16 w + 16))
//   part[row][j] = sum_{e in slab} B[row][e] x_A[e][j] (slab partial of y_r)
// The x_A slab sits in LDS; the rim rows are taken in chunks of RCH, whose B
// (and BE) rows and x_r entries are staged in LDS, so each B value is read from
// memory once for both products.  The partials use the slab layout of the
// general rim pass and are finished by the same kernel.
template <typename T, typename In, typename Out, int NT, int RCH, bool NBE>
__device__ __forceinline__ void rim_mfma_tile(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                              Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                              cpx<T> *__restrict__ part, int slab, int cb, char *smem) {
    constexpr int TE = 64, LS = TE + 1, NC = 16 * NT, XS = RCH + 1;
    cpx<T> *xa = reinterpret_cast<cpx<T> *>(smem);       // [NC][LS]
    cpx<T> *xr = xa + NC * LS;                             // [NC][XS]
    cpx<T> *bs = xr + NC * XS;                             // [RCH][LS]
    cpx<T> *be = NBE ? bs + RCH * LS : bs;                 // [RCH][LS]
    const int rb = cb * NC;
    const long e0 = (long)slab * TE;
    const int rn = min(NC, R - rb);
    if (!cols_live((const void *const *)x.tab, rb, rb + rn - 1)) return;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    // column pointers of the block; idle and missing columns read a live one
    // (their values are masked to zero)
    __shared__ const In *colp[NC];
    __shared__ int colok[NC];
    if (threadIdx.x == 0) {
        const In *live = nullptr;
        for (int j = 0; j < rn && !live; ++j) live = x.col(rb + j);
        for (int j = 0; j < NC; ++j) {
            const In *c = j < rn ? x.col(rb + j) : nullptr;
            colok[j] = c != nullptr;
            colp[j] = c ? c : live;
        }
    }
    __syncthreads();
    const long elast = N - 1;
    stage<4, In>(
        NC * TE, [&](int idx) { return colp[idx / TE][min(e0 + idx % TE, elast)]; },
        [&](int idx, In v) {
            const int j = idx / TE, t = idx - j * TE;
            xa[j * LS + t] = keep(cvt<T>(v), colok[j] && e0 + t < N);
        });
    CAcc<T> ua[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) ua[n].zero();
    for (int rc = 0; rc < Nr; rc += RCH) {
        __syncthreads();
        auto boff = [&](int idx) {
            return (long)min(rc + idx / TE, Nr - 1) * N + min(e0 + idx % TE, elast);
        };
        auto bok = [&](int idx) { return rc + idx / TE < Nr && e0 + idx % TE < N; };
        stage<4, cpx<T>>(
            RCH * TE, [&](int idx) { return B[boff(idx)]; },
            [&](int idx, cpx<T> v) { bs[(idx / TE) * LS + idx % TE] = keep(v, bok(idx)); });
        if constexpr (NBE)
            stage<4, cpx<T>>(
                RCH * TE, [&](int idx) { return BE[boff(idx)]; },
                [&](int idx, cpx<T> v) { be[(idx / TE) * LS + idx % TE] = keep(v, bok(idx)); });
        stage<4, In>(
            NC * RCH, [&](int idx) { return colp[idx / RCH][N + min(rc + idx % RCH, Nr - 1)]; },
            [&](int idx, In v) {
                const int j = idx / RCH, u = idx - j * RCH;
                xr[j * XS + u] = keep(cvt<T>(v), colok[j] && rc + u < Nr);
            });
        __syncthreads();
        // y_A part: A[e][u] = BE[rc + u][e], k = u = 4 s + g (steps past the last rim row skipped)
        const int ks1 = (min(RCH, Nr - rc) + 3) >> 2;
#pragma unroll 4
        for (int s = 0; s < ks1; ++s) {
            const int u = 4 * s + g;
            const cpx<T> a = be[u * LS + 16 * w + i];
            cpx<T> bx[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) bx[n] = xr[(n * 16 + i) * XS + u];
#pragma unroll
            for (int n = 0; n < NT; ++n) ua[n].mac_a(a, bx[n]);
#pragma unroll
            for (int n = 0; n < NT; ++n) ua[n].mac_b(a, bx[n]);
        }
        // slab partials of y_r: A[row][t] = B[rc + row][e0 + t], k = t = 4 s + g
        for (int mt = w; mt < RCH / 16 && rc + 16 * mt < Nr; mt += 4) {
            CAcc<T> pa[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) pa[n].zero();
#pragma unroll 4
            for (int s = 0; s < TE / 4; ++s) {
                const int t = 4 * s + g;
                const cpx<T> a = bs[(16 * mt + i) * LS + t];
                cpx<T> bx[NT];
#pragma unroll
                for (int n = 0; n < NT; ++n) bx[n] = xa[(n * 16 + i) * LS + t];
#pragma unroll
                for (int n = 0; n < NT; ++n) pa[n].mac_a(a, bx[n]);
#pragma unroll
                for (int n = 0; n < NT; ++n) pa[n].mac_b(a, bx[n]);
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int j = n * 16 + i;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rc + 16 * mt + Mfma<T>::row(g, v);
                    if (row < Nr && j < rn) part[((long)slab * Nr + row) * R + rb + j] = pa[n].get(v);
                }
            }
        }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int j = n * 16 + i;
        Out *yc = j < rn ? y.col(rb + j) : nullptr;
        if (yc) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long e = e0 + 16 * w + Mfma<T>::row(g, v);
                if (e < N) yc[e] = cvt<typename Out::value_type>(ua[n].get(v));
            }
        }
    }
}

template <typename T, typename In, typename Out, int NT, int RCH, bool NBE>
__global__ void __launch_bounds__(256) k_rim_mfma(const cpx<T> *__restrict__ B, const cpx<T> *__restrict__ BE,
                                                  Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                                                  cpx<T> *__restrict__ part) {
    extern __shared__ char smem_raw[];
    rim_mfma_tile<T, In, Out, NT, RCH, NBE>(B, BE, x, y, R, N, Nr, part, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T>
constexpr int rim_nt() { return sizeof(T) == 4 ? 2 : 1; }
template <typename T>
constexpr int rim_rch() { return sizeof(T) == 4 ? 64 : 32; }

}  // namespace tp
