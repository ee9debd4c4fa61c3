// Restarted GMRES for Z x = v (eq. MoMMatrixEq), one independent Krylov space
// per right-hand side, driven by a per-column state machine that lives in
// device memory.
//
// A "super-step" is a fixed sequence of launches:
//   advance  -> operator application(s) -> CGS2 (dots, update, dots, update+norm)
//   -> finish (Hessenberg column, Givens rotation, residual estimate)
//   -> x update (triangular solve + x += V y) -> true residual -> normalise.
// Every kernel reads each column's phase and Arnoldi index from device memory
// and does nothing for columns in other phases, so the same launch sequence
// serves every column at every step and the host only polls for completion.
//
// Column phases:
//   ARN      Arnoldi step j: w = Z V_j is orthogonalised into V_{j+1}
//   UPD      cycle over (estimate below threshold, j + 1 == m, breakdown or
//            iteration cap): solve R y = g, x += V y
//   PRE_RES  x updated; its operator application happens next super-step
//   RES      r = v - Z x (FP64): stop, or start a cycle with V_0 = r / ||r||
//   DONE     final
// Plain mode (TP_FP64) applies the FP64 operator both in ARN and RES.  Mixed
// mode (TP_MIXED, iterative refinement) applies the FP32 operator in ARN, the
// FP64 one in RES, and each inner cycle stops at inner_tol * ||r||.  All
// Krylov vectors, inner products, norms and the Hessenberg least-squares
// problem are FP64.
#include <cmath>
#include <cstring>
#include <vector>

#include "tp_internal.h"

namespace tp {

enum : int { PH_IDLE = 0, PH_ARN = 1, PH_UPD = 2, PH_PRE_RES = 3, PH_RES = 4, PH_DONE = 5 };

struct SlotDev {
    const c128 *v;
    c128 *x;
    double tol, inner_tol;
    int max_iter, max_outer;
    int phase, xzero, j, k;
    int iters, outer, status, needs_norm;
    int first, pad0;
    double nrm, beta, vnorm, relres, thr, est;
};

constexpr int kThreads = 256;
constexpr int kEPT = 4;                       // vector elements per thread
constexpr int kChunk = kThreads * kEPT;       // elements per workgroup
constexpr int kMaxRestart = 512;

struct Eng {
    long Nt;
    int m, nch, mixed;
    SlotDev *slots;
    c128 *V, *W, *H, *sn, *g, *h1, *h2, *part;
    double *cs, *pn;
    unsigned *cnt;
    const c128 **tin;   // operator input per column (ARN, and RES in plain mode)
    c128 **tout;
    const c128 **rin;   // FP64 residual input per column (mixed mode)
    c128 **rout;
    __device__ c128 *vec(int s, int i) const { return V + ((long)s * (m + 1) + i) * Nt; }
};

static size_t a256(size_t n) { return (n + 255) & ~(size_t)255; }

struct EngLayout {
    size_t slots, V, W, H, sn, g, h1, h2, part, cs, pn, cnt, tabs, total;
};

static EngLayout eng_layout(long Nt, int m, int R) {
    EngLayout L;
    const size_t nch = (size_t)((Nt + kChunk - 1) / kChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += a256(bytes);
        return o;
    };
    L.slots = take(sizeof(SlotDev) * R);
    L.V = take((size_t)R * (m + 1) * Nt * 16);
    L.W = take((size_t)R * Nt * 16);
    L.H = take((size_t)R * (m + 1) * m * 16);
    L.sn = take((size_t)R * m * 16);
    L.g = take((size_t)R * (m + 1) * 16);
    L.h1 = take((size_t)R * (m + 1) * 16);
    L.h2 = take((size_t)R * (m + 1) * 16);
    L.part = take((size_t)R * (m + 1) * nch * 16);
    L.cs = take((size_t)R * m * 8);
    L.pn = take((size_t)R * nch * 16);
    L.cnt = take((size_t)R * 8 * 4);
    L.tabs = take((size_t)R * 4 * sizeof(void *));
    L.total = off;
    return L;
}

size_t solver_ws_bytes(long Nt, int restart, int max_rhs) { return eng_layout(Nt, restart, max_rhs).total; }

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ c128 shfl_xor_c(c128 v, int mk_) {
    return c128{__shfl_xor(v.x, mk_, 64), __shfl_xor(v.y, mk_, 64)};
}
__device__ __forceinline__ double shfl_xor_d(double v, int mk_) { return __shfl_xor(v, mk_, 64); }

// Sum over the 256 threads of the block; the result is valid in thread 0.
__device__ __forceinline__ c128 block_sum(c128 v) {
    __shared__ c128 red[kThreads / 64];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + shfl_xor_c(v, m);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    c128 s = c128{0, 0};
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) s = s + red[i];
    return s;
}
__device__ __forceinline__ double block_sum_d(double v) {
    __shared__ double redd[kThreads / 64];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) redd[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kThreads / 64; ++i) s += redd[i];
    return s;
}

// Block-completion counter: returns true in every thread of the last block
// to finish (of `total` participating blocks) and resets the counter.
__device__ __forceinline__ bool last_block(unsigned *cnt, unsigned total) {
    __shared__ int am_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(cnt, 1u);
        am_last = (t + 1 == total);
        if (am_last) *cnt = 0;
    }
    __syncthreads();
    if (am_last) __threadfence();
    return am_last != 0;
}

__device__ __forceinline__ double cabs2(c128 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------ kernels
__global__ void k_advance(Eng E, int nslots) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    SlotDev &S = E.slots[s];
    S.needs_norm = 0;
    if (S.phase == PH_PRE_RES) S.phase = PH_RES;
}

// part[s][i][chunk] = sum_{n in chunk} conj(V_i[n]) w[n], w = V_{j+1}; the last
// block sums the chunks in order into h (pass 0 -> h1, pass 1 -> h2).
__global__ void __launch_bounds__(kThreads) k_dots(Eng E, int pass) {
    const int s = blockIdx.z, i = blockIdx.y, ch = blockIdx.x;
    const SlotDev &S = E.slots[s];
    if (S.phase != PH_ARN) return;
    const int j = S.j;
    if (i > j) return;
    const c128 *vi = E.vec(s, i), *w = E.vec(s, j + 1);
    c128 acc = c128{0, 0};
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
        const long n = (long)ch * kChunk + t * kThreads + threadIdx.x;
        if (n < E.Nt) acc = cmac_conj(acc, vi[n], w[n]);
    }
    acc = block_sum(acc);
    c128 *part = E.part + (long)s * (E.m + 1) * E.nch;
    if (threadIdx.x == 0) part[(long)i * E.nch + ch] = acc;
    if (last_block(E.cnt + s * 8 + pass, (unsigned)((j + 1) * E.nch))) {
        c128 *h = (pass == 0 ? E.h1 : E.h2) + (long)s * (E.m + 1);
        for (int ii = threadIdx.x; ii <= j; ii += blockDim.x) {
            c128 t = c128{0, 0};
            for (int c = 0; c < E.nch; ++c) t = t + part[(long)ii * E.nch + c];
            h[ii] = t;
        }
    }
}

// w -= sum_i V_i h_i (h = h1 or h2); on the second pass also ||w||^2 -> nrm.
__global__ void __launch_bounds__(kThreads) k_update(Eng E, int pass) {
    __shared__ c128 hs[kMaxRestart + 1];
    const int s = blockIdx.y, ch = blockIdx.x;
    SlotDev &S = E.slots[s];
    if (S.phase != PH_ARN) return;
    const int j = S.j;
    const c128 *h = (pass == 0 ? E.h1 : E.h2) + (long)s * (E.m + 1);
    for (int i = threadIdx.x; i <= j; i += blockDim.x) hs[i] = h[i];
    __syncthreads();
    c128 *w = E.vec(s, j + 1);
    c128 wv[kEPT];
    long idx[kEPT];
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
        idx[t] = (long)ch * kChunk + t * kThreads + threadIdx.x;
        wv[t] = idx[t] < E.Nt ? w[idx[t]] : c128{0, 0};
    }
    for (int i = 0; i <= j; ++i) {
        const c128 *vi = E.vec(s, i);
        const c128 hn = c128{-hs[i].x, -hs[i].y};
#pragma unroll
        for (int t = 0; t < kEPT; ++t)
            if (idx[t] < E.Nt) wv[t] = cmac(wv[t], vi[idx[t]], hn);
    }
    double nn = 0;
#pragma unroll
    for (int t = 0; t < kEPT; ++t)
        if (idx[t] < E.Nt) {
            w[idx[t]] = wv[t];
            nn += cabs2(wv[t]);
        }
    if (pass == 1) {
        nn = block_sum_d(nn);
        double *pn = E.pn + (long)s * E.nch * 2;
        if (threadIdx.x == 0) pn[ch] = nn;
        if (last_block(E.cnt + s * 8 + 2, (unsigned)E.nch)) {
            if (threadIdx.x == 0) {
                double t = 0;
                for (int c = 0; c < E.nch; ++c) t += pn[c];
                S.nrm = sqrt(t);
            }
        }
    }
}

// Hessenberg column j, previous Givens rotations, new rotation, residual
// estimate |g_{j+1}|, and the phase decision.  One lane per column: the work
// is O(j).
__global__ void k_finish(Eng E, int nslots) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    SlotDev &S = E.slots[s];
    if (S.phase != PH_ARN) return;
    const int m = E.m, j = S.j;
    const c128 *h1 = E.h1 + (long)s * (m + 1), *h2 = E.h2 + (long)s * (m + 1);
    c128 *H = E.H + (long)s * (m + 1) * m, *sn = E.sn + (long)s * m, *g = E.g + (long)s * (m + 1);
    double *cs = E.cs + (long)s * m;
    c128 *Hj = H + (long)j * (m + 1);
    for (int i = 0; i <= j; ++i) Hj[i] = h1[i] + h2[i];
    const double nrm = S.nrm;
    const c128 below = c128{nrm, 0};
    for (int i = 0; i < j; ++i) {   // apply rotation i to rows i, i+1
        const c128 a = Hj[i], b = Hj[i + 1];
        const c128 sv = sn[i];
        const c128 t = c128{cs[i] * a.x, cs[i] * a.y} + sv * b;
        const c128 u = c128{cs[i] * b.x, cs[i] * b.y} - conjg(sv) * a;
        Hj[i] = t;
        Hj[i + 1] = u;
    }
    // new rotation zeroing the subdiagonal entry (real, >= 0)
    const c128 a = Hj[j];
    const double aa = sqrt(cabs2(a));
    double c;
    c128 sv;
    c128 diag;
    if (aa == 0.0) {
        c = 0.0;
        sv = c128{1, 0};
        diag = below;
    } else {
        const double rho = sqrt(aa * aa + nrm * nrm);
        c = aa / rho;
        sv = c128{a.x / aa * nrm / rho, a.y / aa * nrm / rho};    // (a/|a|) b / rho, b real
        diag = c128{a.x / aa * rho, a.y / aa * rho};
    }
    cs[j] = c;
    sn[j] = sv;
    Hj[j] = diag;
    const c128 gj = g[j];
    g[j + 1] = c128{0, 0} - conjg(sv) * gj;
    g[j] = c128{c * gj.x, c * gj.y};
    const double est = sqrt(cabs2(g[j + 1]));
    S.est = est;
    S.k = j + 1;
    S.iters += 1;
    const bool converged = est <= S.thr;
    const bool dead = !(nrm > 1e-300) || !(est == est);
    if (!converged && !dead && j + 1 < m && S.iters < S.max_iter) {
        S.j = j + 1;
        S.needs_norm = 1;
        E.tin[s] = E.vec(s, j + 1);
        E.tout[s] = E.vec(s, j + 2);
    } else {
        S.phase = PH_UPD;
        E.tin[s] = nullptr;
        E.tout[s] = nullptr;
    }
}

// Back substitution R y = g (k x k upper triangular, R in H after the
// rotations), then x += sum_i V_i y_i.  Every block solves the small system
// itself; the last block moves the column to PRE_RES.
__global__ void __launch_bounds__(kThreads) k_xupdate(Eng E) {
    __shared__ c128 ys[kMaxRestart];
    const int s = blockIdx.y, ch = blockIdx.x;
    SlotDev &S = E.slots[s];
    if (S.phase != PH_UPD) return;
    const int m = E.m, k = S.k;
    const c128 *H = E.H + (long)s * (m + 1) * m, *g = E.g + (long)s * (m + 1);
    for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = g[i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        if (threadIdx.x == 0) {
            const c128 d = H[(long)i * (m + 1) + i];
            const double dd = cabs2(d);
            const c128 yi = ys[i];
            ys[i] = dd > 0 ? c128{(yi.x * d.x + yi.y * d.y) / dd, (yi.y * d.x - yi.x * d.y) / dd} : c128{0, 0};
        }
        __syncthreads();
        const c128 yi = ys[i];
        for (int l = threadIdx.x; l < i; l += blockDim.x) ys[l] = ys[l] - H[(long)i * (m + 1) + l] * yi;
        __syncthreads();
    }
    c128 *x = S.x;
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
        const long n = (long)ch * kChunk + t * kThreads + threadIdx.x;
        if (n < E.Nt) {
            c128 acc = x[n];
            for (int i = 0; i < k; ++i) acc = cmac(acc, E.vec(s, i)[n], ys[i]);
            x[n] = acc;
        }
    }
    if (last_block(E.cnt + s * 8 + 3, (unsigned)E.nch)) {
        if (threadIdx.x == 0) {
            S.phase = PH_PRE_RES;
            S.xzero = 0;
            if (E.mixed) {
                E.rin[s] = x;
                E.rout[s] = E.W + (long)s * E.Nt;
            } else {
                E.tin[s] = x;
                E.tout[s] = E.W + (long)s * E.Nt;
            }
        }
    }
}

// r = v - Z x (Z x in W, or x == 0), stored in V_0; ||r||, ||v||; decision.
__global__ void __launch_bounds__(kThreads) k_residual(Eng E) {
    const int s = blockIdx.y, ch = blockIdx.x;
    SlotDev &S = E.slots[s];
    if (S.phase != PH_RES) return;
    const c128 *v = S.v, *Wz = E.W + (long)s * E.Nt;
    c128 *r = E.vec(s, 0);
    const bool xz = S.xzero != 0;
    double rr = 0, vv = 0;
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
        const long n = (long)ch * kChunk + t * kThreads + threadIdx.x;
        if (n < E.Nt) {
            const c128 vn = v[n];
            const c128 rn = xz ? vn : vn - Wz[n];
            r[n] = rn;
            rr += cabs2(rn);
            vv += cabs2(vn);
        }
    }
    rr = block_sum_d(rr);
    vv = block_sum_d(vv);
    double *pn = E.pn + (long)s * E.nch * 2;
    if (threadIdx.x == 0) {
        pn[ch] = rr;
        pn[E.nch + ch] = vv;
    }
    if (last_block(E.cnt + s * 8 + 4, (unsigned)E.nch) && threadIdx.x == 0) {
        double tr = 0, tv = 0;
        for (int c = 0; c < E.nch; ++c) {
            tr += pn[c];
            tv += pn[E.nch + c];
        }
        const double beta = sqrt(tr), vn = sqrt(tv);
        S.vnorm = vn;
        const double rel = vn > 0 ? beta / vn : (beta > 0 ? INFINITY : 0.0);
        S.relres = rel;
        if (!S.first) S.outer += 1;
        S.first = 0;
        E.tin[s] = nullptr;
        E.tout[s] = nullptr;
        if (E.mixed) {
            E.rin[s] = nullptr;
            E.rout[s] = nullptr;
        }
        if (rel <= S.tol) {
            S.phase = PH_DONE;
            S.status = TP_OK;
        } else if (!(rel == rel) || rel == INFINITY) {
            S.phase = PH_DONE;
            S.status = TP_E_BREAKDOWN;
        } else if (S.iters >= S.max_iter || S.outer >= S.max_outer) {
            S.phase = PH_DONE;
            S.status = TP_E_NOCONV;
        } else {
            S.phase = PH_ARN;
            S.j = 0;
            S.k = 0;
            S.beta = beta;
            S.nrm = beta;
            S.needs_norm = 1;
            const double plain_thr = 0.5 * S.tol * vn;
            S.thr = E.mixed ? fmax(S.inner_tol * beta, plain_thr) : plain_thr;
            E.g[(long)s * (E.m + 1)] = c128{beta, 0};
            E.tin[s] = E.vec(s, 0);
            E.tout[s] = E.vec(s, 1);
        }
    }
}

// V_j *= 1 / nrm for columns that start or continue a cycle.
__global__ void __launch_bounds__(kThreads) k_normalize(Eng E) {
    const int s = blockIdx.y, ch = blockIdx.x;
    const SlotDev &S = E.slots[s];
    if (!S.needs_norm || S.phase != PH_ARN) return;
    c128 *vj = E.vec(s, S.j);
    const double sc = S.nrm > 0 ? 1.0 / S.nrm : 0.0;
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
        const long n = (long)ch * kChunk + t * kThreads + threadIdx.x;
        if (n < E.Nt) vj[n] = c128{vj[n].x * sc, vj[n].y * sc};
    }
}

__global__ void k_zero_cols(c128 *x, long ld, long Nt) {
    const int r = blockIdx.y;
    for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < Nt; n += (long)gridDim.x * blockDim.x)
        x[(long)r * ld + n] = c128{0, 0};
}

__global__ void k_clear_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// --------------------------------------------------------------- driver
static hipError_t super_step(tp_plan pl, const Eng &E, int nslots, hipStream_t st) {
    const int m = E.m;
    hipLaunchKernelGGL(k_advance, dim3((nslots + 63) / 64), dim3(64), 0, st, E, nslots);
    hipError_t e;
    if (E.mixed) {
        e = matvec_fp32_wide(pl, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout}, nslots, st);
        if (e) return e;
        e = matvec_fp64(pl, Cols<const c128>{nullptr, 0, E.rin}, Cols<c128>{nullptr, 0, E.rout}, nslots, st);
    } else {
        e = matvec_fp64(pl, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout}, nslots, st);
    }
    if (e) return e;
    const dim3 gd(E.nch, m + 1, nslots), gv(E.nch, nslots), blk(kThreads);
    hipLaunchKernelGGL(k_dots, gd, blk, 0, st, E, 0);
    hipLaunchKernelGGL(k_update, gv, blk, 0, st, E, 0);
    hipLaunchKernelGGL(k_dots, gd, blk, 0, st, E, 1);
    hipLaunchKernelGGL(k_update, gv, blk, 0, st, E, 1);
    hipLaunchKernelGGL(k_finish, dim3((nslots + 63) / 64), dim3(64), 0, st, E, nslots);
    hipLaunchKernelGGL(k_xupdate, gv, blk, 0, st, E);
    hipLaunchKernelGGL(k_residual, gv, blk, 0, st, E);
    hipLaunchKernelGGL(k_normalize, gv, blk, 0, st, E);
    return hipGetLastError();
}

tp_status solve_run(tp_plan pl, const c128 *v, long ldv, c128 *x, long ldx, int nrhs, const tp_solve_opts &o,
                    tp_solve_info *info, hipStream_t st) {
    const long Nt = pl->Nt;
    const int m = o.restart;
    // the engine is carved for the plan's restart; a shorter o.restart uses a prefix
    EngLayout L = eng_layout(Nt, pl->restart, pl->max_rhs);
    char *wsb = (char *)pl->rim_part + a256((size_t)pl->rim_nslab * (pl->Nr ? pl->Nr : 1) * pl->max_rhs * 16);
    Eng E;
    E.Nt = Nt;
    E.m = pl->restart;
    E.nch = (int)((Nt + kChunk - 1) / kChunk);
    E.mixed = o.mode == TP_MIXED;
    E.slots = (SlotDev *)(wsb + L.slots);
    E.V = (c128 *)(wsb + L.V);
    E.W = (c128 *)(wsb + L.W);
    E.H = (c128 *)(wsb + L.H);
    E.sn = (c128 *)(wsb + L.sn);
    E.g = (c128 *)(wsb + L.g);
    E.h1 = (c128 *)(wsb + L.h1);
    E.h2 = (c128 *)(wsb + L.h2);
    E.part = (c128 *)(wsb + L.part);
    E.cs = (double *)(wsb + L.cs);
    E.pn = (double *)(wsb + L.pn);
    E.cnt = (unsigned *)(wsb + L.cnt);
    void **tabs = (void **)(wsb + L.tabs);
    E.tin = (const c128 **)tabs;
    E.tout = (c128 **)(tabs + pl->max_rhs);
    E.rin = (const c128 **)(tabs + 2 * pl->max_rhs);
    E.rout = (c128 **)(tabs + 3 * pl->max_rhs);

    // host-side initial state, copied once
    std::vector<SlotDev> hs(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        SlotDev &S = hs[r];
        std::memset(&S, 0, sizeof(S));
        S.v = v + (long)r * ldv;
        S.x = x + (long)r * ldx;
        S.tol = o.tol;
        S.inner_tol = o.inner_tol;
        S.max_iter = o.max_iter;
        S.max_outer = o.max_outer;
        S.first = 1;
        if (o.x0_given) {
            S.phase = PH_PRE_RES;   // true residual of x0 first
            S.xzero = 0;
        } else {
            S.phase = PH_RES;
            S.xzero = 1;
        }
    }
    // a shorter restart than the plan's uses a prefix of each per-column region
    E.m = m;
    std::vector<void *> htab(4 * (size_t)pl->max_rhs, nullptr);
    for (int r = 0; r < nrhs; ++r)
        if (o.x0_given) {
            if (E.mixed) {
                htab[2 * pl->max_rhs + r] = hs[r].x;
                htab[3 * pl->max_rhs + r] = E.W + (long)r * Nt;
            } else {
                htab[r] = hs[r].x;
                htab[pl->max_rhs + r] = E.W + (long)r * Nt;
            }
        }
    hipError_t e;
    if ((e = hipMemcpyAsync(E.slots, hs.data(), sizeof(SlotDev) * nrhs, hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(tabs, htab.data(), sizeof(void *) * htab.size(), hipMemcpyHostToDevice, st)))
        return hip_fail(e, "solver state upload");
    hipLaunchKernelGGL(k_clear_u32, dim3((nrhs * 8 + 255) / 256), dim3(256), 0, st, E.cnt, nrhs * 8);
    if (!o.x0_given)
        hipLaunchKernelGGL(k_zero_cols, dim3(256, nrhs), dim3(256), 0, st, x, ldx, Nt);
    if ((e = hipGetLastError())) return hip_fail(e, "solver init");

    std::vector<SlotDev> snap(nrhs);
    const long max_steps = (long)o.max_iter * 2 + (long)o.max_outer * 4 + 16;
    long step = 0;
    bool done = false;
    while (!done) {
        for (int t = 0; t < 4 && step < max_steps; ++t, ++step)
            if ((e = super_step(pl, E, nrhs, st))) return hip_fail(e, "solver step");
        if ((e = hipMemcpyAsync(snap.data(), E.slots, sizeof(SlotDev) * nrhs, hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            return hip_fail(e, "solver poll");
        done = true;
        for (int r = 0; r < nrhs; ++r)
            if (snap[r].phase != PH_DONE) done = false;
        if (step >= max_steps) break;
    }
    tp_status ret = TP_OK;
    for (int r = 0; r < nrhs; ++r) {
        const SlotDev &S = snap[r];
        info[r].iters = S.iters;
        info[r].outer_iters = S.outer;
        info[r].relres = S.relres;
        info[r].status = S.phase == PH_DONE ? S.status : TP_E_NOCONV;
        if (info[r].status != TP_OK && ret == TP_OK) ret = (tp_status)info[r].status;
    }
    if (ret == TP_E_NOCONV) set_error("at least one column missed the tolerance");
    if (ret == TP_E_BREAKDOWN) set_error("Krylov breakdown or non-finite residual");
    return ret;
}

}  // namespace tp
