// Restarted GMRES for Z x = v (eq. MoMMatrixEq), one independent Krylov space
// per right-hand side, driven by a per-column state machine in device memory.
//
// A super-step is a fixed sequence of launches, captured once as a HIP graph
// and replayed:
//   commit   apply last step's decisions: next phase, Arnoldi index, operator
//            input/output tables; scale a fresh residual into V_0
//   operator w = Z V_j (Arnoldi columns), W = Z x (residual columns)
//   dots     partial h1 = V^H w                      (per element range)
//   orth1    h1; w' = w - V h1; partial h2 = V^H w', ||w'||^2
//   orth2    h2; w'' = w' - V h2; V_{j+1} = w'' / ||w''|| with
//            ||w''||^2 = ||w'||^2 - ||h2||^2; Hessenberg column, Givens
//            rotation and residual estimate (first block of each column)
//   tail     columns whose cycle ended: R y = g, x += V y;
//            residual columns: r = v - W into V_0, partial ||r||^2, ||v||^2
// Classical Gram-Schmidt with one reorthogonalisation (CGS2) in FP64.
//
// Every kernel reads the column states committed at the start of its
// super-step (state[parity]) and the decisions of earlier kernels; the commit
// kernel writes state[parity] from state[parity ^ 1].  No kernel reads a
// field that another block of the same kernel writes, and every reduction
// sums fixed partial slots in a fixed order (deterministic, batch-invariant).
//
// Plain mode (TP_FP64) applies the FP64 operator for both column kinds.  Mixed
// mode applies the FP32 operator to Arnoldi columns and the FP64 operator to
// residual columns (iterative refinement); each inner cycle stops when the
// estimate drops below inner_tol * ||r||.  Krylov vectors, inner products,
// norms and the small least-squares problem are FP64 throughout.
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "tp_internal.h"

namespace tp {

enum : int { PH_IDLE = 0, PH_INIT = 1, PH_ARN = 2, PH_RES = 3, PH_DONE = 4 };

// committed per-column state (two copies, by super-step parity)
struct SlotState {
    int phase, j, xzero, iters;
    int outer, status, first, pend;    // pend: a preconditioned x update waits in W (RES)
    double thr, beta, vnorm, relres;
};
// fixed per-solve column data
struct SlotConst {
    const c128 *v;
    c128 *x;
    double tol, inner_tol;
    int max_iter, max_outer;
};
// decision of the Arnoldi step of the current super-step (orth2, first block)
struct SlotDec {
    int end, k, breakdown, pad;
    double est, nrm;
};

// Vector kernels use 1024-thread blocks: 256 element lanes x 4 groups of
// basis vectors (group g takes V_i with i = g mod 4), so one pass issues up to
// 16 independent loads per thread and needs a single round of memory latency.
constexpr int kThreads = 1024;
constexpr int kLanes = 256;
constexpr int kGroups = 4;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBlocks = 512;        // element ranges per column
constexpr int kMaxRestart = 512;
constexpr int kG = 16;                 // basis vectors per group and pass
constexpr int kMaxEPT = 2;             // element rounds of 256 per block (Nt <= 262144)

struct Eng {
    long Nt;
    int m, nb, mixed;
    long span;                         // elements per range
    SlotState *st;                     // [2][nslots]
    SlotConst *sc;
    SlotDec *dec;
    c128 *V, *W, *H, *sn, *g, *h1, *y;
    c128 *P1, *P2;                     // [slot][m + 1][nb] partial inner products
    double *cs, *PN, *PR;              // [slot][nb] ||w'||^2; [slot][2][nb] ||r||^2, ||v||^2
    const c128 **tin;                  // operator tables (Arnoldi; plain: both kinds)
    c128 **tout;
    const c128 **rin;                  // FP64 residual tables (mixed)
    c128 **rout;
    const c128 **pin;                  // preconditioner tables: out = base + M^-1 in
    c128 **pout;
    const c128 **pbase;
    int nslots;
    int prec;                          // right preconditioning on
    __device__ c128 *vec(int s, int i) const { return V + ((long)s * (m + 1) + i) * Nt; }
};

static size_t a256(size_t n) { return (n + 255) & ~(size_t)255; }

struct EngLayout {
    size_t st, sc, dec, V, W, H, sn, g, h1, y, P1, P2, cs, PN, PR, tabs, total;
};

static EngLayout eng_layout(long Nt, int m, int R) {
    EngLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += a256(bytes);
        return o;
    };
    L.st = take(2 * sizeof(SlotState) * R);
    L.sc = take(sizeof(SlotConst) * R);
    L.dec = take(sizeof(SlotDec) * R);
    L.V = take((size_t)R * (m + 1) * Nt * 16);
    L.W = take((size_t)R * Nt * 16);
    L.H = take((size_t)R * (m + 1) * m * 16);
    L.sn = take((size_t)R * m * 16);
    L.g = take((size_t)R * (m + 1) * 16);
    L.h1 = take((size_t)R * (m + 1) * 16);
    L.y = take((size_t)R * (m + 1) * 16);
    L.P1 = take((size_t)R * (m + 1) * kMaxBlocks * 16);
    L.P2 = take((size_t)R * (m + 1) * kMaxBlocks * 16);
    L.cs = take((size_t)R * m * 8);
    L.PN = take((size_t)R * kMaxBlocks * 8);
    L.PR = take((size_t)R * 2 * kMaxBlocks * 8);
    L.tabs = take((size_t)R * 7 * sizeof(void *));
    L.total = off;
    return L;
}

size_t solver_ws_bytes(long Nt, int restart, int max_rhs) { return eng_layout(Nt, restart, max_rhs).total; }

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ c128 shfl_xor_c(c128 v, int mk_) {
    return c128{__shfl_xor(v.x, mk_, 64), __shfl_xor(v.y, mk_, 64)};
}
__device__ __forceinline__ double cabs2(c128 a) { return a.x * a.x + a.y * a.y; }

// Sums over the 64 lanes of a wave of 16 values per lane, by a butterfly that
// halves the values each lane keeps at every exchange (17 exchanges instead of
// 16 x 6).  Lane l returns the total of value index (l >> 2) & 15.
template <int HALF, int MSK>
__device__ __forceinline__ void tsum_step(c128 (&v)[16], int lane) {
    const bool hi = (lane & MSK) != 0;
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        if constexpr (MSK >= 16) {
            v[q] = half_sum<MSK>(v[q], v[HALF + q]);   // permlane swap of the two halves
        } else {
            const c128 mine = hi ? v[HALF + q] : v[q];
            const c128 oth = hi ? v[q] : v[HALF + q];
            v[q] = mine + (MSK == 8 ? dpp<kDppRor8>(oth) : shfl_xor_c(oth, MSK));
        }
    }
}
__device__ __forceinline__ c128 wave_tsum16(c128 (&v)[16]) {
    const int lane = threadIdx.x & 63;
    tsum_step<8, 32>(v, lane);
    tsum_step<4, 16>(v, lane);
    tsum_step<2, 8>(v, lane);
    tsum_step<1, 4>(v, lane);
    return xor_sum<1>(xor_sum<2>(v[0]));
}

__device__ __forceinline__ double block_sum_d(double v, double *red /* [kWaves] LDS */) {
    v = wave_allsum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[i];
    __syncthreads();
    return t;
}

// h[i] = sum_b P[i][b], i <= j: 32 threads per i (32 i per pass of 1024
// threads); thread k of an i loads partials b = k, k + 32, ... (at most 16,
// all issued before any is added) and the 32 threads combine by shuffles, so
// a pass costs one round of memory latency.  Fixed order: deterministic.
__device__ __forceinline__ void reduce_partials(const c128 *P, int j, int nb, c128 *h /* LDS */) {
    constexpr int TPI = 32, MAXL = kMaxBlocks / TPI;
    const int k = threadIdx.x & (TPI - 1), ii = threadIdx.x / TPI;
    for (int i0 = 0; i0 <= j; i0 += kThreads / TPI) {
        const int i = i0 + ii;
        c128 v[MAXL];
#pragma unroll
        for (int u = 0; u < MAXL; ++u) {
            const int bb = k + TPI * u;
            v[u] = (i <= j && bb < nb) ? P[(long)i * nb + bb] : c128{0, 0};
        }
        c128 t = v[0];
#pragma unroll
        for (int u = 1; u < MAXL; ++u) t = t + v[u];
        t = sum8(xor_sum<8>(xor_sum<16>(t)));   // the 32 lanes of this i (TPI = 32)
        if (k == 0 && i <= j) h[i] = t;
    }
    __syncthreads();
}
// sum of nb partials by the whole block (fixed order: strided per thread,
// then the block reduction); every thread gets the result
__device__ __forceinline__ double reduce_d(const double *P, int nb, double *red) {
    double t = 0;
    for (int b = threadIdx.x; b < nb; b += kThreads) t += P[b];
    return block_sum_d(t, red);
}

// Element n of this block's range for lane l and round e (rounds of 256).
__device__ __forceinline__ long elem(const Eng &E, int e) {
    return (long)blockIdx.x * E.span + (long)e * kLanes + (threadIdx.x & (kLanes - 1));
}
__device__ __forceinline__ int rounds(const Eng &E) { return (int)((E.span + kLanes - 1) / kLanes); }

// partial inner products P[i][block] = sum_{n in range} conj(V_i[n]) w[n],
// i <= j; group g takes i = g, g + 4, ... (16 per pass, one load each).
// wv[e] holds w at this thread's element of round e (0 outside the range).
__device__ __forceinline__ void partial_dots(const Eng &E, int s, int j, const c128 (&wv)[kMaxEPT], long n1, c128 *P,
                                            c128 *red /* [kWaves][kG] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = threadIdx.x >> 8;
    const int nr = rounds(E);
    for (int i0 = 0; i0 <= j; i0 += kGroups * kG) {
        c128 acc[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) acc[q] = c128{0, 0};
#pragma unroll
        for (int e = 0; e < kMaxEPT; ++e) {
            const long n = elem(E, e);
            if (e >= nr || n >= n1) break;
            const c128 wn = wv[e];
#pragma unroll
            for (int q = 0; q < kG; ++q) {
                const int i = i0 + g + kGroups * q;
                if (i <= j) acc[q] = cmac_conj(acc[q], E.vec(s, i)[n], wn);
            }
        }
        const c128 t = wave_tsum16(acc);
        if ((lane & 3) == 0) red[wave * kG + (lane >> 2)] = t;
        __syncthreads();
        if (threadIdx.x < kGroups * kG) {
            const int gg = threadIdx.x / kG, q = threadIdx.x - gg * kG, i = i0 + gg + kGroups * q;
            if (i <= j) {
                const int w0 = gg * (kLanes / 64);
                c128 tt = red[w0 * kG + q];
#pragma unroll
                for (int k = 1; k < kLanes / 64; ++k) tt = tt + red[(w0 + k) * kG + q];
                P[(long)i * E.nb + blockIdx.x] = tt;
            }
        }
        __syncthreads();
    }
}

// sum_i V_i[n] c[i] over i <= j at this thread's element of round e: each
// group adds its basis vectors, the four group partials meet in LDS.  Every
// thread of group 0 returns the total for its element; other groups get 0.
__device__ __forceinline__ c128 basis_combo(const Eng &E, int s, int j, long n, long n1, const c128 *c,
                                           c128 *part /* [kGroups][kLanes] */) {
    const int g = threadIdx.x >> 8, l = threadIdx.x & (kLanes - 1);
    c128 acc = c128{0, 0};
    if (n < n1) {
        int i = g;
        for (; i + kGroups * 3 <= j; i += kGroups * 4) {
            c128 a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = E.vec(s, i + kGroups * q)[n];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc = cmac(acc, a[q], c[i + kGroups * q]);
        }
        for (; i <= j; i += kGroups) acc = cmac(acc, E.vec(s, i)[n], c[i]);
    }
    part[g * kLanes + l] = acc;
    __syncthreads();
    c128 t = c128{0, 0};
    if (g == 0) t = part[l] + part[kLanes + l] + part[2 * kLanes + l] + part[3 * kLanes + l];
    __syncthreads();
    return t;
}

// w -= sum_i V_i h_i over the range; wv[e] receives the new w at this
// thread's elements (all groups, through LDS); returns this thread's share of
// ||w_new||^2 (group 0 only).
// The stored w is the new w times out_scale.
__device__ __forceinline__ double range_update(const Eng &E, int s, int j, c128 *w, long n1, const c128 *h,
                                               c128 (&wv)[kMaxEPT], c128 *part, c128 *wl /* [kLanes] */,
                                               double out_scale) {
    const int g = threadIdx.x >> 8, l = threadIdx.x & (kLanes - 1);
    const int nr = rounds(E);
    double nn = 0;
#pragma unroll
    for (int e = 0; e < kMaxEPT; ++e) {
        wv[e] = c128{0, 0};
        if (e >= nr) continue;
        const long n = elem(E, e);
        const c128 sum = basis_combo(E, s, j, n, n1, h, part);
        if (g == 0 && n < n1) {
            const c128 wn = w[n] - sum;
            w[n] = scale(wn, out_scale);
            wl[l] = wn;
            nn += cabs2(wn);
        }
        __syncthreads();
        wv[e] = (n < n1) ? wl[l] : c128{0, 0};
        __syncthreads();
    }
    return nn;
}

// ---------------------------------------------------------------- commit
// Transition of one column from the previous super-step's state and results.
struct Next {
    SlotState S;
    int restart;        // a new cycle starts: V_0 = r / beta
    double scale;       // 1 / beta
};

// Called by every thread of a block (the residual case reduces cooperatively).
__device__ __forceinline__ Next transition(const Eng &E, int s, const SlotState &P, double *red) {
    Next nx;
    nx.S = P;
    nx.restart = 0;
    nx.scale = 0;
    const SlotConst &C = E.sc[s];
    if (P.phase == PH_INIT) {
        nx.S.phase = PH_RES;
        nx.S.pend = 0;
    } else if (P.phase == PH_ARN) {
        const SlotDec &D = E.dec[s];
        nx.S.iters = P.iters + 1;
        if (D.end) {
            nx.S.phase = PH_RES;
            nx.S.xzero = 0;
            nx.S.pend = E.prec;
        } else {
            nx.S.j = P.j + 1;
        }
    } else if (P.phase == PH_RES) {
        const double *pr = E.PR + (long)s * 2 * E.nb;
        const double rr = reduce_d(pr, E.nb, red), vv = reduce_d(pr + E.nb, E.nb, red);
        const double beta = sqrt(rr), vn = sqrt(vv);
        // a non-finite ||v|| or ||r|| (NaN compares false) decides before rel
        const bool vbad = !(vv <= DBL_MAX), rbad = !(rr <= DBL_MAX);
        const double rel = (vbad || rbad) ? INFINITY : vn > 0 ? beta / vn : (beta > 0 ? INFINITY : 0.0);
        nx.S.vnorm = vn;
        nx.S.relres = rel;
        if (!P.first) nx.S.outer = P.outer + 1;
        nx.S.first = 0;
        if (vbad) {                  // the right-hand side holds NaN or Inf
            nx.S.phase = PH_DONE;
            nx.S.status = TP_E_INVAL;
        } else if (rel <= C.tol) {
            nx.S.phase = PH_DONE;
            nx.S.status = TP_OK;
        } else if (!(rel == rel) || rel == INFINITY) {
            nx.S.phase = PH_DONE;
            nx.S.status = TP_E_BREAKDOWN;
        } else if (P.iters >= C.max_iter || nx.S.outer >= C.max_outer) {
            nx.S.phase = PH_DONE;
            nx.S.status = TP_E_NOCONV;
        } else {
            nx.S.phase = PH_ARN;
            nx.S.j = 0;
            nx.S.pend = 0;
            nx.S.beta = beta;
            const double plain_thr = 0.5 * C.tol * vn;
            nx.S.thr = E.mixed ? fmax(C.inner_tol * beta, plain_thr) : plain_thr;
            nx.restart = 1;
            nx.scale = 1.0 / beta;
        }
    }
    return nx;
}

__global__ void __launch_bounds__(kThreads) k_commit(Eng E, int par) {
    __shared__ double redd[kWaves];
    const int s = blockIdx.y;
    const SlotState P = E.st[(par ^ 1) * E.nslots + s];
    const Next nx = transition(E, s, P, redd);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        E.st[par * E.nslots + s] = nx.S;
        const SlotConst &C = E.sc[s];
        const c128 *in = nullptr, *rin = nullptr, *pin = nullptr, *pbase = nullptr;
        c128 *out = nullptr, *rout = nullptr, *pout = nullptr;
        c128 *Ws = E.W + (long)s * E.Nt;
        if (nx.S.phase == PH_ARN) {
            in = E.vec(s, nx.S.j);
            out = E.vec(s, nx.S.j + 1);
            if (E.prec) {          // w = Z (M^-1 v_j): M^-1 v_j goes through W
                pin = in;
                pout = Ws;
                in = Ws;
            }
        } else if (nx.S.phase == PH_RES && !nx.S.xzero) {
            rin = C.x;
            rout = Ws;
            if (nx.S.pend) {       // x += M^-1 (V y) before the residual
                pin = Ws;
                pout = C.x;
                pbase = C.x;
            }
        }
        if (E.prec) {
            E.pin[s] = pin;
            E.pout[s] = pout;
            E.pbase[s] = pbase;
        }
        if (E.mixed) {
            E.tin[s] = in;
            E.tout[s] = out;
            E.rin[s] = rin;
            E.rout[s] = rout;
        } else {
            E.tin[s] = in ? in : rin;
            E.tout[s] = in ? out : rout;
        }
        if (nx.restart) E.g[(long)s * (E.m + 1)] = c128{nx.S.beta, 0};
    }
    if (nx.restart) {     // every block scales its range of the new V_0
        c128 *v0 = E.vec(s, 0);
        const long n0 = (long)blockIdx.x * E.span, n1 = min(E.Nt, n0 + E.span);
        for (long n = n0 + threadIdx.x; n < n1; n += kThreads) v0[n] = scale(v0[n], nx.scale);
    }
}

// ------------------------------------------------------------------ CGS2
__global__ void __launch_bounds__(kThreads) k_dots(Eng E, int par) {
    __shared__ c128 red[kWaves * kG];
    const int s = blockIdx.y;
    const SlotState S = E.st[par * E.nslots + s];
    if (S.phase != PH_ARN) return;
    const c128 *w = E.vec(s, S.j + 1);
    c128 wv[kMaxEPT];
    const int nr = rounds(E);
#pragma unroll
    for (int e = 0; e < kMaxEPT; ++e) {
        const long n = elem(E, e);
        wv[e] = (e < nr && n < E.Nt) ? w[n] : c128{0, 0};
    }
    partial_dots(E, s, S.j, wv, E.Nt, E.P1 + (long)s * (E.m + 1) * E.nb, red);
}

__global__ void __launch_bounds__(kThreads) k_orth1(Eng E, int par) {
    __shared__ c128 h[kMaxRestart + 1];
    __shared__ c128 red[kWaves * kG];
    __shared__ c128 part[kGroups * kLanes];
    __shared__ c128 wl[kLanes];
    __shared__ double redd[kWaves];
    const int s = blockIdx.y;
    const SlotState S = E.st[par * E.nslots + s];
    if (S.phase != PH_ARN) return;
    const int j = S.j;
    reduce_partials(E.P1 + (long)s * (E.m + 1) * E.nb, j, E.nb, h);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i <= j; i += kThreads) E.h1[(long)s * (E.m + 1) + i] = h[i];
    c128 *w = E.vec(s, j + 1);
    c128 wv[kMaxEPT];
    double nn = range_update(E, s, j, w, E.Nt, h, wv, part, wl, 1.0);
    nn = block_sum_d(nn, redd);
    if (threadIdx.x == 0) E.PN[(long)s * E.nb + blockIdx.x] = nn;
    partial_dots(E, s, j, wv, E.Nt, E.P2 + (long)s * (E.m + 1) * E.nb, red);
}

__global__ void __launch_bounds__(kThreads) k_orth2(Eng E, int par) {
    __shared__ c128 h[kMaxRestart + 1];
    __shared__ c128 part[kGroups * kLanes];
    __shared__ c128 wl[kLanes];
    __shared__ double redd[kWaves];
    const int s = blockIdx.y;
    const SlotState S = E.st[par * E.nslots + s];
    if (S.phase != PH_ARN) return;
    const int j = S.j, m = E.m;
    reduce_partials(E.P2 + (long)s * (m + 1) * E.nb, j, E.nb, h);
    // ||w''||^2 = ||w'||^2 - ||h2||^2 (the second correction is tiny next to w')
    double hh = 0;
    for (int i = 0; i <= j; ++i) hh += cabs2(h[i]);
    const double ww = reduce_d(E.PN + (long)s * E.nb, E.nb, redd);
    const double nrm = sqrt(fmax(ww - hh, 0.0));
    const double sc = nrm > 1e-300 ? 1.0 / nrm : 0.0;
    c128 *w = E.vec(s, j + 1);
    c128 wv[kMaxEPT];
    range_update(E, s, j, w, E.Nt, h, wv, part, wl, sc);
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    // Hessenberg column j: h1 + h2, then the previous rotations and a new one
    const c128 *h1 = E.h1 + (long)s * (m + 1);
    c128 *H = E.H + (long)s * (m + 1) * m, *sn = E.sn + (long)s * m, *g = E.g + (long)s * (m + 1);
    double *cs = E.cs + (long)s * m;
    c128 *Hj = H + (long)j * (m + 1);
    for (int i = 0; i <= j; ++i) Hj[i] = h1[i] + h[i];
    for (int i = 0; i < j; ++i) {
        const c128 a = Hj[i], b = Hj[i + 1];
        Hj[i] = c128{cs[i] * a.x, cs[i] * a.y} + sn[i] * b;
        Hj[i + 1] = c128{cs[i] * b.x, cs[i] * b.y} - conjg(sn[i]) * a;
    }
    const c128 a = Hj[j];
    const double aa = sqrt(cabs2(a));
    double c;
    c128 sv, diag;
    if (aa == 0.0) {
        c = 0.0;
        sv = c128{1, 0};
        diag = c128{nrm, 0};
    } else {
        const double rho = sqrt(aa * aa + nrm * nrm);
        c = aa / rho;
        sv = c128{a.x / aa * nrm / rho, a.y / aa * nrm / rho};
        diag = c128{a.x / aa * rho, a.y / aa * rho};
    }
    cs[j] = c;
    sn[j] = sv;
    Hj[j] = diag;
    const c128 gj = g[j];
    g[j + 1] = c128{0, 0} - conjg(sv) * gj;
    g[j] = c128{c * gj.x, c * gj.y};
    const double est = sqrt(cabs2(g[j + 1]));
    const SlotConst &C = E.sc[s];
    SlotDec D;
    D.est = est;
    D.nrm = nrm;
    D.k = j + 1;
    D.breakdown = !(nrm > 1e-300) || !(est == est);
    D.end = (est <= S.thr) || D.breakdown || (j + 1 >= m) || (S.iters + 1 >= C.max_iter);
    D.pad = 0;
    E.dec[s] = D;
}

// ------------------------------------------------------------------ tail
// Cycle end (x update) for Arnoldi columns whose step decided to stop, and
// the true residual r = v - W for residual columns.
__global__ void __launch_bounds__(kThreads) k_tail(Eng E, int par) {
    __shared__ c128 ys[kMaxRestart];
    __shared__ c128 part[kGroups * kLanes];
    __shared__ double redd[kWaves];
    const int s = blockIdx.y;
    const SlotState S = E.st[par * E.nslots + s];
    const long n0 = (long)blockIdx.x * E.span, n1 = min(E.Nt, n0 + E.span);
    const SlotConst &C = E.sc[s];
    if (S.phase == PH_ARN) {
        const SlotDec &D = E.dec[s];
        if (!D.end) return;
        const int m = E.m, k = D.k;
        const c128 *H = E.H + (long)s * (m + 1) * m, *g = E.g + (long)s * (m + 1);
        // back substitution R y = g, column-oriented
        for (int i = threadIdx.x; i < k; i += kThreads) ys[i] = g[i];
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
            for (int l = threadIdx.x; l < i; l += kThreads) ys[l] = ys[l] - H[(long)i * (m + 1) + l] * yi;
            __syncthreads();
        }
        // x += V y, or with right preconditioning u = V y into W (the next
        // super-step applies x += M^-1 u)
        c128 *x = E.prec ? E.W + (long)s * E.Nt : C.x;
        const int g0 = threadIdx.x >> 8, nr = rounds(E);
#pragma unroll
        for (int e = 0; e < kMaxEPT; ++e) {
            if (e >= nr) break;
            const long n = elem(E, e);
            const c128 sum = basis_combo(E, s, k - 1, n, E.Nt, ys, part);
            if (g0 == 0 && n < E.Nt) x[n] = E.prec ? sum : x[n] + sum;
        }
    } else if (S.phase == PH_RES) {
        const c128 *v = C.v, *Wz = E.W + (long)s * E.Nt;
        c128 *r = E.vec(s, 0);
        double rr = 0, vv = 0;
        for (long n = n0 + threadIdx.x; n < n1; n += kThreads) {
            const c128 vn = v[n];
            const c128 rn = S.xzero ? vn : vn - Wz[n];
            r[n] = rn;
            rr += cabs2(rn);
            vv += cabs2(vn);
        }
        rr = block_sum_d(rr, redd);
        vv = block_sum_d(vv, redd);
        if (threadIdx.x == 0) {
            E.PR[(long)s * 2 * E.nb + blockIdx.x] = rr;
            E.PR[(long)s * 2 * E.nb + E.nb + blockIdx.x] = vv;
        }
    }
}

__global__ void k_zero_cols(c128 *x, long ld, long Nt) {
    const int r = blockIdx.y;
    for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < Nt; n += (long)gridDim.x * blockDim.x)
        x[(long)r * ld + n] = c128{0, 0};
}

// --------------------------------------------------------------- driver
static hipError_t super_step(tp_plan pl, const Eng &E, int par, hipStream_t st) {
    const dim3 gv(E.nb, E.nslots), blk(kThreads);
    hipLaunchKernelGGL(k_commit, gv, blk, 0, st, E, par);
    hipError_t e;
    if (E.prec && E.mixed) {
        const Cols<const c128> pi{nullptr, 0, E.pin}, pb{nullptr, 0, E.pbase};
        const Cols<c128> po{nullptr, 0, E.pout};
        e = precond_op_mixed(pl, pi, po, pb, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout},
                             Cols<const c128>{nullptr, 0, E.rin}, Cols<c128>{nullptr, 0, E.rout}, E.nslots, st);
    } else if (E.prec) {
        const Cols<const c128> pi{nullptr, 0, E.pin}, pb{nullptr, 0, E.pbase};
        const Cols<c128> po{nullptr, 0, E.pout};
        e = precond_fp64(pl, pi, po, pb, E.nslots, st);
        if (e) return e;
        e = matvec_fp64(pl, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout}, E.nslots, st);
    } else if (E.mixed) {
        e = matvec_mixed_both(pl, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout},
                              Cols<const c128>{nullptr, 0, E.rin}, Cols<c128>{nullptr, 0, E.rout}, E.nslots, st);
    } else {
        e = matvec_fp64(pl, Cols<const c128>{nullptr, 0, E.tin}, Cols<c128>{nullptr, 0, E.tout}, E.nslots, st);
    }
    if (e) return e;
    hipLaunchKernelGGL(k_dots, gv, blk, 0, st, E, par);
    hipLaunchKernelGGL(k_orth1, gv, blk, 0, st, E, par);
    hipLaunchKernelGGL(k_orth2, gv, blk, 0, st, E, par);
    hipLaunchKernelGGL(k_tail, gv, blk, 0, st, E, par);
    return hipGetLastError();
}

constexpr int kStepsPerGraph = 2;     // one super-step per state parity

// Host-side record of the continuous-batching engine of a plan.
struct BatchEngine {
    Eng E;
    int active = 0;
    std::vector<SlotConst> cst;      // per-slot constants (host copy)
    hipGraphExec_t gexec = nullptr;
    int pending = 0;
    long nstep = 0;                  // batch_step calls since batch_begin
};

void solver_drop_graphs(tp_plan pl) {
    for (int i = 0; i < pl->ngraphs; ++i) hipGraphExecDestroy(pl->graphs[i].exec);
    pl->ngraphs = 0;
}

void solver_release(tp_plan pl) {
    solver_drop_graphs(pl);
    for (hipEvent_t &e : pl->ev)
        if (e) {
            hipEventDestroy(e);
            e = nullptr;
        }
    if (pl->cs) {
        hipStreamDestroy(pl->cs);
        pl->cs = nullptr;
    }
    if (pl->host_status) {
        hipHostFree(pl->host_status);
        pl->host_status = nullptr;
    }
    if (pl->host_stage) {
        hipHostFree(pl->host_stage);
        pl->host_stage = nullptr;
    }
    delete static_cast<BatchEngine *>(pl->batch);
    pl->batch = nullptr;
}

static hipError_t solver_resources(tp_plan pl) {
    hipError_t e = hipSuccess;
    if (!pl->cs && (e = hipStreamCreateWithFlags(&pl->cs, hipStreamNonBlocking))) return e;
    for (hipEvent_t &ev : pl->ev)
        if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming))) return e;
    // [2][max_rhs] slot states, then [2][max_rhs] Arnoldi decisions
    if (!pl->host_status &&
        (e = hipHostMalloc(&pl->host_status, 2 * (sizeof(SlotState) + sizeof(SlotDec)) * pl->max_rhs)))
        return e;
    return e;
}

// Graph of two super-steps (parities 0 and 1) for this (mode, columns,
// restart); every kernel argument is fixed by the plan, so the graph is
// captured once and replayed by every later solve of the same shape.
static hipError_t step_graph(tp_plan pl, const Eng &E, hipGraphExec_t *out) {
    for (int i = 0; i < pl->ngraphs; ++i) {
        const auto &g = pl->graphs[i];
        if (g.mode == E.mixed && g.nslots == E.nslots && g.m == E.m && g.steps == kStepsPerGraph &&
            g.precond == E.prec) {
            *out = g.exec;
            return hipSuccess;
        }
    }
    hipError_t e;
    if ((e = hipStreamBeginCapture(pl->cs, hipStreamCaptureModeThreadLocal))) return e;
    hipError_t le = hipSuccess;
    for (int t = 0; t < kStepsPerGraph && le == hipSuccess; ++t) le = super_step(pl, E, t & 1, pl->cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->cs, &g);
    if (le) {
        if (g) hipGraphDestroy(g);
        return le;
    }
    if (e) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e) return e;
    if (pl->ngraphs == 8) {
        hipGraphExecDestroy(pl->graphs[0].exec);
        for (int i = 1; i < 8; ++i) pl->graphs[i - 1] = pl->graphs[i];
        pl->ngraphs = 7;
    }
    pl->graphs[pl->ngraphs++] = {E.mixed, E.nslots, E.m, kStepsPerGraph, E.prec, ex};
    *out = ex;
    return hipSuccess;
}

long solver_max_nt() { return (long)kLanes * kMaxEPT * kMaxBlocks; }

// The engine's device regions for `nslots` columns, restart m and a mode.
static Eng engine_make(tp_plan pl, int m, int mixed, int nslots) {
    const long Nt = pl->Nt;
    EngLayout L = eng_layout(Nt, pl->restart, pl->max_rhs);
    char *wsb = pl->solver_ws;
    Eng E;
    E.Nt = Nt;
    E.m = m;        // a shorter restart than the plan's uses a prefix of each region
    {
        const long ept = (Nt + (long)kLanes * kMaxBlocks - 1) / ((long)kLanes * kMaxBlocks);
        E.span = (long)kLanes * ept;
        E.nb = (int)((Nt + E.span - 1) / E.span);
    }
    E.mixed = mixed;
    E.nslots = nslots;
    E.st = (SlotState *)(wsb + L.st);
    E.sc = (SlotConst *)(wsb + L.sc);
    E.dec = (SlotDec *)(wsb + L.dec);
    E.V = (c128 *)(wsb + L.V);
    E.W = (c128 *)(wsb + L.W);
    E.H = (c128 *)(wsb + L.H);
    E.sn = (c128 *)(wsb + L.sn);
    E.g = (c128 *)(wsb + L.g);
    E.h1 = (c128 *)(wsb + L.h1);
    E.y = (c128 *)(wsb + L.y);
    E.P1 = (c128 *)(wsb + L.P1);
    E.P2 = (c128 *)(wsb + L.P2);
    E.cs = (double *)(wsb + L.cs);
    E.PN = (double *)(wsb + L.PN);
    E.PR = (double *)(wsb + L.PR);
    void **tabs = (void **)(wsb + L.tabs);
    E.tin = (const c128 **)tabs;
    E.tout = (c128 **)(tabs + pl->max_rhs);
    E.rin = (const c128 **)(tabs + 2 * pl->max_rhs);
    E.rout = (c128 **)(tabs + 3 * pl->max_rhs);
    E.pin = (const c128 **)(tabs + 4 * pl->max_rhs);
    E.pout = (c128 **)(tabs + 5 * pl->max_rhs);
    E.pbase = (const c128 **)(tabs + 6 * pl->max_rhs);
    E.prec = 0;
    return E;
}

static SlotState initial_state(int x0_given) {
    SlotState S;
    std::memset(&S, 0, sizeof(S));
    S.phase = PH_INIT;
    S.xzero = x0_given ? 0 : 1;
    S.first = 1;
    return S;
}

static void fill_info(const SlotState &S, tp_solve_info *info) {
    info->iters = S.iters;
    info->outer_iters = S.outer;
    info->relres = S.relres;
    info->status = S.phase == PH_DONE ? S.status : TP_E_NOCONV;
}

tp_status solve_run(tp_plan pl, const c128 *v, long ldv, c128 *x, long ldx, int nrhs, const tp_solve_opts &o,
                    tp_solve_info *info, hipStream_t st) {
    const long Nt = pl->Nt;
    if (Nt > solver_max_nt())
        return fail(TP_E_UNSUPPORTED, "solves are limited to Nt <= " + std::to_string(solver_max_nt()));
    if (pl->batch && static_cast<BatchEngine *>(pl->batch)->active)
        return fail(TP_E_INVAL, "a continuous batch is active on this plan");
    Eng E = engine_make(pl, o.restart, o.mode == TP_MIXED, nrhs);
    E.prec = o.precond ? 1 : 0;
    hipError_t e;
    if ((e = solver_resources(pl))) return hip_fail(e, "solver resources");
    hipStream_t cs = pl->cs;
    SlotState *hstat = (SlotState *)pl->host_status;     // [2][max_rhs], pinned
    SlotDec *hdec = reinterpret_cast<SlotDec *>(hstat + 2 * (size_t)pl->max_rhs);

    // the first super-step (parity 0) commits from the parity-1 copy
    std::vector<SlotState> hs(2 * (size_t)nrhs, initial_state(o.x0_given));
    std::vector<SlotConst> hc(nrhs);
    for (int r = 0; r < nrhs; ++r)
        hc[r] = SlotConst{v + (long)r * ldv, x + (long)r * ldx, o.tol, o.inner_tol, o.max_iter, o.max_outer};
    if ((e = hipEventRecord(pl->ev[0], st)) || (e = hipStreamWaitEvent(cs, pl->ev[0], 0)))
        return hip_fail(e, "solver stream ordering");
    if ((e = hipMemcpyAsync(E.st, hs.data(), sizeof(SlotState) * hs.size(), hipMemcpyHostToDevice, cs)) ||
        (e = hipMemcpyAsync(E.sc, hc.data(), sizeof(SlotConst) * hc.size(), hipMemcpyHostToDevice, cs)))
        return hip_fail(e, "solver state upload");
    if (!o.x0_given) hipLaunchKernelGGL(k_zero_cols, dim3(256, nrhs), dim3(256), 0, cs, x, ldx, Nt);
    if ((e = hipGetLastError())) return hip_fail(e, "solver init");
    if ((e = hipStreamSynchronize(cs))) return hip_fail(e, "solver init sync");

    hipGraphExec_t gexec = nullptr;
    if ((e = step_graph(pl, E, &gexec))) return hip_fail(e, "solver graph capture");
    // Without a starting guess the first super-step only turns INIT into the
    // initial residual r = v: its operator and CGS2 launches would all find no
    // column of their phase. Run just its commit and tail, as parity 1, so
    // that the first replayed super-step (parity 0) starts from that residual.
    if (!o.x0_given) {
        const dim3 gv(E.nb, E.nslots), blk(kThreads);
        hipLaunchKernelGGL(k_commit, gv, blk, 0, cs, E, 1);
        hipLaunchKernelGGL(k_tail, gv, blk, 0, cs, E, 1);
        if ((e = hipGetLastError())) return hip_fail(e, "solver initial residual");
    }

    // replay with one graph of lookahead; the state after a graph is the
    // parity-1 copy (the second super-step's commit). When that state is a
    // residual step, or an Arnoldi step that ended its cycle, the graph in
    // flight may finish every column: the host then waits for it before
    // launching another, so no idle graph runs after convergence.
    const long max_launch = ((long)o.max_iter * 2 + (long)o.max_outer * 4 + 16) / kStepsPerGraph + 2;
    const size_t sbytes = sizeof(SlotState) * nrhs, dbytes = sizeof(SlotDec) * nrhs;
    const SlotState *dev_last = E.st + nrhs;
    auto all_done = [&](int b) {
        for (int r = 0; r < nrhs; ++r)
            if (hstat[b * pl->max_rhs + r].phase != PH_DONE) return false;
        return true;
    };
    auto may_finish = [&](int b) {
        for (int r = 0; r < nrhs; ++r) {
            const SlotState &S = hstat[b * pl->max_rhs + r];
            if (S.phase == PH_RES || (S.phase == PH_ARN && hdec[b * pl->max_rhs + r].end)) return true;
        }
        return false;
    };
    long k = 0;
    bool done = false;
    while (!done && k < max_launch) {
        const int buf = (int)(k & 1);
        if ((e = hipGraphLaunch(gexec, cs)) ||
            (e = hipMemcpyAsync(hstat + buf * pl->max_rhs, dev_last, sbytes, hipMemcpyDeviceToHost, cs)) ||
            (e = hipMemcpyAsync(hdec + buf * pl->max_rhs, E.dec, dbytes, hipMemcpyDeviceToHost, cs)) ||
            (e = hipEventRecord(pl->ev[1 + buf], cs)))
            return hip_fail(e, "solver replay");
        if (k > 0) {
            const int pb = 1 - buf;
            if ((e = hipEventSynchronize(pl->ev[1 + pb]))) return hip_fail(e, "solver poll");
            done = all_done(pb);
            if (!done && may_finish(pb)) {
                if ((e = hipEventSynchronize(pl->ev[1 + buf]))) return hip_fail(e, "solver poll");
                done = all_done(buf);
            }
        }
        ++k;
    }
    if ((e = hipStreamSynchronize(cs))) return hip_fail(e, "solver sync");
    const int last = (int)((k - 1) & 1);
    if ((e = hipEventRecord(pl->ev[3], cs)) || (e = hipStreamWaitEvent(st, pl->ev[3], 0)))
        return hip_fail(e, "solver stream ordering");
    tp_status ret = TP_OK;
    for (int r = 0; r < nrhs; ++r) {
        fill_info(hstat[last * pl->max_rhs + r], &info[r]);
        if (info[r].status != TP_OK && ret == TP_OK) ret = (tp_status)info[r].status;
    }
    if (ret == TP_E_NOCONV) set_error("at least one column missed the tolerance");
    if (ret == TP_E_BREAKDOWN) set_error("Krylov breakdown or non-finite residual");
    if (ret == TP_E_INVAL) set_error("a right-hand side holds a non-finite value");
    return ret;
}

// ------------------------------------------------------ continuous batching
// One engine per plan with max_rhs slots; a slot holds one column from
// admission to retirement.  Admission and release are stream-ordered copies
// (from pinned per-slot staging) into the state that the next commit reads,
// so columns join and leave a running batch without stopping it: the host
// never waits for the device except when it polls.

struct SlotStage {
    SlotConst c;
    SlotState admit, idle;
};

tp_status batch_begin(tp_plan pl, const tp_solve_opts &o) {
    if (pl->Nt > solver_max_nt())
        return fail(TP_E_UNSUPPORTED, "solves are limited to Nt <= " + std::to_string(solver_max_nt()));
    hipError_t e;
    if ((e = solver_resources(pl))) return hip_fail(e, "solver resources");
    if (!pl->host_stage && (e = hipHostMalloc(&pl->host_stage, sizeof(SlotStage) * pl->max_rhs)))
        return hip_fail(e, "batch staging");
    BatchEngine *B = static_cast<BatchEngine *>(pl->batch);
    if (!B) {
        B = new BatchEngine();
        pl->batch = B;
    }
    if ((e = hipStreamSynchronize(pl->cs))) return hip_fail(e, "batch begin sync");
    B->E = engine_make(pl, o.restart, o.mode == TP_MIXED, pl->max_rhs);
    B->E.prec = o.precond ? 1 : 0;
    B->cst.assign(pl->max_rhs, SlotConst{nullptr, nullptr, o.tol, o.inner_tol, o.max_iter, o.max_outer});
    B->pending = 0;
    B->nstep = 0;
    SlotState idle;
    std::memset(&idle, 0, sizeof(idle));
    idle.phase = PH_IDLE;
    std::vector<SlotState> hs(2 * (size_t)pl->max_rhs, idle);
    std::vector<void *> ht(7 * (size_t)pl->max_rhs, nullptr);
    if ((e = hipMemcpyAsync(B->E.st, hs.data(), sizeof(SlotState) * hs.size(), hipMemcpyHostToDevice, pl->cs)) ||
        (e = hipMemcpyAsync(B->E.sc, B->cst.data(), sizeof(SlotConst) * B->cst.size(), hipMemcpyHostToDevice,
                            pl->cs)) ||
        (e = hipMemcpyAsync((void *)B->E.tin, ht.data(), sizeof(void *) * ht.size(), hipMemcpyHostToDevice, pl->cs)) ||
        (e = hipStreamSynchronize(pl->cs)))
        return hip_fail(e, "batch state upload");
    if ((e = step_graph(pl, B->E, &B->gexec))) return hip_fail(e, "batch graph capture");
    B->active = 1;
    return TP_OK;
}

static BatchEngine *active_batch(tp_plan pl) {
    BatchEngine *B = static_cast<BatchEngine *>(pl->batch);
    return (B && B->active) ? B : nullptr;
}

// A slot is only re-admitted after the host saw it finish and released it,
// so its staging record is never rewritten while a copy from it is pending.
tp_status batch_admit(tp_plan pl, int slot, const c128 *v, c128 *x, double tol, int x0_given) {
    BatchEngine *B = active_batch(pl);
    if (!B) return fail(TP_E_INVAL, "no active batch on this plan");
    if (slot < 0 || slot >= pl->max_rhs) return fail(TP_E_INVAL, "slot out of range");
    if (!v || !x) return fail(TP_E_INVAL, "v or x is NULL");
    if (!(tol > 0)) return fail(TP_E_INVAL, "tol must be > 0");
    SlotStage *stg = static_cast<SlotStage *>(pl->host_stage) + slot;
    stg->c = B->cst[slot];
    stg->c.v = v;
    stg->c.x = x;
    stg->c.tol = tol;
    stg->admit = initial_state(x0_given);
    hipError_t e;
    // the next graph's first commit reads parity 1
    if ((e = hipMemcpyAsync(B->E.sc + slot, &stg->c, sizeof(SlotConst), hipMemcpyHostToDevice, pl->cs)) ||
        (e = hipMemcpyAsync(B->E.st + B->E.nslots + slot, &stg->admit, sizeof(SlotState), hipMemcpyHostToDevice,
                            pl->cs)))
        return hip_fail(e, "batch admit");
    if (!x0_given) hipLaunchKernelGGL(k_zero_cols, dim3(256, 1), dim3(256), 0, pl->cs, x, pl->Nt, pl->Nt);
    if ((e = hipGetLastError())) return hip_fail(e, "batch admit");
    return TP_OK;
}

tp_status batch_release(tp_plan pl, int slot) {
    BatchEngine *B = active_batch(pl);
    if (!B) return fail(TP_E_INVAL, "no active batch on this plan");
    if (slot < 0 || slot >= pl->max_rhs) return fail(TP_E_INVAL, "slot out of range");
    SlotStage *stg = static_cast<SlotStage *>(pl->host_stage) + slot;
    std::memset(&stg->idle, 0, sizeof(stg->idle));
    stg->idle.phase = PH_IDLE;
    hipError_t e;
    if ((e = hipMemcpyAsync(B->E.st + B->E.nslots + slot, &stg->idle, sizeof(SlotState), hipMemcpyHostToDevice,
                            pl->cs)))
        return hip_fail(e, "batch release");
    return TP_OK;
}

// Enqueue ngraphs graph replays (2 super-steps each) and an asynchronous
// copy of the slot states after them (status buffer nstep & 1).
tp_status batch_step(tp_plan pl, int ngraphs) {
    BatchEngine *B = active_batch(pl);
    if (!B) return fail(TP_E_INVAL, "no active batch on this plan");
    if (ngraphs < 1) return fail(TP_E_INVAL, "ngraphs must be >= 1");
    hipError_t e;
    for (int i = 0; i < ngraphs; ++i)
        if ((e = hipGraphLaunch(B->gexec, pl->cs))) return hip_fail(e, "batch step");
    const int buf = (int)(B->nstep & 1);
    const size_t sbytes = sizeof(SlotState) * pl->max_rhs;
    SlotState *hs = static_cast<SlotState *>(pl->host_status) + (size_t)buf * pl->max_rhs;
    if ((e = hipMemcpyAsync(hs, B->E.st + B->E.nslots, sbytes, hipMemcpyDeviceToHost, pl->cs)) ||
        (e = hipEventRecord(pl->ev[1 + buf], pl->cs)))
        return hip_fail(e, "batch step status");
    B->nstep += 1;
    B->pending = 1;
    return TP_OK;
}

// Slot status after the step `lag` calls before the latest batch_step (lag 0
// or 1): phases[s] = 0 idle, 1 running, 2 finished; info[s].  wait = 0
// returns TP_E_NOCONV (not an error) if that step is still running.
tp_status batch_poll(tp_plan pl, int lag, int wait, int *phases, tp_solve_info *info) {
    BatchEngine *B = active_batch(pl);
    if (!B) return fail(TP_E_INVAL, "no active batch on this plan");
    if (lag < 0 || lag > 1 || B->nstep <= lag) return fail(TP_E_INVAL, "no such step to poll");
    const int buf = (int)((B->nstep - 1 - lag) & 1);
    hipError_t e;
    if (wait) {
        if ((e = hipEventSynchronize(pl->ev[1 + buf]))) return hip_fail(e, "batch poll");
    } else {
        e = hipEventQuery(pl->ev[1 + buf]);
        if (e == hipErrorNotReady) return TP_E_NOCONV;
        if (e) return hip_fail(e, "batch poll");
    }
    const SlotState *hs = static_cast<const SlotState *>(pl->host_status) + (size_t)buf * pl->max_rhs;
    for (int s = 0; s < pl->max_rhs; ++s) {
        const int ph = hs[s].phase;
        if (phases) phases[s] = ph == PH_IDLE ? 0 : ph == PH_DONE ? 2 : 1;
        if (info) fill_info(hs[s], &info[s]);
    }
    return TP_OK;
}

tp_status batch_end(tp_plan pl) {
    BatchEngine *B = static_cast<BatchEngine *>(pl->batch);
    if (pl->cs) {
        hipError_t e = hipStreamSynchronize(pl->cs);
        if (e) return hip_fail(e, "batch end");
    }
    if (B) B->active = 0;
    return TP_OK;
}

hipStream_t solver_stream(tp_plan pl) { return pl->cs; }

bool solver_batch_active(tp_plan pl) { return active_batch(pl) != nullptr; }

}  // namespace tp
