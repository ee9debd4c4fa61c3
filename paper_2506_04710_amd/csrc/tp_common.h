// Shared types for the gfx950 block-Toeplitz library: complex values, error
// handling and the plan record.  Host and device code include it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/toeplitz.h"

namespace tp {

// Interleaved complex number; 8-byte (float) or 16-byte (double) aligned so
// that one value is one vector load.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    using value_type = T;
    T x, y;
};
using c64 = cpx<float>;
using c128 = cpx<double>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.x, -a.y}; }
// acc + a * b with fused multiply-adds
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmac(cpx<T> acc, cpx<T> a, cpx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmac_conj(cpx<T> acc, cpx<T> a, cpx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <typename T, typename U>
__host__ __device__ __forceinline__ cpx<T> cvt(cpx<U> a) { return {static_cast<T>(a.x), static_cast<T>(a.y)}; }

// Column access for multi-vector operands: either base + r * ld, or a device
// table of column pointers (used by the solver, whose columns live apart).
template <typename V>
struct Cols {
    V *base;
    long ld;
    V *const *tab;
    __device__ __forceinline__ V *col(int r) const { return tab ? tab[r] : base + (long)r * ld; }
};

// Column activity: a NULL entry in a column-pointer table marks an idle column
// (the solver masks columns this way).  Without a table every column is live.
__device__ __forceinline__ bool cols_live(const void *const *tab, int r0, int r1) {
    if (!tab) return true;
    for (int r = r0; r <= r1; ++r)
        if (tab[r]) return true;
    return false;
}

// Load or store through a pointer known to address global memory (device
// buffers), so that the access is a global instruction rather than a flat one
// (a pointer read from a table is otherwise generic).
// (Member-wise: a whole-struct copy through the cast pointer loses the
// address space again.)
template <typename T>
__device__ __forceinline__ cpx<T> ldg(const cpx<T> *p) {
    const __attribute__((address_space(1))) cpx<T> *g = (const __attribute__((address_space(1))) cpx<T> *)p;
    return cpx<T>{g->x, g->y};
}
template <typename T>
__device__ __forceinline__ void stg(cpx<T> *p, cpx<T> v) {
    __attribute__((address_space(1))) cpx<T> *g = (__attribute__((address_space(1))) cpx<T> *)p;
    g->x = v.x;
    g->y = v.y;
}

// v if c, else 0, by masking the bits: the load of v always issues (the
// caller clamps its address), so no branch forms around it.
__device__ __forceinline__ c64 keep(c64 v, bool c) {
    const unsigned m = c ? ~0u : 0u;
    return c64{__uint_as_float(__float_as_uint(v.x) & m), __uint_as_float(__float_as_uint(v.y) & m)};
}
__device__ __forceinline__ c128 keep(c128 v, bool c) {
    const unsigned long long m = c ? ~0ull : 0ull;
    return c128{__longlong_as_double((long long)((unsigned long long)__double_as_longlong(v.x) & m)),
                __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v.y) & m))};
}

// Keep a value in registers at this point: an empty asm statement that reads
// it, so a load producing it completes here and is not moved into the code
// that consumes it.
template <typename T>
__device__ __forceinline__ void pin(const cpx<T> &v) {
    asm volatile("" : : "v"(v.x), "v"(v.y));
}

// ------------------------------------------------------------- lane sums
// Sums with a partner lane inside a wave without the LDS crossbar
// (__shfl_xor compiles to ds_bpermute): DPP quad permutations for lane l ^ 1
// and l ^ 2, the row rotation by 8 for l ^ 8, the half-row mirror l ^ 7 (used
// once the quads agree), and the gfx950 permlane swaps for l ^ 16 and l ^ 32:
// permlane32_swap(a, b) leaves (a_lo, b_lo) in its first result and
// (a_hi, b_hi) in its second (halves of 32 lanes); permlane16_swap does the
// same with the even and odd rows of 16 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) { return __uint_as_float(dpp_u32<CTRL>(__float_as_uint(v))); }
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned long long lo = dpp_u32<CTRL>((unsigned)u), hi = dpp_u32<CTRL>((unsigned)(u >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <int CTRL, typename T>
__device__ __forceinline__ cpx<T> dpp(cpx<T> v) { return cpx<T>{dpp<CTRL>(v.x), dpp<CTRL>(v.y)}; }

template <int B>
__device__ __forceinline__ void lane_swap(unsigned a, unsigned b, unsigned &d, unsigned &s) {
    static_assert(B == 16 || B == 32, "permlane swaps exchange rows (16) or halves (32)");
    if constexpr (B == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        d = r[0];
        s = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        d = r[0];
        s = r[1];
    }
}
// Halving step on lane bit B (16 or 32): lanes with the bit clear return
// lo + the partner's lo, the others hi + the partner's hi.
template <int B>
__device__ __forceinline__ float half_sum(float lo, float hi) {
    unsigned d, s;
    lane_swap<B>(__float_as_uint(lo), __float_as_uint(hi), d, s);
    return __uint_as_float(d) + __uint_as_float(s);
}
template <int B>
__device__ __forceinline__ double half_sum(double lo, double hi) {
    const unsigned long long a = (unsigned long long)__double_as_longlong(lo),
                             b = (unsigned long long)__double_as_longlong(hi);
    unsigned d0, s0, d1, s1;
    lane_swap<B>((unsigned)a, (unsigned)b, d0, s0);
    lane_swap<B>((unsigned)(a >> 32), (unsigned)(b >> 32), d1, s1);
    const double d = __longlong_as_double((long long)(((unsigned long long)d1 << 32) | d0));
    const double s = __longlong_as_double((long long)(((unsigned long long)s1 << 32) | s0));
    return d + s;
}
template <int B, typename T>
__device__ __forceinline__ cpx<T> half_sum(cpx<T> lo, cpx<T> hi) {
    return cpx<T>{half_sum<B>(lo.x, hi.x), half_sum<B>(lo.y, hi.y)};
}
// v + v of lane l ^ M (M = 1, 2, 8, 16, 32)
template <int M, typename V>
__device__ __forceinline__ V xor_sum(V v) {
    static_assert(M == 1 || M == 2 || M == 8 || M == 16 || M == 32, "no single-instruction partner for M");
    if constexpr (M == 1) return v + dpp<kDppXor1>(v);
    else if constexpr (M == 2) return v + dpp<kDppXor2>(v);
    else if constexpr (M == 8) return v + dpp<kDppRor8>(v);
    else return half_sum<M>(v, v);
}
// Sum over the 8 lanes that share lane >> 3 (every one of them gets it).
template <typename V>
__device__ __forceinline__ V sum8(V v) {
    v = xor_sum<1>(v);
    v = xor_sum<2>(v);
    return v + dpp<kDppHalfMirror>(v);
}
// Sum over the whole wave (every lane gets it).
template <typename V>
__device__ __forceinline__ V wave_allsum(V v) {
    v = xor_sum<32>(v);
    v = xor_sum<16>(v);
    v = xor_sum<8>(v);
    return sum8(v);
}

// Threads per workgroup of the transform, product and rim kernels.  Loops use
// this constant rather than blockDim.x: the latter is read from the dispatch
// packet in memory, and a barrier between two uses forces a fresh read.
constexpr int kBlock = 256;

// Loop over i < n with U independent loads in flight per thread: ld(i) (which
// must be safe to call for every i < n) is issued U times, the values are
// pinned, and only then does use(i, v) consume them, so a round costs one
// memory latency instead of U.
template <int U, typename V, typename Ld, typename Use>
__device__ __forceinline__ void batched(int n, Ld ld, Use use, int nt = kBlock) {
    for (int base = threadIdx.x; base < n; base += U * nt) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(min(base + u * nt, n - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) pin(v[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * nt < n) use(base + u * nt, v[u]);
    }
}

// Radix plan of one transform length P (mixed radix, in-place decimation in
// time): stage s combines sub-transforms of length L[s] with radix radix[s].
// perm (device) maps natural input index n to its LDS slot; tw holds
// exp(-2 pi i k / P), k < P.
struct FFTDesc {
    int P;
    int nst;
    int radix[12];
    int L[12];
    const int *perm;
    const c128 *tw64;
    const c64 *tw32;
};

constexpr int kMaxP = 512;

// Placed rim: the rim functions are extra channels of element cells (a margin
// part sits at a cell with a fixed local offset, so every coupling depends only
// on the cell difference and the whole operator is the restriction of one
// two-level block-Toeplitz operator with b + nrc channels per cell).  Channel
// p of cell e is element basis p for p < be, and for p >= be rim function
// idx[e * nrc + p - be] (unknown N + that), or no unknown when that is -1.
// idx == nullptr: every channel is an element basis function.
struct RimMap {
    const int *idx;
    int be, nrc;
    long N;
};
// Index into a column of cell e's channel p, or -1 (unoccupied rim channel).
__device__ __forceinline__ long cell_unknown(const RimMap &m, int e, int p) {
    if (p < m.be) return (long)e * m.be + p;
    const int r = m.idx[(long)e * m.nrc + (p - m.be)];
    return r < 0 ? -1 : m.N + r;
}

// Stored spectrum block of frequency k = kx Py + ky.  With half the spectrum
// stored (columns kx < kxh), a column kx >= kxh is read as the transpose of
// the block at (Px - kx, -ky mod Py).
__device__ __forceinline__ long spec_src(long k, int Px, int Py, int kxh, bool &tr) {
    const int kx = (int)(k / Py), ky = (int)(k - (long)kx * Py);
    tr = kx >= kxh;
    return tr ? (long)(Px - kx) * Py + (ky == 0 ? 0 : Py - ky) : k;
}

}  // namespace tp

// Plan record (host memory; every pointer is into the caller's device buffer).
struct tp_plan_s {
    int Nx, Ny, b, Nr;
    // channels per cell of the transforms and spectrum blocks: b, or b + nrc
    // with a placed rim (rim_map: [Nx Ny][nrc] rim function or -1, device)
    int bc, nrc;
    const int *rim_map;
    int Px, Py;
    long N, Nt;
    int max_rhs, restart;
    tp_prec prec;
    int reciprocal;
    // symmetric generators (Z_{-m,-n} = Z_{m,n}^T): the spectrum holds only
    // the columns kx < kxh = Px / 2 + 1, since Ghat(-k) = Ghat(k)^T; else
    // kxh = Px and every column is stored
    int half, kxh;
    char *base;
    size_t total;
    // operator copies
    tp::c128 *G64;
    tp::c64 *G32;
    tp::c128 *B64, *BE64, *C64;   // B [Nr][N], B_er^T [Nr][N] (non-reciprocal), C [Nr][Nr]
    tp::c64 *B32, *BE32, *C32;
    size_t spectrum_bytes, rim_bytes;
    // block-circulant preconditioner, built on request into a second caller
    // buffer: per-frequency S = G^-1 / (Px Py)^2 and D = 1 / diag(C)
    tp::c128 *S64 = nullptr, *D64 = nullptr;
    tp::c64 *S32 = nullptr, *D32 = nullptr;
    int has_precond = 0;
    // Schur-complement elimination of the rim, built on request into a third
    // caller buffer: F = A^-1 B_er [Nr][N], S^-1 = (C - B F)^-1 [Nr][Nr], and
    // scratch columns for the solves
    tp::c128 *schurF = nullptr, *schurSinv = nullptr, *schurPart = nullptr, *schurY = nullptr;
    double *schurRed = nullptr;
    int *schurFlag = nullptr;
    int has_schur = 0;
    // transform tables
    tp::FFTDesc fx, fy;
    // matvec workspace
    void *gridA, *gridB;          // [max(Ny*Px, Px*Py)][b*max_rhs] complex128-sized each
    // FP32 grids of their own, max_rhs columns (plans with both copies): the
    // mixed solver's FP32 and FP64 operator instances then share each launch
    void *gridA32 = nullptr, *gridB32 = nullptr;
    void *rim_part;               // [nslab][Nr][max_rhs] complex128-sized
    void *ypart;                  // half spectrum, one column: mirror parts [nchunk][Ny][Px - kxh][b]
    char *solver_ws;              // Krylov workspace
    int rim_te;                   // rim columns per slab
    int rim_nslab;
    // solver workspace
    char *ws;
    size_t ws_bytes;
    size_t workspace_bytes;
    // launch options (toeplitz_plan_set_option; the tuner sets them)
    int opt_spectrum_pass = TP_PASS_AUTO;
    int opt_mfma_cols = 0;        // columns per workgroup of the matrix-core product (0 = default)
    int opt_mfma_min_r = 0;       // columns from which the matrix-core kernels run (0 = default)
    int opt_fft2_lds = 0;         // LDS bytes the 2-D transform tiles may take (0 = 48 KB)
    int opt_multi_fused = 0;      // 1: many columns on the 2-D tiles in one persistent launch
    int opt_prod_lds = 0;         // FP32 product with the block in LDS: 16 * column tiles + row tiles (0: off)
    int opt_rim_overlap = 1;      // 1: the dense rim's matrix-core slabs and the forward 2-D tiles in one launch
    int opt_dual_launch = 1;      // 1: the mixed solver's FP32 and FP64 operators share launches where they can
    int *fctr = nullptr;          // task queue and completion counters of that launch (workspace)
    // instrumentation only, on a copy of the record: launch this stage alone
    int only_stage = -1;
    // solver launch resources, created on the first solve and released by
    // toeplitz_plan_destroy: a stream for graph capture and replay (default
    // priority), events ordering it against the caller's stream, pinned host
    // buffers for status polling, and captured super-step graphs.
    hipStream_t cs = nullptr;
    hipEvent_t ev[4] = {};
    void *host_status = nullptr;
    struct GraphEntry {
        int mode, nslots, m, steps, precond;
        hipGraphExec_t exec;
    };
    GraphEntry graphs[8] = {};
    int ngraphs = 0;
    // continuous batching: host record of the engine and pinned staging for
    // slot admission / release copies
    void *batch = nullptr;
    void *host_stage = nullptr;
};
