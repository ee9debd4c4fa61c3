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

}  // namespace tp

// Plan record (host memory; every pointer is into the caller's device buffer).
struct tp_plan_s {
    int Nx, Ny, b, Nr;
    int Px, Py;
    long N, Nt;
    int max_rhs, restart;
    tp_prec prec;
    int reciprocal;
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
    // transform tables
    tp::FFTDesc fx, fy;
    // matvec workspace
    void *gridA, *gridB;          // [max(Ny*Px, Px*Py)][b*max_rhs] complex128-sized each
    void *rim_part;               // [nslab][Nr][max_rhs] complex128-sized
    int rim_te;                   // rim columns per slab
    int rim_nslab;
    // solver workspace
    char *ws;
    size_t ws_bytes;
    size_t workspace_bytes;
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
