// C ABI of the library: plan sizing and construction, operator application,
// solve, spectrum export, errors.  Argument checks run before any device work.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tp_internal.h"

namespace tp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
tp_status fail(tp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
tp_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TP_E_HIP;
}

// ------------------------------------------------------------ transform sizes
static bool smooth7(int n) {
    for (int f : {2, 3, 5, 7})
        while (n % f == 0) n /= f;
    return n == 1;
}

int choose_grid(int n) {
    int P = 2 * n - 1;
    while (!smooth7(P)) ++P;
    return P;
}

int fft_factor(int P, int *radix, int *L) {
    int n = P, ns = 0;
    std::vector<int> f;
    // fewest stages: radix 8 and 9 where they divide, then 4, 2, 3, 5, 7
    for (int r : {8, 4, 2, 9, 3, 5, 7})
        while (n % r == 0) { f.push_back(r); n /= r; }
    int len = 1;
    for (int r : f) {
        radix[ns] = r;
        L[ns] = len;
        len *= r;
        ++ns;
    }
    return ns;
}

// Slot of natural input n: the last stage splits n by n mod r into blocks of
// length P / r; recurse on n / r inside the block.
void fft_perm(int P, int nst, const int *radix, int *perm) {
    for (int n = 0; n < P; ++n) {
        int pos = 0, len = P, m = n;
        for (int s = nst - 1; s >= 0; --s) {
            const int r = radix[s];
            len /= r;
            pos += (m % r) * len;
            m /= r;
        }
        perm[n] = pos;
    }
}

#ifndef TP_RIM_SLAB_MAX
#define TP_RIM_SLAB_MAX 256
#endif
int rim_slab_width(long N) {
    // widest slab (64, 128 or 256 columns, at most TP_RIM_SLAB_MAX) that
    // still gives >= 512 workgroups
    if (N >= 512L * 256 && TP_RIM_SLAB_MAX >= 256) return 256;
    if (N >= 512L * 128 && TP_RIM_SLAB_MAX >= 128) return 128;
    return 64;
}

// ------------------------------------------------------------ plan layout
static size_t al(size_t n) { return (n + 255) & ~(size_t)255; }

struct Layout {
    int Px, Py;
    size_t G64, G32, B64, BE64, C64, B32, BE32, C32;   // offsets (SIZE_MAX = absent)
    size_t tab, ws, total;
    size_t spec1, rim1;      // bytes per copy (complex128)
    size_t grid_bytes, rimpart_bytes, ypart_bytes, dual_bytes, solver_bytes, scratch_bytes, ws_bytes;
    int rim_te, rim_nslab;
    int kxh;                 // stored spectrum columns
};

static bool overflow_mul(size_t a, size_t b, size_t *out) {
    if (a && b > SIZE_MAX / a) return true;
    *out = a * b;
    return false;
}

// sym: TP_SYM_RIM (one dense rim block) | TP_SYM_GEN (half the spectrum).
// nrc > 0: a placed rim (the rim functions are nrc extra channels of the
// element cells, no dense rim blocks); 0: dense rim blocks.
static tp_status make_layout(int Nx, int Ny, int b, int Nr, int nrc, int sym, tp_prec prec, int max_rhs,
                             int restart, Layout *L) {
    const bool reciprocal = (sym & TP_SYM_RIM) != 0, half = (sym & TP_SYM_GEN) != 0;
    if (Nx < 1 || Ny < 1 || b < 1 || Nr < 0 || max_rhs < 1 || restart < 1)
        return fail(TP_E_INVAL, "Nx, Ny, b, max_rhs, restart must be >= 1 and Nr >= 0");
    if (prec != TP_FP64 && prec != TP_FP32 && prec != TP_MIXED) return fail(TP_E_INVAL, "unknown precision");
    if (Nx > 256 || Ny > 256) return fail(TP_E_INVAL, "Nx and Ny are limited to 256 (transform length <= 512)");
    if (b > 256) return fail(TP_E_INVAL, "b is limited to 256");
    if (Nr > 2048) return fail(TP_E_INVAL, "Nr is limited to 2048");
    if (nrc < 0 || (nrc > 0 && Nr < 1)) return fail(TP_E_INVAL, "rim channels need nrc >= 0 and, if nrc > 0, Nr >= 1");
    if (b + nrc > 256) return fail(TP_E_INVAL, "b + nrc is limited to 256");
    const int bc = b + nrc;                    // channels per cell
    const bool dense_rim = Nr > 0 && nrc == 0;
    if (restart > 512) return fail(TP_E_INVAL, "restart is limited to 512");
    L->Px = choose_grid(Nx);
    L->Py = choose_grid(Ny);
    if (L->Px > kMaxP || L->Py > kMaxP) return fail(TP_E_INVAL, "transform length exceeds 512");
    const size_t N = (size_t)Nx * Ny * b, Nt = N + Nr, P = (size_t)L->Px * L->Py;
    const size_t bb = (size_t)bc * bc;
    // half spectrum: columns kx <= Px / 2 (Ghat(-k) = Ghat(k)^T)
    L->kxh = half ? L->Px / 2 + 1 : L->Px;
    const size_t nblk = (size_t)L->kxh * L->Py;
    size_t t;
    if (overflow_mul(nblk, bb, &t) || overflow_mul(t, 16, &L->spec1)) return fail(TP_E_INVAL, "size overflow");
    const size_t nrim = reciprocal ? 1 : 2;
    L->rim1 = dense_rim ? (nrim * (size_t)Nr * N + (size_t)Nr * Nr) * 16 : 0;
    const bool f64 = prec != TP_FP32, f32 = prec != TP_FP64;
    size_t off = 0;
    auto take = [&](bool present, size_t bytes) -> size_t {
        if (!present) return SIZE_MAX;
        size_t o = off;
        off += al(bytes);
        return o;
    };
    L->G64 = take(f64, L->spec1);
    L->G32 = take(f32, L->spec1 / 2);
    L->B64 = take(f64 && dense_rim, (size_t)Nr * N * 16);
    L->BE64 = take(f64 && dense_rim && !reciprocal, (size_t)Nr * N * 16);
    L->C64 = take(f64 && dense_rim, (size_t)Nr * Nr * 16);
    L->B32 = take(f32 && dense_rim, (size_t)Nr * N * 8);
    L->BE32 = take(f32 && dense_rim && !reciprocal, (size_t)Nr * N * 8);
    L->C32 = take(f32 && dense_rim, (size_t)Nr * Nr * 8);
    // tables: digit reversals, twiddles (FP64, FP32), the rim channel map
    const size_t tab_bytes = al((size_t)(L->Px + L->Py) * 4) + al((size_t)(L->Px + L->Py) * 16) +
                             al((size_t)(L->Px + L->Py) * 8) + al((size_t)Nx * Ny * nrc * 4);
    L->tab = take(true, tab_bytes);
    // workspace: two transform grids, rim partial sums, Krylov storage
    const size_t gpts = std::max((size_t)Ny * L->Px, P);
    L->grid_bytes = al(gpts * (size_t)bc * max_rhs * 16);
    L->rim_te = rim_slab_width((long)N);
    L->rim_nslab = (int)((N + L->rim_te - 1) / L->rim_te);
    L->rimpart_bytes = dense_rim ? al((size_t)L->rim_nslab * Nr * max_rhs * 16) : al(16);
    // single-column half-spectrum path: mirror parts per row chunk of 8
    L->ypart_bytes = half ? al((size_t)((bc + 7) / 8) * Ny * (L->Px - L->kxh) * bc * 16) : 0;
    // FP32 grids for the mixed solver's shared launches
    L->dual_bytes = (f32 && f64) ? al(gpts * (size_t)bc * max_rhs * 8) : 0;
    L->solver_bytes = al(solver_ws_bytes((long)Nt, restart, max_rhs));
    // plan-time scratch: device copy of the generators + the x-transformed rows
    // (+ a staging copy of one dense rim block)
    L->scratch_bytes = al((size_t)(2 * Ny - 1) * (2 * Nx - 1) * bb * 16) + al((size_t)(2 * Ny - 1) * L->Px * bb * 16) +
                       (dense_rim ? al((size_t)Nr * std::max(N, (size_t)Nr) * 16) : 0);
    L->ws_bytes = std::max(2 * L->grid_bytes + L->rimpart_bytes + L->ypart_bytes + 256 + 2 * L->dual_bytes +
                               L->solver_bytes,
                           L->scratch_bytes);
    L->ws = take(true, L->ws_bytes);
    L->total = off;
    return TP_OK;
}

}  // namespace tp

using namespace tp;

extern "C" {

const char *toeplitz_last_error(void) { return g_err.c_str(); }

tp_status toeplitz_gen_symmetric(int Nx, int Ny, int b, const double *gen, int *symmetric) {
    if (!symmetric) return fail(TP_E_INVAL, "symmetric is NULL");
    *symmetric = 0;
    if (!gen) return fail(TP_E_INVAL, "gen is NULL");
    if (Nx < 1 || Ny < 1 || b < 1 || Nx > 256 || Ny > 256 || b > 256)
        return fail(TP_E_INVAL, "Nx, Ny, b must be in [1, 256]");
    // gen[n][m][p][q] against gen[2Ny-2-n][2Nx-2-m][q][p], bit for bit
    const long W = 2 * Nx - 1, H = 2 * Ny - 1, bb = (long)b * b;
    for (long n = 0; n < H; ++n)
        for (long m = 0; m < W; ++m) {
            const double *a = gen + 2 * ((n * W + m) * bb);
            const double *c = gen + 2 * (((H - 1 - n) * W + (W - 1 - m)) * bb);
            for (int pp = 0; pp < b; ++pp)
                for (int q = 0; q < b; ++q) {
                    const double *u = a + 2 * ((long)pp * b + q), *v = c + 2 * ((long)q * b + pp);
                    if (memcmp(u, v, 2 * sizeof(double)) != 0) return TP_OK;
                }
        }
    *symmetric = 1;
    return TP_OK;
}

tp_status toeplitz_plan_bytes(int Nx, int Ny, int b, int Nr, int sym, tp_prec prec, int max_rhs, int restart,
                              size_t *bytes) {
    if (!bytes) return fail(TP_E_INVAL, "bytes is NULL");
    if (sym & ~(TP_SYM_RIM | TP_SYM_GEN)) return fail(TP_E_INVAL, "sym holds unknown bits");
    Layout L;
    tp_status s = make_layout(Nx, Ny, b, Nr, 0, sym, prec, max_rhs, restart, &L);
    if (s != TP_OK) return s;
    *bytes = L.total;
    return TP_OK;
}

tp_status toeplitz_plan_bytes_placed(int Nx, int Ny, int b, int Nr, int nrc, int sym, tp_prec prec, int max_rhs,
                                     int restart, size_t *bytes) {
    if (!bytes) return fail(TP_E_INVAL, "bytes is NULL");
    if (sym & ~(TP_SYM_RIM | TP_SYM_GEN)) return fail(TP_E_INVAL, "sym holds unknown bits");
    if (nrc < 1) return fail(TP_E_INVAL, "a placed rim needs nrc >= 1");
    Layout L;
    tp_status s = make_layout(Nx, Ny, b, Nr, nrc, sym, prec, max_rhs, restart, &L);
    if (s != TP_OK) return s;
    *bytes = L.total;
    return TP_OK;
}

}  // extern "C"

namespace tp {

static bool all_finite(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// Checks shared by both plan constructors, before any device work: pointers,
// alignment, shapes (make_layout) and finite operator entries (a NaN or Inf
// would only surface as a Krylov breakdown much later).
static tp_status check_create_inputs(int Nx, int Ny, int b, int Nr, int nrc, const double *gen, const double *rim_re,
                                     const double *rim_er, const double *rim_rr, tp_prec prec, int max_rhs,
                                     int restart, void *dev_buf, tp_plan *out) {
    if (!out) return fail(TP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!gen) return fail(TP_E_INVAL, "gen is NULL");
    if (Nr > 0 && (!rim_re || !rim_rr)) return fail(TP_E_INVAL, "rim_re and rim_rr are required when Nr > 0");
    if (!dev_buf) return fail(TP_E_INVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf) & 255) return fail(TP_E_INVAL, "dev_buf must be 256-byte aligned");
    Layout L0;
    tp_status s0 = make_layout(Nx, Ny, b, Nr, nrc, rim_er ? 0 : TP_SYM_RIM, prec, max_rhs, restart, &L0);
    if (s0 != TP_OK) return s0;
    const long N = (long)Nx * Ny * b;
    if (!all_finite(gen, 2 * (size_t)(2 * Ny - 1) * (2 * Nx - 1) * b * b))
        return fail(TP_E_INVAL, "gen holds a non-finite value");
    if (Nr > 0 && (!all_finite(rim_re, 2 * (size_t)Nr * N) || !all_finite(rim_rr, 2 * (size_t)Nr * Nr) ||
                   (rim_er && !all_finite(rim_er, 2 * (size_t)Nr * N))))
        return fail(TP_E_INVAL, "a rim block holds a non-finite value");
    return TP_OK;
}

// The generator of a placed rim: blocks of bc = b + nrc channels per cell,
// gext[n + Ny - 1][m + Nx - 1][p][q] coupling channel p of cell (ix + m, iy + n)
// (row) with channel q of cell (ix, iy).  Element channels (p, q < b) are the
// element generators; a rim channel takes its couplings from the dense rim
// blocks at every pair of cells they connect, and every value one block entry
// receives must be the same bit for bit (else the rim is not block Toeplitz
// in this placement: TP_E_INVAL).  Entries no pair of occupied cells reaches
// stay zero; the restricted operator never reads them.  map[e * nrc + c]: the
// rim function at channel b + c of cell e, or -1.
static tp_status build_placed_gen(int Nx, int Ny, int b, int Nr, int nrc, const double *gen, const double *rim_re,
                                  const double *rim_er, const double *rim_rr, const int *place,
                                  std::vector<c128> &gext, std::vector<int> &map) {
    const int bc = b + nrc, W = 2 * Nx - 1, H = 2 * Ny - 1;
    const long N = (long)Nx * Ny * b;
    const size_t bb = (size_t)bc * bc;
    map.assign((size_t)Nx * Ny * nrc, -1);
    for (int r = 0; r < Nr; ++r) {
        const int cx = place[3 * r], cy = place[3 * r + 1], c = place[3 * r + 2];
        if (cx < 0 || cx >= Nx || cy < 0 || cy >= Ny || c < 0 || c >= nrc)
            return fail(TP_E_INVAL, "rim function " + std::to_string(r) + " is placed outside the cells or channels");
        int &slot = map[((size_t)cy * Nx + cx) * nrc + c];
        if (slot >= 0)
            return fail(TP_E_INVAL, "rim functions " + std::to_string(slot) + " and " + std::to_string(r) +
                                        " share a cell and channel");
        slot = r;
    }
    gext.assign((size_t)H * W * bb, c128{0.0, 0.0});
    std::vector<unsigned char> set((size_t)H * W * bb, 0);
    auto at = [&](int m, int n, int p, int q) {
        return ((size_t)(n + Ny - 1) * W + (m + Nx - 1)) * bb + (size_t)p * bc + q;
    };
    auto put = [&](size_t o, const double *src) {
        if (set[o]) return memcmp(&gext[o], src, sizeof(c128)) == 0;
        memcpy(&gext[o], src, sizeof(c128));
        set[o] = 1;
        return true;
    };
    for (int n = 0; n < H; ++n)
        for (int m = 0; m < W; ++m)
            for (int p = 0; p < b; ++p)
                memcpy(&gext[at(m - (Nx - 1), n - (Ny - 1), p, 0)], gen + 2 * (((size_t)n * W + m) * b * b + (size_t)p * b),
                       (size_t)b * sizeof(c128));
    auto not_toeplitz = [&](const char *block, int r) {
        return fail(TP_E_INVAL, std::string("the rim is not block Toeplitz in this placement: ") + block +
                                    " entries of rim function " + std::to_string(r) +
                                    " differ between cell pairs of equal offset");
    };
    for (int r = 0; r < Nr; ++r) {
        const int cx = place[3 * r], cy = place[3 * r + 1], c = place[3 * r + 2];
        for (int ly = 0; ly < Ny; ++ly)
            for (int lx = 0; lx < Nx; ++lx) {
                const long e0 = ((long)ly * Nx + lx) * b;
                // rim row (channel b + c of cell (cx, cy)), element column
                const size_t o = at(cx - lx, cy - ly, b + c, 0);
                for (int q = 0; q < b; ++q)
                    if (!put(o + q, rim_re + 2 * ((size_t)r * N + e0 + q))) return not_toeplitz("rim-element", r);
                // element row, rim column
                const size_t oe = at(lx - cx, ly - cy, 0, b + c);
                for (int p = 0; p < b; ++p) {
                    const double *src = rim_er ? rim_er + 2 * ((size_t)(e0 + p) * Nr + r) : rim_re + 2 * ((size_t)r * N + e0 + p);
                    if (!put(oe + (size_t)p * bc, src)) return not_toeplitz("element-rim", r);
                }
            }
        for (int t = 0; t < Nr; ++t) {
            const int tx = place[3 * t], ty = place[3 * t + 1], d = place[3 * t + 2];
            if (!put(at(cx - tx, cy - ty, b + c, b + d), rim_rr + 2 * ((size_t)r * Nr + t)))
                return not_toeplitz("rim-rim", r);
        }
    }
    return TP_OK;
}

// Plan construction once the generators are final: gen holds blocks of
// bc = b + nrc channels; the dense rim blocks only when nrc = 0; map_host
// ([Nx Ny][nrc]) only when nrc > 0.
static tp_status create_plan(int Nx, int Ny, int b, int Nr, int nrc, const double *gen, const int *map_host,
                             const double *rim_re, const double *rim_er, const double *rim_rr, int reciprocal,
                             tp_prec prec, int max_rhs, int restart, void *dev_buf, size_t dev_bytes,
                             void *hip_stream, tp_plan *out) {
    const int bc = b + nrc;
    int gsym = 0;
    toeplitz_gen_symmetric(Nx, Ny, bc, gen, &gsym);
    Layout L;
    tp_status s = make_layout(Nx, Ny, b, Nr, nrc, (reciprocal ? TP_SYM_RIM : 0) | (gsym ? TP_SYM_GEN : 0), prec,
                              max_rhs, restart, &L);
    if (s != TP_OK) return s;
    if (dev_bytes < L.total)
        return fail(TP_E_NOMEM, "device buffer holds " + std::to_string(dev_bytes) + " bytes, plan needs " +
                                    std::to_string(L.total));
    hipStream_t st = (hipStream_t)hip_stream;
    tp_plan_s *pl = new (std::nothrow) tp_plan_s();
    if (!pl) return fail(TP_E_NOMEM, "host allocation failed");
    char *base = (char *)dev_buf;
    auto at = [&](size_t off) -> char * { return off == SIZE_MAX ? nullptr : base + off; };
    pl->Nx = Nx; pl->Ny = Ny; pl->b = b; pl->Nr = Nr;
    pl->bc = bc; pl->nrc = nrc; pl->rim_map = nullptr;
    pl->Px = L.Px; pl->Py = L.Py;
    pl->N = (long)Nx * Ny * b; pl->Nt = pl->N + Nr;
    pl->max_rhs = max_rhs; pl->restart = restart; pl->prec = prec; pl->reciprocal = reciprocal;
    pl->half = gsym; pl->kxh = L.kxh;
    pl->base = base; pl->total = L.total;
    pl->G64 = (c128 *)at(L.G64); pl->G32 = (c64 *)at(L.G32);
    pl->B64 = (c128 *)at(L.B64); pl->BE64 = (c128 *)at(L.BE64); pl->C64 = (c128 *)at(L.C64);
    pl->B32 = (c64 *)at(L.B32); pl->BE32 = (c64 *)at(L.BE32); pl->C32 = (c64 *)at(L.C32);
    pl->spectrum_bytes = L.spec1; pl->rim_bytes = L.rim1;
    pl->ws = at(L.ws); pl->ws_bytes = L.ws_bytes; pl->workspace_bytes = L.ws_bytes;
    pl->gridA = pl->ws;
    pl->gridB = pl->ws + L.grid_bytes;
    pl->rim_part = pl->ws + 2 * L.grid_bytes;
    pl->ypart = L.ypart_bytes ? pl->ws + 2 * L.grid_bytes + L.rimpart_bytes : nullptr;
    // the persistent multi-column launch's queue and counters (256 bytes)
    pl->fctr = (int *)(pl->ws + 2 * L.grid_bytes + L.rimpart_bytes + L.ypart_bytes);
    char *dual = pl->ws + 2 * L.grid_bytes + L.rimpart_bytes + L.ypart_bytes + 256;
    pl->gridA32 = L.dual_bytes ? dual : nullptr;
    pl->gridB32 = L.dual_bytes ? dual + L.dual_bytes : nullptr;
    pl->solver_ws = dual + 2 * L.dual_bytes;
    pl->rim_te = L.rim_te; pl->rim_nslab = L.rim_nslab;

    // transform tables
    const int Px = L.Px, Py = L.Py;
    char *tab = at(L.tab);
    int *perm_x = (int *)tab, *perm_y = perm_x + Px;
    c128 *tw64_x = (c128 *)(tab + al((size_t)(Px + Py) * 4)), *tw64_y = tw64_x + Px;
    c64 *tw32_x = (c64 *)(tab + al((size_t)(Px + Py) * 4) + al((size_t)(Px + Py) * 16)), *tw32_y = tw32_x + Px;
    int *map_dev = nrc ? (int *)(tab + al((size_t)(Px + Py) * 4) + al((size_t)(Px + Py) * 16) +
                                 al((size_t)(Px + Py) * 8))
                       : nullptr;
    pl->rim_map = map_dev;
    std::vector<int> hperm(Px + Py);
    std::vector<c128> htw64(Px + Py);
    std::vector<c64> htw32(Px + Py);
    FFTDesc *descs[2] = {&pl->fx, &pl->fy};
    const int Ps[2] = {Px, Py};
    for (int d = 0; d < 2; ++d) {
        FFTDesc &D = *descs[d];
        D.P = Ps[d];
        D.nst = fft_factor(D.P, D.radix, D.L);
        const int o = d ? Px : 0;
        fft_perm(D.P, D.nst, D.radix, hperm.data() + o);
        for (int k = 0; k < D.P; ++k) {
            const long double a = 2.0L * 3.141592653589793238462643383279503L * (long double)k / (long double)D.P;
            htw64[o + k] = {(double)cosl(a), (double)-sinl(a)};
            htw32[o + k] = {(float)htw64[o + k].x, (float)htw64[o + k].y};
        }
        D.perm = d ? perm_y : perm_x;
        D.tw64 = d ? tw64_y : tw64_x;
        D.tw32 = d ? tw32_y : tw32_x;
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(perm_x, hperm.data(), sizeof(int) * (Px + Py), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(tw64_x, htw64.data(), sizeof(c128) * (Px + Py), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(tw32_x, htw32.data(), sizeof(c64) * (Px + Py), hipMemcpyHostToDevice, st)) ||
        (nrc && (e = hipMemcpyAsync(map_dev, map_host, sizeof(int) * (size_t)Nx * Ny * nrc, hipMemcpyHostToDevice,
                                    st)))) {
        delete pl;
        return hip_fail(e, "plan tables upload");
    }
    // spectrum: generators -> scratch, two transform passes -> G64 / G32
    const size_t bb = (size_t)bc * bc;
    const size_t gen_bytes = (size_t)(2 * Ny - 1) * (2 * Nx - 1) * bb * 16;
    c128 *gen_dev = (c128 *)pl->ws;
    c128 *tmp = (c128 *)(pl->ws + al(gen_bytes));
    c128 *rim_tmp = (c128 *)(pl->ws + al(gen_bytes) + al((size_t)(2 * Ny - 1) * Px * bb * 16));
    if ((e = hipMemcpyAsync(gen_dev, gen, gen_bytes, hipMemcpyHostToDevice, st))) {
        delete pl;
        return hip_fail(e, "generator upload");
    }
    if ((e = spectrum_build(pl, gen_dev, tmp, st))) {
        delete pl;
        return hip_fail(e, "spectrum build");
    }
    // rim blocks: complex128 copies and/or complex64 casts
    if (Nr > 0 && nrc == 0) {
        const size_t nN = (size_t)Nr * pl->N, nC = (size_t)Nr * Nr;
        std::vector<c128> ber;
        if (!reciprocal) {      // store B_er transposed, [Nr][N], like B
            ber.resize(nN);
            const c128 *src = (const c128 *)rim_er;
            for (long ei = 0; ei < pl->N; ++ei)
                for (int r = 0; r < Nr; ++r) ber[(size_t)r * pl->N + ei] = src[(size_t)ei * Nr + r];
        }
        struct Item { const void *src; size_t n; c128 *d64; c64 *d32; };
        Item items[3] = {{rim_re, nN, pl->B64, pl->B32},
                         {reciprocal ? nullptr : (const void *)ber.data(), nN, pl->BE64, pl->BE32},
                         {rim_rr, nC, pl->C64, pl->C32}};
        for (const Item &it : items) {
            if (!it.src) continue;
            c128 *stage = it.d64 ? it.d64 : rim_tmp;
            if ((e = hipMemcpyAsync(stage, it.src, it.n * 16, hipMemcpyHostToDevice, st))) {
                delete pl;
                return hip_fail(e, "rim upload");
            }
            if (it.d32 && (e = cast_to_c64(stage, it.d32, (long)it.n, st))) {
                delete pl;
                return hip_fail(e, "rim cast");
            }
            if (!it.d64 && (e = hipStreamSynchronize(st))) {   // rim_tmp is reused by the next item
                delete pl;
                return hip_fail(e, "rim cast sync");
            }
        }
    }
    if ((e = hipStreamSynchronize(st))) {
        delete pl;
        return hip_fail(e, "plan create");
    }
    *out = pl;
    return TP_OK;
}

}  // namespace tp

extern "C" {

tp_status toeplitz_plan_create(int Nx, int Ny, int b, int Nr, const double *gen, const double *rim_re,
                               const double *rim_er, const double *rim_rr, tp_prec prec, int max_rhs, int restart,
                               void *dev_buf, size_t dev_bytes, void *hip_stream, tp_plan *out) {
    tp_status s = check_create_inputs(Nx, Ny, b, Nr, 0, gen, rim_re, rim_er, rim_rr, prec, max_rhs, restart, dev_buf,
                                      out);
    if (s != TP_OK) return s;
    return create_plan(Nx, Ny, b, Nr, 0, gen, nullptr, rim_re, rim_er, rim_rr, rim_er == nullptr, prec, max_rhs,
                       restart, dev_buf, dev_bytes, hip_stream, out);
}

tp_status toeplitz_plan_create_placed(int Nx, int Ny, int b, int Nr, const double *gen, const double *rim_re,
                                      const double *rim_er, const double *rim_rr, const int *rim_place, int nrc,
                                      tp_prec prec, int max_rhs, int restart, void *dev_buf, size_t dev_bytes,
                                      void *hip_stream, tp_plan *out) {
    if (out) *out = nullptr;
    if (Nr < 1 || nrc < 1) return fail(TP_E_INVAL, "a placed rim needs Nr >= 1 and nrc >= 1");
    if (!rim_place) return fail(TP_E_INVAL, "rim_place is NULL");
    tp_status s = check_create_inputs(Nx, Ny, b, Nr, nrc, gen, rim_re, rim_er, rim_rr, prec, max_rhs, restart,
                                      dev_buf, out);
    if (s != TP_OK) return s;
    std::vector<c128> gext;
    std::vector<int> map;
    try {
        s = build_placed_gen(Nx, Ny, b, Nr, nrc, gen, rim_re, rim_er, rim_rr, rim_place, gext, map);
    } catch (const std::bad_alloc &) {
        return fail(TP_E_NOMEM, "host allocation of the placed generators failed");
    }
    if (s != TP_OK) return s;
    return create_plan(Nx, Ny, b, Nr, nrc, reinterpret_cast<const double *>(gext.data()), map.data(), nullptr,
                       nullptr, nullptr, rim_er == nullptr, prec, max_rhs, restart, dev_buf, dev_bytes, hip_stream,
                       out);
}

tp_status toeplitz_plan_set_option(tp_plan p, int option, int value) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    if (p->batch && solver_batch_active(p)) return fail(TP_E_INVAL, "a continuous batch is active on this plan");
    switch (option) {
        case TP_OPT_SPECTRUM_PASS:
            if (value != TP_PASS_AUTO && value != TP_PASS_FUSED && value != TP_PASS_PAIRS)
                return fail(TP_E_INVAL, "unknown spectrum pass");
            solver_drop_graphs(p);     // captured graphs hold the launch shapes
            p->opt_spectrum_pass = value;
            return TP_OK;
        case TP_OPT_MFMA_COLS:
            if (value != 0 && value != 16 && value != 32 && value != 64)
                return fail(TP_E_INVAL, "matrix-core columns must be 0, 16, 32 or 64");
            solver_drop_graphs(p);
            p->opt_mfma_cols = value;
            return TP_OK;
        case TP_OPT_MFMA_MIN_R:
            if (value != 0 && (value < 2 || value > 4096)) return fail(TP_E_INVAL, "threshold must be 0 or 2..4096");
            solver_drop_graphs(p);
            p->opt_mfma_min_r = value;
            return TP_OK;
        case TP_OPT_DUAL_LAUNCH:
            if (value != 0 && value != 1) return fail(TP_E_INVAL, "shared launches must be 0 or 1");
            solver_drop_graphs(p);
            p->opt_dual_launch = value;
            return TP_OK;
        case TP_OPT_RIM_OVERLAP:
            if (value != 0 && value != 1) return fail(TP_E_INVAL, "rim overlap must be 0 or 1");
            solver_drop_graphs(p);
            p->opt_rim_overlap = value;
            return TP_OK;
        case TP_OPT_PROD_LDS: {
            const int cg = (value >> 4) & 15, rt = value & 15;
            if (value != 0 && (value < 0 || value >= 512 || cg < 1 || (rt != 2 && rt != 3 && rt != 6)))
                return fail(TP_E_INVAL,
                            "LDS product: 16 * column tiles (1..15) + row tiles (2, 3 or 6), + 256 for the pair "
                            "form, or 0");
            solver_drop_graphs(p);
            p->opt_prod_lds = value;
            return TP_OK;
        }
        case TP_OPT_MULTI_FUSED:
            if (value != 0 && value != 1) return fail(TP_E_INVAL, "persistent multi-column launch must be 0 or 1");
            solver_drop_graphs(p);
            p->opt_multi_fused = value;
            return TP_OK;
        case TP_OPT_FFT2_LDS:
            if (value != 0 && (value < 16384 || value > 160 * 1024))
                return fail(TP_E_INVAL, "2-D tile LDS must be 0 or 16384..163840 bytes");
            solver_drop_graphs(p);
            p->opt_fft2_lds = value;
            return TP_OK;
        default:
            return fail(TP_E_INVAL, "unknown option");
    }
}

tp_status toeplitz_plan_get_option(tp_plan p, int option, int *value) {
    if (!p || !value) return fail(TP_E_INVAL, "plan or value is NULL");
    switch (option) {
        case TP_OPT_SPECTRUM_PASS: *value = p->opt_spectrum_pass; return TP_OK;
        case TP_OPT_MFMA_COLS: *value = p->opt_mfma_cols; return TP_OK;
        case TP_OPT_MFMA_MIN_R: *value = p->opt_mfma_min_r; return TP_OK;
        case TP_OPT_FFT2_LDS: *value = p->opt_fft2_lds; return TP_OK;
        case TP_OPT_MULTI_FUSED: *value = p->opt_multi_fused; return TP_OK;
        case TP_OPT_PROD_LDS: *value = p->opt_prod_lds; return TP_OK;
        case TP_OPT_RIM_OVERLAP: *value = p->opt_rim_overlap; return TP_OK;
        case TP_OPT_DUAL_LAUNCH: *value = p->opt_dual_launch; return TP_OK;
        default: return fail(TP_E_INVAL, "unknown option");
    }
}

tp_status toeplitz_plan_path(tp_plan p, tp_prec which, int precond, int nrhs, int *flags) {
    if (!p || !flags) return fail(TP_E_INVAL, "plan or flags is NULL");
    if (which != TP_FP64 && which != TP_FP32 && which != TP_MIXED)
        return fail(TP_E_INVAL, "precision must be TP_FP64, TP_FP32 or TP_MIXED");
    if (nrhs < 1 || nrhs > p->max_rhs) return fail(TP_E_INVAL, "nrhs must be in [1, max_rhs]");
    if (precond && !p->has_precond) return fail(TP_E_INVAL, "the plan has no preconditioner");
    if (which != TP_FP64 && !p->G32) return fail(TP_E_UNSUPPORTED, "plan holds no FP32 operator");
    if (which == TP_FP64 && !p->G64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 operator");
    *flags = tp::path_flags(p, which == TP_FP64, precond != 0, nrhs);
    int lg;
    if (which == TP_MIXED && precond && nrhs == 1 && tp::precond_op_joined_ok(p, &lg)) *flags |= TP_PATH_JOINED;
    return TP_OK;
}

tp_status toeplitz_plan_info(tp_plan p, tp_plan_desc *d) {
    if (!p || !d) return fail(TP_E_INVAL, "NULL argument");
    d->Nx = p->Nx; d->Ny = p->Ny; d->b = p->b; d->Nr = p->Nr;
    d->Px = p->Px; d->Py = p->Py; d->N = p->N; d->Nt = p->Nt;
    d->max_rhs = p->max_rhs; d->restart = p->restart; d->prec = p->prec;
    d->spectrum_bytes = p->spectrum_bytes; d->rim_bytes = p->rim_bytes;
    d->workspace_bytes = p->workspace_bytes; d->total_bytes = p->total;
    d->reciprocal = p->reciprocal;
    d->half_spectrum = p->half;
    d->nrc = p->nrc;
    d->bc = p->bc;
    return TP_OK;
}

}  // extern "C"

namespace tp {

// Argument checks shared by the operator and preconditioner applications:
// element size of the vectors (complex128 for TP_FP64 and TP_MIXED, complex64
// for TP_FP32), shapes, overlap, and no continuous batch on the plan (its
// graphs use the same workspace on the plan's own stream).
tp_status check_apply(tp_plan p, tp_prec which, const void *x, long ldx, const void *y, long ldy, int nrhs) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    if (!x || !y) return fail(TP_E_INVAL, "x or y is NULL");
    if (which != TP_FP64 && which != TP_FP32 && which != TP_MIXED)
        return fail(TP_E_INVAL, "precision must be TP_FP64, TP_FP32 or TP_MIXED");
    if (nrhs < 1 || nrhs > p->max_rhs) return fail(TP_E_INVAL, "nrhs must be in [1, max_rhs]");
    if (ldx < p->Nt || ldy < p->Nt) return fail(TP_E_INVAL, "leading dimension smaller than Nt");
    const size_t es = which == TP_FP32 ? 8 : 16;
    const char *xa = (const char *)x, *ya = (const char *)y;
    const size_t xb = ((size_t)ldx * (nrhs - 1) + p->Nt) * es, yb = ((size_t)ldy * (nrhs - 1) + p->Nt) * es;
    if (xa < ya + yb && ya < xa + xb) return fail(TP_E_INVAL, "x and y overlap");
    if (p->batch && solver_batch_active(p)) return fail(TP_E_INVAL, "a continuous batch is active on this plan");
    if (which != TP_FP64 && !p->G32) return fail(TP_E_UNSUPPORTED, "plan holds no FP32 operator");
    if (which == TP_FP64 && !p->G64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 operator");
    return TP_OK;
}

}  // namespace tp

extern "C" {

tp_status toeplitz_matvec(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                          void *hip_stream) {
    tp_status s = check_apply(p, which, x, ldx, y, ldy, nrhs);
    if (s != TP_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    if (which == TP_FP64)
        e = matvec_fp64(p, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                        nrhs, st);
    else if (which == TP_FP32)
        e = matvec_fp32(p, Cols<const c64>{(const c64 *)x, ldx, nullptr}, Cols<c64>{(c64 *)y, ldy, nullptr}, nrhs,
                        st);
    else   // FP32 operator on complex128 vectors: the inner operator of a mixed solve
        e = matvec_fp32_wide(p, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                             nrhs, st);
    if (e != hipSuccess) return hip_fail(e, "matvec launch");
    return TP_OK;
}

tp_status toeplitz_matvec_profile(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                                  int reps, void *hip_stream, double *stage_ms) {
    if (!stage_ms || reps < 1) return fail(TP_E_INVAL, "stage_ms is NULL or reps < 1");
    // same checks as a plain application
    tp_status s = toeplitz_matvec(p, which, x, ldx, y, ldy, nrhs, hip_stream);
    if (s != TP_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t ev[kMatvecStages + 1];
    for (int i = 0; i <= kMatvecStages; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int k = 0; k < i; ++k) hipEventDestroy(ev[k]);
            return fail(TP_E_HIP, "event create");
        }
    for (int i = 0; i < kMatvecStages; ++i) stage_ms[i] = 0.0;
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        if (which == TP_FP64)
            e = matvec_fp64_timed(p, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                                  nrhs, st, ev);
        else if (which == TP_FP32)
            e = matvec_fp32_timed(p, Cols<const c64>{(const c64 *)x, ldx, nullptr}, Cols<c64>{(c64 *)y, ldy, nullptr},
                                  nrhs, st, ev);
        else
            e = matvec_fp32_wide_timed(p, Cols<const c128>{(const c128 *)x, ldx, nullptr},
                                       Cols<c128>{(c128 *)y, ldy, nullptr}, nrhs, st, ev);
        if (e == hipSuccess) e = hipEventSynchronize(ev[kMatvecStages]);
        for (int i = 0; i < kMatvecStages && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            stage_ms[i] += ms / reps;
        }
    }
    for (int i = 0; i <= kMatvecStages; ++i) hipEventDestroy(ev[i]);
    return e == hipSuccess ? TP_OK : hip_fail(e, "matvec profile");
}

tp_status toeplitz_stage_time(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                              int stage, int reps, void *hip_stream, double *ms) {
    if (!ms || reps < 1 || stage < 0 || stage > 5) return fail(TP_E_INVAL, "ms is NULL, reps < 1 or stage not in 0..5");
    // a full application first: it checks the arguments and leaves every
    // stage's input in the workspace
    tp_status s = toeplitz_matvec(p, which, x, ldx, y, ldy, nrhs, hip_stream);
    if (s != TP_OK) return s;
    tp_plan_s q = *p;
    q.only_stage = stage;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(TP_E_HIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(TP_E_HIP, "event create");
    }
    hipError_t e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        if (which == TP_FP64)
            e = matvec_fp64(&q, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                            nrhs, st);
        else if (which == TP_FP32)
            e = matvec_fp32(&q, Cols<const c64>{(const c64 *)x, ldx, nullptr}, Cols<c64>{(c64 *)y, ldy, nullptr},
                            nrhs, st);
        else
            e = matvec_fp32_wide(&q, Cols<const c128>{(const c128 *)x, ldx, nullptr},
                                 Cols<c128>{(c128 *)y, ldy, nullptr}, nrhs, st);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "stage timing");
    *ms = (double)f / reps;
    return TP_OK;
}

tp_status toeplitz_plan_spectrum(tp_plan p, tp_prec which, int kx, int ky, void *host_out) {
    if (!p || !host_out) return fail(TP_E_INVAL, "NULL argument");
    if (kx < 0 || kx >= p->Px || ky < 0 || ky >= p->Py) return fail(TP_E_INVAL, "frequency out of range");
    const size_t bb = (size_t)p->bc * p->bc;
    // a column the plan does not store is the transpose of the block at (-kx, -ky)
    const bool tr = kx >= p->kxh;
    const size_t k = tr ? (size_t)(p->Px - kx) * p->Py + (ky ? p->Py - ky : 0) : (size_t)kx * p->Py + ky;
    hipError_t e;
    size_t es;
    if (which == TP_FP64) {
        if (!p->G64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 operator");
        es = 16;
        e = hipMemcpy(host_out, p->G64 + k * bb, bb * es, hipMemcpyDeviceToHost);
    } else if (which == TP_FP32) {
        if (!p->G32) return fail(TP_E_UNSUPPORTED, "plan holds no FP32 operator");
        es = 8;
        e = hipMemcpy(host_out, p->G32 + k * bb, bb * es, hipMemcpyDeviceToHost);
    } else {
        return fail(TP_E_INVAL, "precision must be TP_FP64 or TP_FP32");
    }
    if (e != hipSuccess) return hip_fail(e, "spectrum copy");
    if (tr) {
        char *o = static_cast<char *>(host_out), tmp[16];
        const int b = p->bc;
        for (int i = 0; i < b; ++i)
            for (int j = i + 1; j < b; ++j) {
                char *a = o + ((size_t)i * b + j) * es, *c = o + ((size_t)j * b + i) * es;
                memcpy(tmp, a, es);
                memcpy(a, c, es);
                memcpy(c, tmp, es);
            }
    }
    return TP_OK;
}

// Preconditioner buffer: the inverted stored spectrum blocks per precision the
// plan holds, 1 / diag(C) per precision when there is a rim, a status word.
static size_t precond_layout(size_t nblk, int b, int Nr, bool f64, bool f32, size_t *s64, size_t *s32, size_t *d64,
                             size_t *d32, size_t *flag) {
    const size_t bb = (size_t)b * b;
    size_t off = 0;
    auto take = [&](bool on, size_t bytes) {
        const size_t o = off;
        if (on) off += al(bytes);
        return on ? o : (size_t)-1;
    };
    *s64 = take(f64, nblk * bb * 16);
    *s32 = take(f32, nblk * bb * 8);
    *d64 = take(f64 && Nr > 0, (size_t)Nr * 16);
    *d32 = take(f32 && Nr > 0, (size_t)Nr * 8);
    *flag = take(true, 256);
    return off;
}
static size_t precond_layout(tp_plan p, size_t *s64, size_t *s32, size_t *d64, size_t *d32, size_t *flag) {
    // a placed rim's channels are inverted with the element channels (no D)
    return precond_layout((size_t)p->kxh * p->Py, p->bc, p->nrc ? 0 : p->Nr, p->G64 != nullptr, p->G32 != nullptr, s64, s32, d64,
                          d32, flag);
}

tp_status toeplitz_precond_bytes(tp_plan p, size_t *bytes) {
    if (!p || !bytes) return fail(TP_E_INVAL, "plan or bytes is NULL");
    size_t a, b, c, d, f;
    *bytes = precond_layout(p, &a, &b, &c, &d, &f);
    return TP_OK;
}

tp_status toeplitz_precond_bytes_for(int Nx, int Ny, int b, int Nr, int sym, tp_prec prec, size_t *bytes) {
    if (!bytes) return fail(TP_E_INVAL, "bytes is NULL");
    if (sym & ~(TP_SYM_RIM | TP_SYM_GEN)) return fail(TP_E_INVAL, "sym holds unknown bits");
    if (prec == TP_FP32) return fail(TP_E_UNSUPPORTED, "the preconditioner is built from the FP64 spectrum");
    Layout L;
    tp_status s = make_layout(Nx, Ny, b, Nr, 0, sym, prec, 1, 1, &L);
    if (s != TP_OK) return s;
    size_t a, c, d, e, f;
    *bytes = precond_layout((size_t)L.kxh * L.Py, b, Nr, true, prec == TP_MIXED, &a, &c, &d, &e, &f);
    return TP_OK;
}

tp_status toeplitz_precond_create(tp_plan p, void *dev_buf, size_t dev_bytes, void *hip_stream) {
    if (!p || !dev_buf) return fail(TP_E_INVAL, "plan or dev_buf is NULL");
    if (!p->G64) return fail(TP_E_UNSUPPORTED, "the preconditioner is built from the FP64 spectrum");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0) return fail(TP_E_INVAL, "dev_buf must be 256-byte aligned");
    if (p->batch && solver_batch_active(p)) return fail(TP_E_INVAL, "a continuous batch is active on this plan");
    size_t o64, o32, od64, od32, of;
    const size_t need = precond_layout(p, &o64, &o32, &od64, &od32, &of);
    if (dev_bytes < need) return fail(TP_E_NOMEM, "dev_buf smaller than toeplitz_precond_bytes()");
    char *base = static_cast<char *>(dev_buf);
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t nS = (size_t)p->kxh * p->Py * p->bc * p->bc;
    // captured solver graphs hold the previous S and D pointers as kernel
    // arguments: drop them before repointing
    solver_drop_graphs(p);
    p->has_precond = 0;
    p->S64 = reinterpret_cast<c128 *>(base + o64);
    p->S32 = o32 != (size_t)-1 ? reinterpret_cast<c64 *>(base + o32) : nullptr;
    p->D64 = od64 != (size_t)-1 ? reinterpret_cast<c128 *>(base + od64) : nullptr;
    p->D32 = od32 != (size_t)-1 ? reinterpret_cast<c64 *>(base + od32) : nullptr;
    int *flag = reinterpret_cast<int *>(base + of);
    hipError_t e;
    if ((e = hipMemsetAsync(flag, 0, sizeof(int), st)) ||
        (e = hipMemcpyAsync(p->S64, p->G64, nS * 16, hipMemcpyDeviceToDevice, st)) ||
        (e = precond_build(p, p->S64, flag, st)))
        return hip_fail(e, "preconditioner build");
    if (p->S32 && (e = cast_to_c64(p->S64, p->S32, (long)nS, st))) return hip_fail(e, "preconditioner cast");
    if (p->D32 && (e = cast_to_c64(p->D64, p->D32, p->Nr, st))) return hip_fail(e, "preconditioner cast");
    int hflag = 0;
    if ((e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st)) || (e = hipStreamSynchronize(st)))
        return hip_fail(e, "preconditioner status");
    if (hflag) return fail(TP_E_BREAKDOWN, "a spectrum block or a diagonal entry of C is singular");
    p->has_precond = 1;
    return TP_OK;
}

tp_status toeplitz_precond_apply(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                                 void *hip_stream) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    if (!p->has_precond) return fail(TP_E_INVAL, "the plan has no preconditioner (toeplitz_precond_create)");
    tp_status s = check_apply(p, which, x, ldx, y, ldy, nrhs);
    if (s != TP_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    if (which == TP_FP64) {
        if (!p->S64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 preconditioner");
        e = precond_fp64(p, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                         Cols<const c128>{nullptr, 0, nullptr}, nrhs, st);
    } else {
        if (!p->S32) return fail(TP_E_UNSUPPORTED, "plan holds no FP32 preconditioner");
        if (which == TP_FP32)
            e = precond_fp32(p, Cols<const c64>{(const c64 *)x, ldx, nullptr}, Cols<c64>{(c64 *)y, ldy, nullptr},
                             Cols<const c64>{nullptr, 0, nullptr}, nrhs, st);
        else
            e = precond_fp32_wide(p, Cols<const c128>{(const c128 *)x, ldx, nullptr},
                                  Cols<c128>{(c128 *)y, ldy, nullptr}, Cols<const c128>{nullptr, 0, nullptr}, nrhs, st);
    }
    if (e != hipSuccess) return hip_fail(e, "preconditioner launch");
    return TP_OK;
}

void toeplitz_solve_opts_default(tp_solve_opts *o) {
    if (!o) return;
    o->tol = 1e-8;
    o->restart = 0;
    o->max_iter = 2000;
    o->max_outer = 50;
    o->mode = TP_FP64;
    o->x0_given = 0;
    o->inner_tol = 1e-4;
    o->precond = 0;
}

tp_status toeplitz_solve(tp_plan p, const void *v, long ldv, void *x, long ldx, int nrhs, const tp_solve_opts *opts,
                         tp_solve_info *info, void *hip_stream) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    if (!v || !x || !info) return fail(TP_E_INVAL, "v, x or info is NULL");
    if (nrhs < 1 || nrhs > p->max_rhs) return fail(TP_E_INVAL, "nrhs must be in [1, max_rhs]");
    if (ldv < p->Nt || ldx < p->Nt) return fail(TP_E_INVAL, "leading dimension smaller than Nt");
    const char *va = (const char *)v, *xa = (const char *)x;
    const size_t vb = ((size_t)ldv * (nrhs - 1) + p->Nt) * 16, xb = ((size_t)ldx * (nrhs - 1) + p->Nt) * 16;
    if (va < xa + xb && xa < va + vb) return fail(TP_E_INVAL, "v and x overlap");
    tp_solve_opts o;
    toeplitz_solve_opts_default(&o);
    if (opts) o = *opts;
    if (o.restart <= 0) o.restart = p->restart;
    if (o.restart > p->restart) return fail(TP_E_INVAL, "restart exceeds the plan's restart");
    if (!(o.tol > 0) || o.max_iter < 1 || o.max_outer < 1) return fail(TP_E_INVAL, "bad tol / max_iter / max_outer");
    if (o.mode == TP_FP64) {
        if (!p->G64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 operator");
    } else if (o.mode == TP_MIXED) {
        if (!p->G64 || !p->G32) return fail(TP_E_UNSUPPORTED, "mixed solves need a TP_MIXED plan");
        if (!(o.inner_tol > 0 && o.inner_tol < 1)) return fail(TP_E_INVAL, "inner_tol must be in (0, 1)");
    } else {
        return fail(TP_E_INVAL, "solve mode must be TP_FP64 or TP_MIXED");
    }
    if (o.precond && !p->has_precond) return fail(TP_E_INVAL, "precond requested but the plan has none");
    return solve_run(p, (const c128 *)v, ldv, (c128 *)x, ldx, nrhs, o, info, (hipStream_t)hip_stream);
}

static tp_status check_batch_opts(tp_plan p, tp_solve_opts &o, const tp_solve_opts *opts) {
    toeplitz_solve_opts_default(&o);
    if (opts) o = *opts;
    if (o.restart <= 0) o.restart = p->restart;
    if (o.restart > p->restart) return fail(TP_E_INVAL, "restart exceeds the plan's restart");
    if (!(o.tol > 0) || o.max_iter < 1 || o.max_outer < 1) return fail(TP_E_INVAL, "bad tol / max_iter / max_outer");
    if (o.mode == TP_FP64) {
        if (!p->G64) return fail(TP_E_UNSUPPORTED, "plan holds no FP64 operator");
    } else if (o.mode == TP_MIXED) {
        if (!p->G64 || !p->G32) return fail(TP_E_UNSUPPORTED, "mixed solves need a TP_MIXED plan");
        if (!(o.inner_tol > 0 && o.inner_tol < 1)) return fail(TP_E_INVAL, "inner_tol must be in (0, 1)");
    } else {
        return fail(TP_E_INVAL, "solve mode must be TP_FP64 or TP_MIXED");
    }
    if (o.precond && !p->has_precond) return fail(TP_E_INVAL, "precond requested but the plan has none");
    return TP_OK;
}

tp_status toeplitz_batch_begin(tp_plan p, const tp_solve_opts *opts) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    tp_solve_opts o;
    tp_status s = check_batch_opts(p, o, opts);
    if (s != TP_OK) return s;
    return batch_begin(p, o);
}

tp_status toeplitz_batch_admit(tp_plan p, int slot, const void *v, void *x, double tol, int x0_given,
                               void *hip_stream) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    hipStream_t cs = solver_stream(p);
    if (!cs) return fail(TP_E_INVAL, "no active batch on this plan");
    hipError_t e;
    // the engine stream waits for the caller's pending writes of v (and x0)
    if ((e = hipEventRecord(p->ev[0], (hipStream_t)hip_stream)) || (e = hipStreamWaitEvent(cs, p->ev[0], 0)))
        return hip_fail(e, "batch admit ordering");
    return batch_admit(p, slot, (const c128 *)v, (c128 *)x, tol, x0_given);
}

tp_status toeplitz_batch_release(tp_plan p, int slot) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    return batch_release(p, slot);
}

tp_status toeplitz_batch_step(tp_plan p, int ngraphs) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    return batch_step(p, ngraphs);
}

tp_status toeplitz_batch_poll(tp_plan p, int lag, int wait, int *phases, tp_solve_info *info) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    return batch_poll(p, lag, wait, phases, info);
}

tp_status toeplitz_batch_end(tp_plan p) {
    if (!p) return fail(TP_E_INVAL, "plan is NULL");
    return batch_end(p);
}

tp_status toeplitz_port_smatrix(int p, long Nt, const void *X, long ldx, const long *port_rows,
                                const double *edge_len, double Z0, void *S, long lds, void *work, size_t work_bytes,
                                void *hip_stream) {
    if (p < 1 || p > 1024) return fail(TP_E_INVAL, "p must be in [1, 1024]");
    if (Nt < 1 || ldx < Nt || lds < p) return fail(TP_E_INVAL, "need Nt >= 1, ldx >= Nt and lds >= p");
    if (!X || !port_rows || !S || !work) return fail(TP_E_INVAL, "X, port_rows, S or work is NULL");
    if ((reinterpret_cast<uintptr_t>(work) & 7) != 0) return fail(TP_E_INVAL, "work must be 8-byte aligned");
    if (work_bytes < smatrix_work_bytes(p)) return fail(TP_E_INVAL, "work buffer too small");
    if (!(Z0 > 0) || !std::isfinite(Z0)) return fail(TP_E_INVAL, "Z0 must be a positive finite number");
    for (int i = 0; i < p; ++i)
        if (port_rows[i] < 0 || port_rows[i] >= Nt) return fail(TP_E_INVAL, "port row outside [0, Nt)");
    if (edge_len)
        for (int i = 0; i < p; ++i)
            if (!(edge_len[i] > 0) || !std::isfinite(edge_len[i])) return fail(TP_E_INVAL, "edge lengths must be > 0");
    return port_smatrix(p, (const c128 *)X, ldx, port_rows, edge_len, Z0, (c128 *)S, lds, work,
                        (hipStream_t)hip_stream);
}

tp_status toeplitz_far_field(int Nx, int Ny, int b, int Nr, double dx, double dy, const double *elem_pos,
                             const double *elem_tan, const double *rim_pos, const double *rim_tan, const void *I,
                             long ldi, int nrhs, const double *dirs, int nang, double k, double eta, void *F,
                             void *hip_stream) {
    if (Nx < 1 || Ny < 1 || b < 1 || Nr < 0 || Nx > 1024 || Ny > 1024 || b > 1024)
        return fail(TP_E_INVAL, "need 1 <= Nx, Ny, b <= 1024 and Nr >= 0");
    if (nrhs < 1 || nrhs > 65535 || nang < 1) return fail(TP_E_INVAL, "nrhs must be in [1, 65535] and nang >= 1");
    const long Nt = (long)Nx * Ny * b + Nr;
    if (ldi < Nt) return fail(TP_E_INVAL, "ldi smaller than Nt");
    if (!elem_pos || !elem_tan || !I || !dirs || !F) return fail(TP_E_INVAL, "a required pointer is NULL");
    if (Nr > 0 && (!rim_pos || !rim_tan)) return fail(TP_E_INVAL, "rim_pos / rim_tan are NULL with Nr > 0");
    if (!std::isfinite(dx) || !std::isfinite(dy) || !std::isfinite(k) || !std::isfinite(eta))
        return fail(TP_E_INVAL, "dx, dy, k and eta must be finite");
    return far_field(Nx, Ny, b, Nr, dx, dy, elem_pos, elem_tan, rim_pos, rim_tan, (const c128 *)I, ldi, nrhs, dirs,
                     nang, k, eta, (c128 *)F, (hipStream_t)hip_stream);
}

void toeplitz_plan_destroy(tp_plan p) {
    if (!p) return;
    solver_release(p);
    delete p;
}

}  // extern "C"
