// Launchers of the matrix-core kernels (bodies in tp_mfma.h).
#include <type_traits>

#include "tp_mfma.h"

namespace tp {

template <typename T, int NT>
static void launch_prod_mfma(const cpx<T> *G, const cpx<T> *in, int b, int R, int Px, int Py, int kxh, cpx<T> *out,
                             const void *const *act, hipStream_t st) {
    const int KP = (b + 7) >> 3;
    const size_t sh = (size_t)16 * NT * (8 * KP + 2) * sizeof(cpx<T>);
    const int waves = (b + 15) / 16;
    const long nitem = (long)Px * Py * ((R + 16 * NT - 1) / (16 * NT));
    dim3 grid((unsigned)(((nitem + 7) / 8) * 8));
    if (b % 2 == 0)
        hipLaunchKernelGGL((k_prod_mfma<T, NT, TP_PROD_KC, true>), grid, dim3(64 * waves), sh, st, G, in, b, R, Px, Py, kxh,
                           out, act);
    else
        hipLaunchKernelGGL((k_prod_mfma<T, NT, TP_PROD_KC, false>), grid, dim3(64 * waves), sh, st, G, in, b, R, Px, Py, kxh,
                           out, act);
}

template <typename T>
hipError_t prod_mfma(const cpx<T> *G, const cpx<T> *in, int b, int R, int Px, int Py, int kxh, cpx<T> *out,
                     const void *const *act, hipStream_t st, int cols) {
    // default tile: 16 columns up to 16 (a 32-column tile would compute as
    // many padded columns as real ones), else 32 for FP32 and 16 for FP64
    if (cols == 0) cols = (sizeof(T) == 4 && R > 16) ? 32 : 16;
    if (cols >= 64 && sizeof(T) == 4)
        launch_prod_mfma<T, 4>(G, in, b, R, Px, Py, kxh, out, act, st);
    else if (cols >= 32)
        launch_prod_mfma<T, 2>(G, in, b, R, Px, Py, kxh, out, act, st);
    else
        launch_prod_mfma<T, 1>(G, in, b, R, Px, Py, kxh, out, act, st);
    return hipGetLastError();
}
template hipError_t prod_mfma<float>(const c64 *, const c64 *, int, int, int, int, int, c64 *, const void *const *,
                                     hipStream_t, int);
template hipError_t prod_mfma<double>(const c128 *, const c128 *, int, int, int, int, int, c128 *,
                                      const void *const *, hipStream_t, int);


size_t prod_lds_bytes(int b) {
    const int KP = (b + 7) >> 3;
    return (size_t)b * (8 * KP + 2) * sizeof(c64);
}

template <int RT, int KPM>
static void launch_prod_lds(const c64 *G, const c64 *in, int b, int R, int Px, int Py, int kxh, c64 *out,
                            const void *const *act, hipStream_t st, int CG, bool pair) {
    const int nrt = (b + 15) >> 4, RG = (nrt + RT - 1) / RT;
    const int ntc = (R + 15) >> 4, ncg = (ntc + CG - 1) / CG;
    const long nitem = (long)(pair ? kxh : Px) * Py * ncg;
    dim3 grid((unsigned)(((nitem + 7) / 8) * 8));
    const dim3 blk(64 * CG * RG);
    const size_t sh = prod_lds_bytes(b);
    if (b % 2 == 0) {
        if (pair)
            hipLaunchKernelGGL((k_prod_lds<float, RT, KPM, true, true>), grid, blk, sh, st, G, in, b, R, Px, Py, kxh,
                               CG, out, act);
        else
            hipLaunchKernelGGL((k_prod_lds<float, RT, KPM, true, false>), grid, blk, sh, st, G, in, b, R, Px, Py,
                               kxh, CG, out, act);
    } else {
        if (pair)
            hipLaunchKernelGGL((k_prod_lds<float, RT, KPM, false, true>), grid, blk, sh, st, G, in, b, R, Px, Py,
                               kxh, CG, out, act);
        else
            hipLaunchKernelGGL((k_prod_lds<float, RT, KPM, false, false>), grid, blk, sh, st, G, in, b, R, Px, Py,
                               kxh, CG, out, act);
    }
}

// FP32 product with the spectrum block in LDS (b <= 128): RT row tiles per
// wave, CG column tiles per workgroup (CG x ceil(ceil(b / 16) / RT) waves);
// pair: one workgroup per stored block of a half spectrum, applied to its
// frequency and to the mirror.
hipError_t prod_lds(const c64 *G, const c64 *in, int b, int R, int Px, int Py, int kxh, c64 *out,
                    const void *const *act, hipStream_t st, int CG, int RT, bool pair) {
    const int KP = (b + 7) >> 3;
    auto go = [&](auto rt) {
        constexpr int RTc = decltype(rt)::value;
        if (KP <= 8) launch_prod_lds<RTc, 8>(G, in, b, R, Px, Py, kxh, out, act, st, CG, pair);
        else if (KP <= 12) launch_prod_lds<RTc, 12>(G, in, b, R, Px, Py, kxh, out, act, st, CG, pair);
        else launch_prod_lds<RTc, 16>(G, in, b, R, Px, Py, kxh, out, act, st, CG, pair);
    };
    if (RT <= 2) go(std::integral_constant<int, 2>());
    else if (RT <= 3) go(std::integral_constant<int, 3>());
    else go(std::integral_constant<int, 6>());
    return hipGetLastError();
}

template <typename T>
size_t rim_mfma_lds(bool nbe) {
    constexpr int NC = 16 * rim_nt<T>(), RCH = rim_rch<T>();
    return ((size_t)NC * 65 + (size_t)NC * (RCH + 1) + (nbe ? 2 : 1) * (size_t)RCH * 65) * sizeof(cpx<T>);
}
template size_t rim_mfma_lds<float>(bool);
template size_t rim_mfma_lds<double>(bool);

template <typename T, typename In, typename Out>
hipError_t rim_mfma(const cpx<T> *B, const cpx<T> *BE, Cols<const In> x, Cols<Out> y, int R, long N, int Nr,
                    int nslab, cpx<T> *part, hipStream_t st) {
    constexpr int NT = rim_nt<T>(), RCH = rim_rch<T>();
    dim3 grid(nslab, (R + 16 * NT - 1) / (16 * NT));
    if (BE) {
        hipLaunchKernelGGL((k_rim_mfma<T, In, Out, NT, RCH, true>), grid, dim3(256), rim_mfma_lds<T>(true), st, B,
                           BE, x, y, R, N, Nr, part);
    } else {
        hipLaunchKernelGGL((k_rim_mfma<T, In, Out, NT, RCH, false>), grid, dim3(256), rim_mfma_lds<T>(false), st,
                           B, B, x, y, R, N, Nr, part);
    }
    return hipGetLastError();
}
template hipError_t rim_mfma<float, c64, c64>(const c64 *, const c64 *, Cols<const c64>, Cols<c64>, int, long, int,
                                              int, c64 *, hipStream_t);
template hipError_t rim_mfma<float, c128, c128>(const c64 *, const c64 *, Cols<const c128>, Cols<c128>, int, long,
                                                int, int, c64 *, hipStream_t);
template hipError_t rim_mfma<double, c128, c128>(const c128 *, const c128 *, Cols<const c128>, Cols<c128>, int,
                                                 long, int, int, c128 *, hipStream_t);

}  // namespace tp
