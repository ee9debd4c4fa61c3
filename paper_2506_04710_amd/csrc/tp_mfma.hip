// Launchers of the matrix-core kernels (bodies in tp_mfma.h).
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
        hipLaunchKernelGGL((k_prod_mfma<T, NT, 4, true>), grid, dim3(64 * waves), sh, st, G, in, b, R, Px, Py, kxh,
                           out, act);
    else
        hipLaunchKernelGGL((k_prod_mfma<T, NT, 4, false>), grid, dim3(64 * waves), sh, st, G, in, b, R, Px, Py, kxh,
                           out, act);
}

template <typename T>
hipError_t prod_mfma(const cpx<T> *G, const cpx<T> *in, int b, int R, int Px, int Py, int kxh, cpx<T> *out,
                     const void *const *act, hipStream_t st, int cols) {
    if (cols == 0) cols = sizeof(T) == 4 ? 32 : 16;
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
