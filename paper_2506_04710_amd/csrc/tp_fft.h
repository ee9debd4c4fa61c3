// Batched complex DFTs of small length P staged in LDS.
//
// A workgroup owns a tile buf[P][CC] (point-major, CC channels contiguous) and
// transforms every channel along the point axis.  The transform is an in-place
// mixed-radix decimation-in-time FFT: the input is loaded in digit-reversed
// order (FFTDesc::perm) and each stage combines R sub-transforms of length L
// into one of length L*R:
//   X[j + L*k2] = sum_q w_R^(q*k2) * (w_{L R}^(q*j) * Y_q[j]),  w_M = exp(-+2 pi i / M),
// reading and writing the same R slots, so a stage needs no staging buffer and
// the output comes out in natural order.  Consecutive work items map to
// consecutive channels, so LDS accesses of a wave are contiguous.
#pragma once

#include "tp_common.h"

namespace tp {

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twid(const cpx<T> *twl, int idx) {
    cpx<T> w = twl[idx];
    if (INV) w.y = -w.y;
    return w;
}

// Radix-R DFT of a[0..R) in registers; twl holds exp(-2 pi i k / P), Pr = P / R.
template <typename T, int R, bool INV>
__device__ __forceinline__ void small_dft(cpx<T> (&a)[R], const cpx<T> *twl, int Pr) {
    if constexpr (R == 2) {
        cpx<T> t = a[0] - a[1];
        a[0] = a[0] + a[1];
        a[1] = t;
    } else if constexpr (R == 4) {
        cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2], t2 = a[1] + a[3], t3 = a[1] - a[3];
        // multiply t3 by -i (forward) or +i (inverse)
        cpx<T> u = INV ? mk<T>(-t3.y, t3.x) : mk<T>(t3.y, -t3.x);
        a[0] = t0 + t2;
        a[2] = t0 - t2;
        a[1] = t1 + u;
        a[3] = t1 - u;
    } else {
        cpx<T> y[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            cpx<T> s = a[0];
#pragma unroll
            for (int q = 1; q < R; ++q) s = cmac(s, twid<T, INV>(twl, ((q * k) % R) * Pr), a[q]);
            y[k] = s;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = y[k];
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(cpx<T> *buf, int lgCC, int P, int L, const cpx<T> *twl) {
    const int CC = 1 << lgCC;
    const int nb = P / R;
    const int stride = P / (L * R);
    const int Pr = P / R;
    const int total = nb << lgCC;
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int ch = it & (CC - 1);
        const int bf = it >> lgCC;
        const int j = bf % L;
        const int base = (bf - j) * R + j;      // (bf / L) * L * R + j
        cpx<T> a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = buf[((base + q * L) << lgCC) + ch];
        if (j != 0) {
#pragma unroll
            for (int q = 1; q < R; ++q) a[q] = a[q] * twid<T, INV>(twl, q * j * stride);
        }
        small_dft<T, R, INV>(a, twl, Pr);
#pragma unroll
        for (int q = 0; q < R; ++q) buf[((base + q * L) << lgCC) + ch] = a[q];
    }
    __syncthreads();
}

// Transform all CC = 2^lgCC channels of buf (loaded in perm order, barrier done).
template <typename T, bool INV>
__device__ void lds_fft(cpx<T> *buf, int lgCC, const FFTDesc &d, const cpx<T> *twl) {
    for (int s = 0; s < d.nst; ++s) {
        switch (d.radix[s]) {
            case 2: fft_stage<T, 2, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 3: fft_stage<T, 3, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 4: fft_stage<T, 4, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 5: fft_stage<T, 5, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 7: fft_stage<T, 7, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            default: break;   // the host only builds radices 2, 3, 4, 5, 7
        }
    }
}

template <typename T>
__device__ __forceinline__ const cpx<T> *tw_of(const FFTDesc &d);
template <>
__device__ __forceinline__ const c128 *tw_of<double>(const FFTDesc &d) { return d.tw64; }
template <>
__device__ __forceinline__ const c64 *tw_of<float>(const FFTDesc &d) { return d.tw32; }

// Copy the twiddle table into LDS (caller synchronises).
template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T> *twl, const FFTDesc &d) {
    const cpx<T> *tw = tw_of<T>(d);
    for (int k = threadIdx.x; k < d.P; k += blockDim.x) twl[k] = tw[k];
}

}  // namespace tp
