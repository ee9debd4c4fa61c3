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

// cos and sin of 2 pi m / R for m = 0..R-1 (odd R), to 40 digits
template <int R>
struct Roots;
template <>
struct Roots<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.8660254037844386467637231707529361834714,
                                    -0.8660254037844386467637231707529361834714};
};
template <>
struct Roots<5> {
    static constexpr double c[5] = {1.0, 0.3090169943749474241022934171828190588602,
                                    -0.8090169943749474241022934171828190588602,
                                    -0.8090169943749474241022934171828190588602,
                                    0.3090169943749474241022934171828190588602};
    static constexpr double s[5] = {0.0, 0.9510565162951535721164393333793821434057,
                                    0.5877852522924731291687059546390727685977,
                                    -0.5877852522924731291687059546390727685977,
                                    -0.9510565162951535721164393333793821434057};
};
template <>
struct Roots<7> {
    static constexpr double c[7] = {1.0, 0.6234898018587335305250048840042398106323,
                                    -0.2225209339563144042889025644967947594664,
                                    -0.9009688679024191262361023195074450511659,
                                    -0.9009688679024191262361023195074450511659,
                                    -0.2225209339563144042889025644967947594664,
                                    0.6234898018587335305250048840042398106323};
    static constexpr double s[7] = {0.0, 0.7818314824680298087084445266740577502323,
                                    0.9749279121818236070181316829939312172328,
                                    0.4338837391175581204757683328483587546100,
                                    -0.4338837391175581204757683328483587546100,
                                    -0.9749279121818236070181316829939312172328,
                                    -0.7818314824680298087084445266740577502323};
};

// Radix-R DFT of a[0..R) in registers (forward: w = exp(-2 pi i / R)).
// Odd R pairs inputs q and R - q: with s_q = a_q + a_{R-q}, d_q = a_q - a_{R-q}
// and t = 2 pi q k / R,
//   y_k     = a_0 + sum_q (cos t) s_q - i (sin t) d_q
//   y_{R-k} = a_0 + sum_q (cos t) s_q + i (sin t) d_q
// (signs of the sine terms swap for the inverse).
template <typename T, int R, bool INV>
__device__ __forceinline__ void small_dft(cpx<T> (&a)[R]) {
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
        constexpr int H = (R - 1) / 2;
        cpx<T> sp[H + 1], dm[H + 1];
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            sp[q] = a[q] + a[R - q];
            dm[q] = a[q] - a[R - q];
        }
        cpx<T> y0 = a[0];
#pragma unroll
        for (int q = 1; q <= H; ++q) y0 = y0 + sp[q];
        cpx<T> lo[H + 1], hi[H + 1];
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            cpx<T> re = a[0], im = mk<T>(0, 0);
#pragma unroll
            for (int q = 1; q <= H; ++q) {
                const T c = (T)Roots<R>::c[(q * k) % R], sn = (T)Roots<R>::s[(q * k) % R];
                re.x = fma(c, sp[q].x, re.x);
                re.y = fma(c, sp[q].y, re.y);
                im.x = fma(sn, dm[q].x, im.x);
                im.y = fma(sn, dm[q].y, im.y);
            }
            // -i * im = (im.y, -im.x); +i * im = (-im.y, im.x)
            const cpx<T> mi = mk<T>(im.y, -im.x), pi = mk<T>(-im.y, im.x);
            lo[k] = re + (INV ? pi : mi);
            hi[k] = re + (INV ? mi : pi);
        }
        a[0] = y0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            a[k] = lo[k];
            a[R - k] = hi[k];
        }
    }
}

// Quotient and remainder of n by d for 0 <= n < 2^22, 1 <= d < 2^12, from the
// single-precision reciprocal rd = 1/d: the estimate is off by at most one
// and is corrected with one compare each way.
__device__ __forceinline__ int small_divmod(int n, int d, float rd, int &rem) {
    int q = (int)((float)n * rd);
    int r = n - q * d;
    if (r >= d) {
        ++q;
        r -= d;
    }
    if (r < 0) {
        --q;
        r += d;
    }
    rem = r;
    return q;
}

// One radix-R stage over nout transforms (transform o starts at o * so; point
// n of it sits at n * sp), each over the CC contiguous channels.  Every
// butterfly applies its twiddles (w^0 = 1 for j = 0), so the data and twiddle
// reads of an item issue together.
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage_axis(cpx<T> *buf, int lgCC, int P, int L, int sp, int nout, int so,
                                               const cpx<T> *twl) {
    const int CC = 1 << lgCC;
    const int nb = P / R;
    const int stride = P / (L * R);
    const int total = (nout * nb) << lgCC;
    const float rnb = 1.0f / (float)nb, rL = 1.0f / (float)L;
    for (int it = threadIdx.x; it < total; it += kBlock) {
        const int ch = it & (CC - 1);
        const int rest = it >> lgCC;
        int bf, j;
        const int o = small_divmod(rest, nb, rnb, bf);
        const int grp = small_divmod(bf, L, rL, j);
        const int base = grp * L * R + j;
        cpx<T> *b0 = buf + o * so + ch;
        cpx<T> a[R], w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = b0[(base + q * L) * sp];
#pragma unroll
        for (int q = 1; q < R; ++q) w[q] = twid<T, INV>(twl, q * j * stride);
#pragma unroll
        for (int q = 1; q < R; ++q) a[q] = a[q] * w[q];
        small_dft<T, R, INV>(a);
#pragma unroll
        for (int q = 0; q < R; ++q) b0[(base + q * L) * sp] = a[q];
    }
    __syncthreads();
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(cpx<T> *buf, int lgCC, int P, int L, const cpx<T> *twl) {
    fft_stage_axis<T, R, INV>(buf, lgCC, P, L, 1 << lgCC, 1, 0, twl);
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

// Two-dimensional tiles: nout transforms of length P along one axis of an LDS
// array whose point stride is sp and whose transforms start so apart (both in
// values), each over the CC = 2^lgCC contiguous channels.  Input in
// digit-reversed order along the axis, output natural.
template <typename T, bool INV>
__device__ void lds_fft_axis(cpx<T> *buf, int lgCC, const FFTDesc &d, int sp, int nout, int so,
                             const cpx<T> *twl) {
    for (int s = 0; s < d.nst; ++s) {
        switch (d.radix[s]) {
            case 2: fft_stage_axis<T, 2, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl); break;
            case 3: fft_stage_axis<T, 3, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl); break;
            case 4: fft_stage_axis<T, 4, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl); break;
            case 5: fft_stage_axis<T, 5, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl); break;
            case 7: fft_stage_axis<T, 7, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl); break;
            default: break;
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
    for (int k = threadIdx.x; k < d.P; k += kBlock) twl[k] = tw[k];
}

}  // namespace tp
