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

// exp(-2 pi i m / 9), m = 1, 2, 4, and cos(pi / 4), to 40 digits
struct Roots9 {
    static constexpr double c1 = 0.7660444431189780352023926505554166739358, s1 = 0.6427876096865393263226434099072634329076;
    static constexpr double c2 = 0.1736481776669303488517166267693147960004, s2 = 0.9848077530122080593667430245895230136706;
    static constexpr double c4 = -0.9396926207859083840541092773247314699362, s4 = 0.3420201433256687330440996146822595807631;
};
constexpr double kSqrtHalf = 0.7071067811865475244008443621048490392848;

template <typename T, int R, bool INV>
__device__ __forceinline__ void small_dft(cpx<T> (&a)[R]);

// a * exp(-+ i t) for the root (c, s) = (cos t, sin t)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot(cpx<T> a, T c, T s) {
    const T sg = INV ? s : -s;   // forward multiplies by c - i s
    return mk<T>(a.x * c - a.y * sg, a.x * sg + a.y * c);
}

// Radix-R DFT of a[0..R) in registers (forward: w = exp(-2 pi i / R)).
// R = 8 is two radix-4 DFTs of the even and odd inputs joined by w^k; R = 9
// is 3 x 3: radix-3 DFTs over n1 (n = 3 n1 + n2), the twiddles
// w9^(n2 k1), radix-3 DFTs over n2, giving y[k1 + 3 k2].
// Odd R pairs inputs q and R - q: with s_q = a_q + a_{R-q}, d_q = a_q - a_{R-q}
// and t = 2 pi q k / R,
//   y_k     = a_0 + sum_q (cos t) s_q - i (sin t) d_q
//   y_{R-k} = a_0 + sum_q (cos t) s_q + i (sin t) d_q
// (signs of the sine terms swap for the inverse).
template <typename T, int R, bool INV>
__device__ __forceinline__ void small_dft(cpx<T> (&a)[R]) {
    if constexpr (R == 8) {
        cpx<T> e[4] = {a[0], a[2], a[4], a[6]}, o[4] = {a[1], a[3], a[5], a[7]};
        small_dft<T, 4, INV>(e);
        small_dft<T, 4, INV>(o);
        const T h = (T)kSqrtHalf;
        const cpx<T> o1 = rot<T, INV>(o[1], h, h), o3 = rot<T, INV>(o[3], -h, h);
        // w^2 = -i (forward) or +i (inverse)
        const cpx<T> o2 = INV ? mk<T>(-o[2].y, o[2].x) : mk<T>(o[2].y, -o[2].x);
        a[0] = e[0] + o[0];
        a[4] = e[0] - o[0];
        a[1] = e[1] + o1;
        a[5] = e[1] - o1;
        a[2] = e[2] + o2;
        a[6] = e[2] - o2;
        a[3] = e[3] + o3;
        a[7] = e[3] - o3;
    } else if constexpr (R == 9) {
        cpx<T> t[3][3];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
            cpx<T> u[3] = {a[n2], a[n2 + 3], a[n2 + 6]};
            small_dft<T, 3, INV>(u);
#pragma unroll
            for (int k1 = 0; k1 < 3; ++k1) t[n2][k1] = u[k1];
        }
        t[1][1] = rot<T, INV>(t[1][1], (T)Roots9::c1, (T)Roots9::s1);
        t[1][2] = rot<T, INV>(t[1][2], (T)Roots9::c2, (T)Roots9::s2);
        t[2][1] = rot<T, INV>(t[2][1], (T)Roots9::c2, (T)Roots9::s2);
        t[2][2] = rot<T, INV>(t[2][2], (T)Roots9::c4, (T)Roots9::s4);
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            cpx<T> u[3] = {t[0][k1], t[1][k1], t[2][k1]};
            small_dft<T, 3, INV>(u);
            a[k1] = u[0];
            a[k1 + 3] = u[1];
            a[k1 + 6] = u[2];
        }
    } else if constexpr (R == 2) {
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

// One radix-R stage over nout transforms (transform o starts at o * so, or at
// ofs[o] * so with a start table; point n of it sits at n * sp), each over the
// CC contiguous channels.  Every butterfly applies its twiddles (w^0 = 1 for
// j = 0), so the data and twiddle reads of an item issue together.
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage_axis(cpx<T> *buf, int lgCC, int P, int L, int sp, int nout, int so,
                                               const cpx<T> *twl, const int *ofs = nullptr) {
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
        cpx<T> *b0 = buf + (ofs ? ofs[o] : o) * so + ch;
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

// Decimation in frequency.  A stage above maps the R slots base + q L of one
// butterfly by M[k2][q] = F_R[k2][q] w^(q j stride); the DFT matrix is
// symmetric, so the transposed stages, applied in reverse order to input in
// natural order, give the same transform with the output in digit-reversed
// order (slot perm[k] holds X[k]).  The transposed stage takes the radix-R
// DFT first and then multiplies output q by w^(q j stride).
//
// fft_stage2 runs one stage (DIT or DIF) over two tiles at once, b1 with a
// channel stride of 2^lg1 and b2 (may be null) with 2^lg2, so that the two
// transforms share the stage's barrier.  Only the first nc1 (nc2) channels of
// a tile are transformed (the rest of its stride is padding).
template <typename T, int R, bool INV, bool DIF, int NT = kBlock>
__device__ __forceinline__ void fft_stage2(cpx<T> *b1, int lg1, int nc1, cpx<T> *b2, int lg2, int nc2, int P, int L,
                                           const cpx<T> *twl) {
    // NI butterflies per thread and round: their LDS reads issue together
    // (indices past the end are clamped; such a duplicate is not stored)
    constexpr int NI = sizeof(T) == 4 ? 2 : 1;
    const int nb = P / R;
    const int stride = P / (L * R);
    const int n1 = nb * nc1, total = n1 + (b2 ? nb * nc2 : 0);
    const float rL = 1.0f / (float)L, rc1 = 1.0f / (float)nc1, rc2 = 1.0f / (float)nc2;
    for (int it0 = threadIdx.x; it0 < total; it0 += NI * NT) {
        cpx<T> a[NI][R], w[NI][R];
        cpx<T> *b0[NI];
        int base[NI], lgv[NI];
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            const int it = min(it0 + ii * NT, total - 1);
            const bool sec = it >= n1;
            const int lg = sec ? lg2 : lg1, i2 = sec ? it - n1 : it;
            int ch;
            const int bf = small_divmod(i2, sec ? nc2 : nc1, sec ? rc2 : rc1, ch);
            int j;
            const int grp = small_divmod(bf, L, rL, j);
            base[ii] = grp * L * R + j;
            lgv[ii] = lg;
            b0[ii] = (sec ? b2 : b1) + ch;
#pragma unroll
            for (int q = 0; q < R; ++q) a[ii][q] = b0[ii][(base[ii] + q * L) << lg];
#pragma unroll
            for (int q = 1; q < R; ++q) w[ii][q] = twid<T, INV>(twl, q * j * stride);
        }
#pragma unroll
        for (int ii = 0; ii < NI; ++ii) {
            if constexpr (DIF) {
                small_dft<T, R, INV>(a[ii]);
#pragma unroll
                for (int q = 1; q < R; ++q) a[ii][q] = a[ii][q] * w[ii][q];
            } else {
#pragma unroll
                for (int q = 1; q < R; ++q) a[ii][q] = a[ii][q] * w[ii][q];
                small_dft<T, R, INV>(a[ii]);
            }
        }
#pragma unroll
        for (int ii = 0; ii < NI; ++ii)
            if (it0 + ii * NT < total)
#pragma unroll
                for (int q = 0; q < R; ++q) b0[ii][(base[ii] + q * L) << lgv[ii]] = a[ii][q];
    }
    __syncthreads();
}

// Two tiles transformed together (b2 may be null; barrier done before) by NT
// threads: nc1 of b1's 2^lg1 channel slots, nc2 of b2's 2^lg2.  DIT: input in
// digit-reversed order, output natural.  DIF: input natural, output
// digit-reversed.
template <typename T, bool INV, bool DIF, int NT = kBlock>
__device__ void lds_fft2(cpx<T> *b1, int lg1, int nc1, cpx<T> *b2, int lg2, int nc2, const FFTDesc &d,
                         const cpx<T> *twl) {
    for (int t = 0; t < d.nst; ++t) {
        const int s = DIF ? d.nst - 1 - t : t;
        switch (d.radix[s]) {
            case 2: fft_stage2<T, 2, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 3: fft_stage2<T, 3, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 4: fft_stage2<T, 4, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 5: fft_stage2<T, 5, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 7: fft_stage2<T, 7, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 8: fft_stage2<T, 8, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            case 9: fft_stage2<T, 9, INV, DIF, NT>(b1, lg1, nc1, b2, lg2, nc2, d.P, d.L[s], twl); break;
            default: break;
        }
    }
}

template <typename T, bool INV>
__device__ void lds_fft(cpx<T> *buf, int lgCC, const FFTDesc &d, const cpx<T> *twl) {
    for (int s = 0; s < d.nst; ++s) {
        switch (d.radix[s]) {
            case 2: fft_stage<T, 2, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 3: fft_stage<T, 3, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 4: fft_stage<T, 4, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 5: fft_stage<T, 5, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 7: fft_stage<T, 7, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 8: fft_stage<T, 8, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            case 9: fft_stage<T, 9, INV>(buf, lgCC, d.P, d.L[s], twl); break;
            default: break;   // the host only builds radices 2, 3, 4, 5, 7, 8, 9
        }
    }
}

// Two-dimensional tiles: nout transforms of length P along one axis of an LDS
// array whose point stride is sp and whose transforms start so apart (both in
// values; with a start table ofs, transform o starts at ofs[o] * so), each
// over the CC = 2^lgCC contiguous channels.  Input in digit-reversed order
// along the axis, output natural.
template <typename T, bool INV>
__device__ void lds_fft_axis(cpx<T> *buf, int lgCC, const FFTDesc &d, int sp, int nout, int so,
                             const cpx<T> *twl, const int *ofs = nullptr) {
    for (int s = 0; s < d.nst; ++s) {
        switch (d.radix[s]) {
            case 2: fft_stage_axis<T, 2, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 3: fft_stage_axis<T, 3, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 4: fft_stage_axis<T, 4, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 5: fft_stage_axis<T, 5, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 7: fft_stage_axis<T, 7, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 8: fft_stage_axis<T, 8, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
            case 9: fft_stage_axis<T, 9, INV>(buf, lgCC, d.P, d.L[s], sp, nout, so, twl, ofs); break;
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
