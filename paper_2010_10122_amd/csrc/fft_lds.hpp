// Mixed-radix FFT of K interleaved columns held in LDS (gfx950).
//
// Stockham autosort formulation: pass s with radix R reads butterfly j from
// j + r*N/R, applies the twiddles exp(dir 2 pi i (j mod Ns) r / (Ns R)),
// does a radix-R DFT and writes to (j div Ns) Ns R + (j mod Ns) + r Ns; after
// all passes the data are in natural order.  There is one LDS buffer: every
// thread first pulls all of its butterfly inputs into registers, the
// workgroup synchronises, then the outputs are written back.  Element n of
// column k lives at buf[n * K + k], so K contiguous global values map to K
// contiguous LDS words.  Twiddles come from a per-length table
// tw[t] = exp(-2 pi i t / N) computed in FP64 on the host.
#pragma once
#include "device_common.hpp"

namespace wg {

constexpr int kFftMaxPass = 16;
constexpr int kFftMaxC = 24;      // complex values a thread holds per pass

struct FftDesc {
    int n;                        // transform length
    int npass;
    int radix[kFftMaxPass];
};

// Small DFTs in registers, sign DIR (-1: exp(-2 pi i jk/R), +1: exp(+...)).
template <int R, int DIR, typename C> struct Dft;

template <int DIR, typename C> struct Dft<2, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int DIR, typename C> struct Dft<3, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(C{}.x);
        const R h = (R)0.8660254037844386;   // sin(2 pi / 3)
        C s = cadd(v[1], v[2]);
        C d = csub(v[1], v[2]);
        C x0 = cadd(v[0], s);
        C t = cmake<C>(v[0].x - (R)0.5 * s.x, v[0].y - (R)0.5 * s.y);
        C u = cscale(cmul_i<DIR>(d), h);
        v[0] = x0;
        v[1] = cadd(t, u);
        v[2] = csub(t, u);
    }
};

template <int DIR, typename C> struct Dft<4, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        C t0 = cadd(v[0], v[2]);
        C t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]);
        C t3 = cmul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

// Odd prime radix: X_k = v0 + sum_{m=1}^{(R-1)/2} [(v_m + v_{R-m}) cos(2 pi k m / R)
//                              + DIR i (v_m - v_{R-m}) sin(2 pi k m / R)]
template <int DIR, typename C> struct Dft<5, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(C{}.x);
        const R c1 = (R)0.30901699437494745, s1 = (R)0.9510565162951535;
        const R c2 = (R)-0.8090169943749475, s2 = (R)0.5877852522924731;
        C a1 = cadd(v[1], v[4]), b1 = cmul_i<DIR>(csub(v[1], v[4]));
        C a2 = cadd(v[2], v[3]), b2 = cmul_i<DIR>(csub(v[2], v[3]));
        C x0 = cadd(v[0], cadd(a1, a2));
        C p1 = cmake<C>(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
        C q1 = cmake<C>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
        C p2 = cmake<C>(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
        C q2 = cmake<C>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
        v[0] = x0;
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

template <int DIR, typename C> struct Dft<7, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(C{}.x);
        const R c1 = (R)0.6234898018587335, s1 = (R)0.7818314824680298;
        const R c2 = (R)-0.2225209339563144, s2 = (R)0.9749279121818236;
        const R c3 = (R)-0.9009688679024191, s3 = (R)0.4338837391175581;
        C a1 = cadd(v[1], v[6]), b1 = cmul_i<DIR>(csub(v[1], v[6]));
        C a2 = cadd(v[2], v[5]), b2 = cmul_i<DIR>(csub(v[2], v[5]));
        C a3 = cadd(v[3], v[4]), b3 = cmul_i<DIR>(csub(v[3], v[4]));
        C x0 = cadd(v[0], cadd(a1, cadd(a2, a3)));
        // k = 1: cos(m), sin(m) for m = 1, 2, 3
        C p1 = cmake<C>(v[0].x + c1 * a1.x + c2 * a2.x + c3 * a3.x,
                        v[0].y + c1 * a1.y + c2 * a2.y + c3 * a3.y);
        C q1 = cmake<C>(s1 * b1.x + s2 * b2.x + s3 * b3.x, s1 * b1.y + s2 * b2.y + s3 * b3.y);
        // k = 2: angles 2, 4 = -3, 6 = -1 (mod 7)
        C p2 = cmake<C>(v[0].x + c2 * a1.x + c3 * a2.x + c1 * a3.x,
                        v[0].y + c2 * a1.y + c3 * a2.y + c1 * a3.y);
        C q2 = cmake<C>(s2 * b1.x - s3 * b2.x - s1 * b3.x, s2 * b1.y - s3 * b2.y - s1 * b3.y);
        // k = 3: angles 3, 6 = -1, 9 = 2 (mod 7)
        C p3 = cmake<C>(v[0].x + c3 * a1.x + c1 * a2.x + c2 * a3.x,
                        v[0].y + c3 * a1.y + c1 * a2.y + c2 * a3.y);
        C q3 = cmake<C>(s3 * b1.x - s1 * b2.x + s2 * b3.x, s3 * b1.y - s1 * b2.y + s2 * b3.y);
        v[0] = x0;
        v[1] = cadd(p1, q1);
        v[6] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[5] = csub(p2, q2);
        v[3] = cadd(p3, q3);
        v[4] = csub(p3, q3);
    }
};

// Radix 8 as two radix-4 DFTs on the even and odd samples plus a twiddled
// radix-2 combination: X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k,
// w = exp(DIR 2 pi i / 8).
template <int DIR, typename C> struct Dft<8, DIR, C> {
    __device__ __forceinline__ static void run(C *v) {
        using R = decltype(C{}.x);
        const R r2 = (R)0.7071067811865476;
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, DIR, C>::run(e);
        Dft<4, DIR, C>::run(o);
        // w^1 = (1 + DIR i)/sqrt2, w^2 = DIR i, w^3 = (-1 + DIR i)/sqrt2
        C o1 = cscale(cadd(o[1], cmul_i<DIR>(o[1])), r2);
        C o2 = cmul_i<DIR>(o[2]);
        C o3 = cscale(csub(cmul_i<DIR>(o[3]), o[3]), r2);
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <int RADIX, int DIR, typename C>
__device__ __forceinline__ void fft_pass(C *buf, int N, int K, int Ns, const C *__restrict__ tw,
                                         int tid, int nth) {
    constexpr int MAXB = (kFftMaxC + RADIX - 1) / RADIX;
    const int M = N / RADIX;
    const int W = M * K;
    const int tstride = N / (Ns * RADIX);
    C v[MAXB][RADIX];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        int w = tid + b * nth;
        if (w < W) {
            int j = w / K, col = w - j * K;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[b][r] = buf[(j + r * M) * K + col];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        int w = tid + b * nth;
        if (w < W) {
            int j = w / K, col = w - j * K;
            int jm = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RADIX; ++r) {
                    C t = tw[jm * r * tstride];
                    v[b][r] = DIR < 0 ? cmul(v[b][r], t) : cmulconj(v[b][r], t);
                }
            }
            Dft<RADIX, DIR, C>::run(v[b]);
            int base = (j - jm) * RADIX + jm;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[(base + r * Ns) * K + col] = v[b][r];
        }
    }
    __syncthreads();
}

// In-place (in LDS) FFT of K interleaved columns of length d.n.  Requires
// d.n * K <= nth * kFftMaxC.  Caller synchronises before (data loaded) and
// may read the result after return (ends with a barrier).
template <int DIR, typename C>
__device__ void lds_fft(C *buf, int K, const FftDesc &d, const C *__restrict__ tw, int tid, int nth) {
    int Ns = 1;
    for (int s = 0; s < d.npass; ++s) {
        const int r = d.radix[s];
        switch (r) {
            case 8: fft_pass<8, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            case 4: fft_pass<4, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            case 2: fft_pass<2, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            case 3: fft_pass<3, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            case 5: fft_pass<5, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            case 7: fft_pass<7, DIR>(buf, d.n, K, Ns, tw, tid, nth); break;
            default: break;
        }
        Ns *= r;
    }
}

}  // namespace wg
