// Mixed-radix FFT of K interleaved columns (gfx950).
//
// Stockham autosort formulation: pass s with radix R reads butterfly j from
// j + r*N/R, applies the twiddles exp(dir 2 pi i (j mod Ns) r / (Ns R)),
// does a radix-R DFT in registers and writes to
// (j div Ns) Ns R + (j mod Ns) + r Ns; after all passes the data are in
// natural order.  Radices go up to 16 (composite ones as two register
// stages with compile-time inner twiddles), so a length of a few thousand
// takes three passes.  The first pass reads its inputs straight from the
// caller (global memory, with any fused pre-processing) and the last pass
// hands its outputs straight to the caller, so only the passes in between
// go through LDS.  There is one LDS buffer: every thread pulls all of its
// butterfly inputs into registers, the workgroup synchronises, then the
// outputs are written back.  Element n of column k lives at
// buf[(n + n/16) * K + k] (one pad element per 16 against bank conflicts of
// the strided writes), so K contiguous global values map to K contiguous LDS
// words.  Inter-pass twiddles come from a per-length table
// tw[t] = exp(-2 pi i t / N) computed in FP64 on the host.
#pragma once
#include <utility>
#include "device_common.hpp"

namespace wg {

constexpr int kFftMaxPass = 16;
constexpr int kFftMaxC = 24;      // complex values a thread holds per pass (N * K <= threads * kFftMaxC)
constexpr int kFftMaxSlots = 32;
  // last-pass outputs per thread: ceil(kFftMaxC / R) * R <= 32 for R <= 16

// LDS words for length n (pad included)
__host__ __device__ constexpr int fft_lds_len(int n) { return n + n / 16; }
__device__ __forceinline__ int fft_lidx(int o) { return o + (o >> 4); }

// ---- compile-time roots of unity ------------------------------------------
// sin and cos of small arguments by their Taylor series; 2 pi m / r is first
// reduced exactly (in integers) to an angle in [0, pi/4] and an octant.
constexpr double ct_sin_small(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos_small(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// cos or sin (want_sin) of 2 pi m / r
constexpr double ct_trig2pi(long m, long r, bool want_sin) {
    m %= r;
    if (m < 0) m += r;
    // angle = 2 pi m / r = (pi/4) * (8 m / r): octant q and remainder f = (8m mod r) / r in [0, 1)
    const long q = (8 * m) / r;
    const long rem = 8 * m - q * r;
    const double pi4 = 0.78539816339744830961566084581988;
    double t = pi4 * (double)rem / (double)r;          // in [0, pi/4)
    // odd octants: use pi/4 - t about the octant boundary
    const bool odd = (q & 1) != 0;
    if (odd) t = pi4 * (double)(r - rem) / (double)r;
    const double s0 = ct_sin_small(t), c0 = ct_cos_small(t);
    // base angle of the octant pair: q / 2 quarter turns; within it, angle = t (even) or pi/2 - t (odd)
    double c = odd ? s0 : c0, s = odd ? c0 : s0;       // cos, sin of the angle within the quarter
    const long quarter = q / 2;
    double cr = c, sr = s;
    if (quarter == 1) { cr = -s; sr = c; }
    else if (quarter == 2) { cr = -c; sr = -s; }
    else if (quarter == 3) { cr = s; sr = -c; }
    return want_sin ? sr : cr;
}

template <int R, int M, int DIR> struct Root {
    static constexpr double re = ct_trig2pi(M, R, false);
    static constexpr double im = DIR * ct_trig2pi(M, R, true);
};

// v * exp(DIR 2 pi i M / R)
template <int R, int M, int DIR, typename C> __device__ __forceinline__ C rot(C v) {
    using T = decltype(C{}.x);
    constexpr int m = M % R;
    if constexpr (m == 0) {
        return v;
    } else if constexpr (4 * m == R) {
        return cmul_i<DIR>(v);
    } else if constexpr (2 * m == R) {
        return cmake<C>(-v.x, -v.y);
    } else if constexpr (4 * m == 3 * R) {
        return cmul_i<-DIR>(v);
    } else {
        constexpr T c = (T)Root<R, M, DIR>::re, s = (T)Root<R, M, DIR>::im;
        return cmake<C>(v.x * c - v.y * s, v.x * s + v.y * c);
    }
}

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


// Composite radix A*B in registers: A-point DFTs over x[B n1 + n2] for each
// n2, inner twiddles exp(DIR 2 pi i n2 k1 / (A B)), then B-point DFTs over
// n2 for each k1; output k1 + A k2.
template <int A, int B, int DIR, typename C> struct DftComp {
    static constexpr int R = A * B;
    template <int... I> __device__ __forceinline__ static void twid(C *y, std::integer_sequence<int, I...>) {
        ((y[I] = rot<R, (I / A) * (I % A), DIR, C>(y[I])), ...);
    }
    __device__ __forceinline__ static void run(C *v) {
        C y[R];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) {
            C t[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
            Dft<A, DIR, C>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) y[n2 * A + k1] = t[k1];
        }
        twid(y, std::make_integer_sequence<int, R>{});
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            C t[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2 * A + k1];
            Dft<B, DIR, C>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = t[k2];
        }
    }
};
template <int DIR, typename C> struct Dft<6, DIR, C> : DftComp<2, 3, DIR, C> {};
template <int DIR, typename C> struct Dft<9, DIR, C> : DftComp<3, 3, DIR, C> {};
template <int DIR, typename C> struct Dft<10, DIR, C> : DftComp<2, 5, DIR, C> {};
template <int DIR, typename C> struct Dft<12, DIR, C> : DftComp<4, 3, DIR, C> {};
template <int DIR, typename C> struct Dft<14, DIR, C> : DftComp<2, 7, DIR, C> {};
template <int DIR, typename C> struct Dft<15, DIR, C> : DftComp<3, 5, DIR, C> {};
template <int DIR, typename C> struct Dft<16, DIR, C> : DftComp<4, 4, DIR, C> {};

// One Stockham pass of radix RADIX over K interleaved columns of length N.
// first: inputs come from load(n, col) instead of LDS; last: outputs go to
// store(o, col, value, slot) instead of LDS, slot = b * RADIX + r being fixed
// for a given (thread, output) so that callers may keep per-output
// registers.  Barriers: a pass that reads and then writes LDS synchronises
// in between; a pass that writes LDS synchronises after.
// Twiddles of a butterfly: w^r, r = 1 .. RADIX-1, with w = tw[jm * tstride].
// Table reads are issued before the LDS reads and the barrier; the compact
// form reads w, w^4 and w^8 only and forms the other powers by at most four
// complex products (a few ulp in FP32; its registers stay few).
template <int RADIX, typename C> struct TwPre {
    C w1, w4, w8;
};
template <int RADIX, typename C>
__device__ __forceinline__ TwPre<RADIX, C> tw_read(const C *__restrict__ tw, int e) {
    TwPre<RADIX, C> t;
    t.w1 = tw[e];
    if constexpr (RADIX > 4) t.w4 = tw[4 * e];
    if constexpr (RADIX > 8) t.w8 = tw[8 * e];
    return t;
}
template <int RADIX, typename C> __device__ __forceinline__ void tw_powers(const TwPre<RADIX, C> &t, C *w) {
    w[1] = t.w1;
    if constexpr (RADIX > 2) w[2] = cmul(t.w1, t.w1);
    if constexpr (RADIX > 3) w[3] = cmul(w[2], t.w1);
    if constexpr (RADIX > 4) {
        w[4] = t.w4;
#pragma unroll
        for (int r = 5; r < RADIX && r < 8; ++r) w[r] = cmul(t.w4, w[r - 4]);
    }
    if constexpr (RADIX > 8) {
        w[8] = t.w8;
#pragma unroll
        for (int r = 9; r < RADIX; ++r) w[r] = cmul(t.w8, w[r - 8]);
    }
}

// CAP: values per thread the caller guarantees (N * K <= NTH * CAP); 0 for
// the default, N * K <= 12288 for the widest workgroups, else
// <= NTH * kFftMaxC.  A smaller CAP keeps fewer registers per pass.
template <int NTH, int CAP> constexpr int fft_cap() { return CAP > 0 ? CAP : (NTH >= 512 ? 12288 / NTH : kFftMaxC); }

// Butterfly indices without integer division: the column count K is a
// power of two (a shift and a mask), and j mod Ns comes from the FP32
// reciprocal of Ns.  For j < 2^20, (j + 1/2) / Ns lies at least 1/(2 Ns) from
// an integer, and the rounding of 1/Ns and of the product (together below
// 1.5 2^-23 relative) moves it by less than 2^20 / Ns * 1.5 2^-23 < 1/(4 Ns),
// so the truncated quotient is exact.
struct FftIdx {
    int kshift, kmask, ns;
    float rns;
    __device__ __forceinline__ FftIdx(int K, int Ns)
        : kshift(__builtin_ctz((unsigned)K)), kmask(K - 1), ns(Ns), rns(1.0f / (float)Ns) {}
    __device__ __forceinline__ int row(int w) const { return w >> kshift; }
    __device__ __forceinline__ int col(int w) const { return w & kmask; }
    __device__ __forceinline__ int mod_ns(int j) const {
        const int q = (int)(((float)j + 0.5f) * rns);
        return j - q * ns;
    }
};

template <int RADIX, int DIR, int NTH, bool first, bool last, bool PF, int CAP, typename C, typename Load,
          typename Store>
__device__ __forceinline__ void fft_pass(C *buf, int N, int K, int Ns, const C *__restrict__ tw, Load &load,
                                         Store &store) {
    constexpr int MAXC = fft_cap<NTH, CAP>();
    constexpr int MAXB = (MAXC + RADIX - 1) / RADIX;
    const int tid = threadIdx.x;
    const int M = N / RADIX;
    const int W = M * K;
    const int tstride = N / (Ns * RADIX);
    const FftIdx ix(K, Ns);
    C v[MAXB][RADIX];
    // PF: every twiddle read up front (FP32 only; worth its registers where
    // few workgroups share a CU, the column passes); otherwise the compact
    // form above, also read up front
    // (FP64: plain reads where they are used, to keep its registers)
    constexpr bool full = PF && sizeof(C) == 8;
    constexpr bool compact = !PF && sizeof(C) == 8;
    C t[full ? MAXB : 1][RADIX - 1];
    TwPre<RADIX, C> tp[compact ? MAXB : 1];
    if constexpr (!first && (full || compact)) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int w = tid + b * NTH;
            if (w < W) {
                const int jm = ix.mod_ns(ix.row(w));
                if constexpr (full) {
#pragma unroll
                    for (int r = 1; r < RADIX; ++r) t[b][r - 1] = tw[jm * r * tstride];
                } else {
                    tp[b] = tw_read<RADIX>(tw, jm * tstride);
                }
            }
        }
    }
    if constexpr (first) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int w = tid + b * NTH;
            if (w < W) {
                const int j = ix.row(w), col = ix.col(w);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[b][r] = load(j + r * M, col);
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int w = tid + b * NTH;
            if (w < W) {
                const int j = ix.row(w), col = ix.col(w);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[b][r] = buf[(fft_lidx(j + r * M) << ix.kshift) + col];
            }
        }
        if constexpr (!last) __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int w = tid + b * NTH;
        if (w < W) {
            const int j = ix.row(w), col = ix.col(w);
            const int jm = ix.mod_ns(j);
            if constexpr (!first && (full || compact)) {
                C wr[RADIX];
                if constexpr (full) {
#pragma unroll
                    for (int r = 1; r < RADIX; ++r) wr[r] = t[full ? b : 0][r - 1];
                } else {
                    tw_powers<RADIX>(tp[compact ? b : 0], wr);
                }
#pragma unroll
                for (int r = 1; r < RADIX; ++r) v[b][r] = DIR < 0 ? cmul(v[b][r], wr[r]) : cmulconj(v[b][r], wr[r]);
            } else if constexpr (!first) {
#pragma unroll
                for (int r = 1; r < RADIX; ++r) {
                    const C tr = tw[jm * r * tstride];
                    v[b][r] = DIR < 0 ? cmul(v[b][r], tr) : cmulconj(v[b][r], tr);
                }
            }
            Dft<RADIX, DIR, C>::run(v[b]);
            const int base = (j - jm) * RADIX + jm;
            if constexpr (last) {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) store(base + r * Ns, col, v[b][r], b * RADIX + r);
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) buf[(fft_lidx(base + r * Ns) << ix.kshift) + col] = v[b][r];
            }
        }
    }
    if constexpr (!last) __syncthreads();
}

// a middle pass (LDS to LDS) as a function of its own: keeps the register
// allocation of the passes separate
struct NoIo {
    template <typename... A> __device__ __forceinline__ void operator()(A...) const {}
};
template <int RADIX, int DIR, int NTH, bool PF, int CAP, typename C>
__device__ __noinline__ void fft_pass_mid(C *buf, int N, int K, int Ns, const C *__restrict__ tw) {
    NoIo none;
    fft_pass<RADIX, DIR, NTH, false, false, PF, CAP>(buf, N, K, Ns, tw, none, none);
}

// one pass of runtime radix r with compile-time role
template <int DIR, int NTH, bool first, bool last, bool PF, int CAP, typename C, typename Load, typename Store>
__device__ __forceinline__ void fft_pass_r(int r, C *buf, int N, int K, int Ns, const C *__restrict__ tw,
                                           Load &load, Store &store) {
    if constexpr (!first && !last) {
        switch (r) {
            case 16: fft_pass_mid<16, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 15: fft_pass_mid<15, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 14: fft_pass_mid<14, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 12: fft_pass_mid<12, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 10: fft_pass_mid<10, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 9: fft_pass_mid<9, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 8: fft_pass_mid<8, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 7: fft_pass_mid<7, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 6: fft_pass_mid<6, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 5: fft_pass_mid<5, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 4: fft_pass_mid<4, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 3: fft_pass_mid<3, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            case 2: fft_pass_mid<2, DIR, NTH, PF, CAP>(buf, N, K, Ns, tw); break;
            default: break;
        }
        return;
    }
    switch (r) {
        case 16: fft_pass<16, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 15: fft_pass<15, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 14: fft_pass<14, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 12: fft_pass<12, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 10: fft_pass<10, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 9: fft_pass<9, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 8: fft_pass<8, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 7: fft_pass<7, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 6: fft_pass<6, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 5: fft_pass<5, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 4: fft_pass<4, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 3: fft_pass<3, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        case 2: fft_pass<2, DIR, NTH, first, last, PF, CAP>(buf, N, K, Ns, tw, load, store); break;
        default: break;
    }
}

// FFT of K interleaved columns of length d.n (K a power of two, d.n * K <= NTH * fft_cap<NTH, CAP>()).
// Input: with IN_LDS the caller has written element n of column col to
// buf[fft_lidx(n) * K + col] and synchronised; otherwise the first pass
// calls load(n, col) -> C.  Output: with OUT_LDS the result is left at
// buf[fft_lidx(o) * K + col] (synchronised); otherwise the last pass calls
// store(o, col, value, slot).  buf holds fft_lds_len(d.n) * K complex
// values.  The caller must synchronise between two calls that share buf.
// PF: prefetch each pass's twiddles (FP32 only).
// Passes that only move data between LDS buffers run as functions of their
// own (fft_pass_mid), which keeps each pass's register allocation apart.
template <bool IN_LDS, bool OUT_LDS, int DIR, int NTH, bool PF, int CAP = 0, typename C, typename Load,
          typename Store>
__device__ __forceinline__ void lds_fft(C *buf, int K, const FftDesc &d, const C *__restrict__ tw, Load &&load,
                                        Store &&store) {
    // d.npass >= 2: every length here is a multiple of 16 and at least 48
    if constexpr (IN_LDS) fft_pass_r<DIR, NTH, false, false, PF, CAP>(d.radix[0], buf, d.n, K, 1, tw, load, store);
    else fft_pass_r<DIR, NTH, true, false, PF, CAP>(d.radix[0], buf, d.n, K, 1, tw, load, store);
    int Ns = d.radix[0];
    for (int s = 1; s < d.npass - 1; ++s) {
        fft_pass_r<DIR, NTH, false, false, PF, CAP>(d.radix[s], buf, d.n, K, Ns, tw, load, store);
        Ns *= d.radix[s];
    }
    if constexpr (OUT_LDS) fft_pass_r<DIR, NTH, false, false, PF, CAP>(d.radix[d.npass - 1], buf, d.n, K, Ns, tw, load, store);
    else fft_pass_r<DIR, NTH, false, true, PF, CAP>(d.radix[d.npass - 1], buf, d.n, K, Ns, tw, load, store);
}

}  // namespace wg
