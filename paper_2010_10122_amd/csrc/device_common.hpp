// Device-side building blocks shared by the wgrid kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace wg {

// ---- complex helpers on HIP's vector types (re in .x, im in .y) ----------
template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };
template <typename R> using Cx = typename CplxOf<R>::T;

template <typename C> __device__ __forceinline__ C cmake(decltype(C{}.x) re, decltype(C{}.x) im) {
    C c;
    c.x = re;
    c.y = im;
    return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmulconj(C a, C b) {   // a * conj(b)
    return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) {
    return cmake<C>(a.x * s, a.y * s);
}
// multiply by +i (dir = +1) or -i (dir = -1)
template <int DIR, typename C> __device__ __forceinline__ C cmul_i(C a) {
    return DIR > 0 ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

constexpr double kC = 299792458.0;          // speed of light, m/s
constexpr double kTwoPi = 6.283185307179586476925286766559;

// ---- geometry of a plan, passed by value to kernels ----------------------
struct Geom {
    int nu, nv;          // oversampled grid
    int ntu, ntv;        // tiles per axis (nu / 16, nv / 16)
    int nw;              // w-planes
    int npix_x, npix_y;
    int alpha;
    int do_w;
    double half;         // alpha / 2
    double pixsize_x, pixsize_y;
    double w0, dw;
    int64_t n_chan;
};

// Per-visibility coordinates in the fixed FP64 operation order of the
// binning specification: effective coordinates (Sect. 2), Hermitian fold
// to w >= 0 (eq. Hermitian-symmetry), wrap of u*dl into [0, 1) (the chi of
// eq. nfft), grid coordinates in cells and the first touched cell/plane.
// Every operation is rounded on its own (no contraction), so that keys
// computed here and again by the apply kernels agree bit for bit.
struct VisCoord {
    double gu, gv, xw;   // grid coordinates (cells, cells, planes)
    double ou, ov, ow;   // (first cell) - coordinate, in [-alpha/2, -alpha/2 + 1)
    int iu, iv;          // first touched cell, wrapped into [0, N)
    int iw;              // first touched w-plane
    bool flip;           // fold applied: conjugate the visibility
};

__device__ __forceinline__ VisCoord vis_coord(double u_m, double v_m, double w_m, double scale,
                                              const Geom &g) {
#pragma clang fp contract(off)
    VisCoord c;
    double uu = u_m * scale;
    double vv = v_m * scale;
    double ww = g.do_w ? w_m * scale : 0.0;
    c.flip = ww < 0.0;
    if (c.flip) {
        uu = -uu;
        vv = -vv;
        ww = -ww;
    }
    double xu = uu * g.pixsize_x;
    double xv = vv * g.pixsize_y;
    double fu = xu - floor(xu);
    double fv = xv - floor(xv);
    c.gu = fu * (double)g.nu;
    c.gv = fv * (double)g.nv;
    double cu = ceil(c.gu - g.half);
    double cv = ceil(c.gv - g.half);
    c.ou = cu - c.gu;
    c.ov = cv - c.gv;
    int iu = (int)cu, iv = (int)cv;
    c.iu = iu < 0 ? iu + g.nu : iu;
    c.iv = iv < 0 ? iv + g.nv : iv;
    if (g.do_w) {
        c.xw = (ww - g.w0) / g.dw;
        double cw = ceil(c.xw - g.half);
        c.ow = cw - c.xw;
        c.iw = (int)cw;
    } else {
        c.xw = 0.0;
        c.ow = 0.0;
        c.iw = 0;
    }
    return c;
}

// Kernel values at the alpha cells of the u, v and w axes of one visibility
// from the piecewise polynomials of Sect. 4.2: every cell of an axis shares
// the local variable z = 2 (offset + alpha/2) - 1 in [-1, 1), and cell i
// uses its own coefficients (coef is degree-major: coef[d * ALPHA + i]).
// One read of each coefficient row serves all the axes (alpha independent
// Horner chains per axis and step).  Without the w term (W false) only u
// and v are evaluated and kw is the single plane's unit weight.
template <int ALPHA, typename R, bool W>
__device__ __forceinline__ void kernel_values(R zu, R zv, R zw, const R *__restrict__ coef, int degree,
                                              R ku[ALPHA], R kv[ALPHA], R kw[ALPHA]) {
#pragma unroll
    for (int i = 0; i < ALPHA; ++i) {
        ku[i] = kv[i] = coef[degree * ALPHA + i];
        kw[i] = W ? ku[i] : (R)(i == 0);
    }
    for (int d = degree - 1; d >= 0; --d) {
#pragma unroll
        for (int i = 0; i < ALPHA; ++i) {
            const R c = coef[d * ALPHA + i];
            ku[i] = ku[i] * zu + c;
            kv[i] = kv[i] * zv + c;
            if (W) kw[i] = kw[i] * zw + c;
        }
    }
}
template <int ALPHA, typename R>
__device__ __forceinline__ void kernel_values_z3(bool do_w, R zu, R zv, R zw, const R *__restrict__ coef,
                                                 int degree, R ku[ALPHA], R kv[ALPHA], R kw[ALPHA]) {
    if (do_w) kernel_values<ALPHA, R, true>(zu, zv, zw, coef, degree, ku, kv, kw);
    else kernel_values<ALPHA, R, false>(zu, zv, zw, coef, degree, ku, kv, kw);
}

// sin and cos of 2 pi ph for ph in [-1/2, 1/2] (a phase in turns, already
// reduced by its nearest integer in FP64), result in FP32.  The quarter
// turn k = rint(4 ph) is split off in FP64, so the FP32 remainder
// t = 2 pi (ph - k / 4) lies in [-pi/4, pi/4]; there the Taylor series of
// sin (to t^9) and cos (to t^10) are truncated below 2e-9, under half an
// FP32 ulp of the result; the quadrant then swaps and negates.
__device__ __forceinline__ void sincos_turns_f32(double ph, float &sn, float &cs) {
    const double k = rint(4.0 * ph);
    const float t = (float)(kTwoPi * (ph - 0.25 * k));
    const float t2 = t * t;
    const float s = t * (1.0f + t2 * (-1.0f / 6.0f + t2 * (1.0f / 120.0f + t2 * (-1.0f / 5040.0f +
                                                                                 t2 * (1.0f / 362880.0f)))));
    const float c = 1.0f + t2 * (-0.5f + t2 * (1.0f / 24.0f + t2 * (-1.0f / 720.0f + t2 * (1.0f / 40320.0f +
                                                                                       t2 * (-1.0f / 3628800.0f)))));
    const int q = (int)k & 3;
    const float s1 = (q & 1) ? c : s;
    const float c1 = (q & 1) ? -s : c;
    sn = (q & 2) ? -s1 : s1;
    cs = (q & 2) ? -c1 : c1;
}

// The nine (tile, rank) runs of the gridder stream that tile (A, B) takes:
// its own tile's four ranks, ranks 1-2 of the tile left (B - 1), ranks 2-3
// of the tile above (A - 1), rank 2 of the diagonal one; returned as the row
// (tile * 4 + rank) of the class tables.  Tiles wrap around the grid.
constexpr int kGridSegs = 9;
__device__ __forceinline__ int64_t grid_seg_bin(int sg, int A, int B, int ntu, int ntv) {
    // segment -> (tile offset up, tile offset left, rank)
    int du = 0, dv = 0, rank = sg;
    if (sg >= 4 && sg < 6) { dv = 1; rank = sg - 3; }          // 1, 2
    else if (sg >= 6 && sg < 8) { du = 1; rank = sg - 4; }     // 2, 3
    else if (sg == 8) { du = 1; dv = 1; rank = 2; }
    int tu = A - du, tv = B - dv;
    if (tu < 0) tu += ntu;
    if (tv < 0) tv += ntv;
    return ((int64_t)tu * ntv + tv) * 4 + rank;
}

// blockIdx -> work-item remap that keeps neighbouring tiles on one XCD:
// workgroups are dealt round-robin over the 8 XCDs, so give XCD x the
// contiguous range [x * per, (x + 1) * per).  Returns -1 for padding blocks.
__device__ __forceinline__ int xcd_remap(int bid, int nitems) {
    const int per = (nitems + 7) / 8;
    int item = (bid % 8) * per + bid / 8;
    return item < nitems ? item : -1;
}

}  // namespace wg
