// FFT passes with the u-axis transform split in two (four-step form), so
// that every pass reads and writes whole rows or wide row pieces.
//
// The u transform of length N_u = S * N1 (S in {4, 8, 16} rows, N1 = N_u/S)
// is taken as
//     X[k2 + S k1] = sum_a1 w_N1^(a1 k1) [ w_N^(a1 k2) sum_a2 w_S^(a2 k2) x[a1 + N1 a2] ]
// (w = e^(+-2 pi i / .)): an S-point DFT across S rows spaced N1 apart,
// a twiddle, then N1-point DFTs.  Gridding fuses the S-point stage into
// the row (v) pass: one workgroup transforms the S rows a1 + N1 a2 of a
// plane, keeps its share of their retained outputs in registers and writes
// the S-point DFT of them.  The N1-point column transforms then read rows
// of a block of Q adjacent columns (Q complex values contiguous) instead of
// K <= 4 columns of full length.  Degridding runs the mirror image: the
// N1-point column transforms of the screened image first, then the S-point
// stage fused into the row pass, which writes whole grid rows.
//
// Intermediate layout Y[p][k2][a1][q], q in [0, npix_y) contiguous: plane
// p of the batch, k2 in [0, S), a1 in [0, N1).
#pragma once
#include "device_common.hpp"
#include "fft_lds.hpp"

namespace wg {

struct SplitGeom {
    int nu, nv, npix_x, npix_y;
    int S, N1;            // N_u = S * N1
    int Q;                // columns per workgroup of the N1-point passes
    int do_w;
    double w0, dw;
};

// grid row ka (u frequency) <-> image row pp, with ka = (pp - h) mod N_u:
// returns pp, or -1 where ka is not one of the npix_x retained rows
__device__ __forceinline__ int split_image_row(int ka, const SplitGeom &sg) {
    const int h = sg.npix_x / 2;
    if (ka < sg.npix_x - h) return ka + h;
    if (ka >= sg.nu - h) return ka - (sg.nu - h);
    return -1;
}

// Gridding, pass 1 (rows along v, fused S-point stage along u).  Block
// (a1, p): rows a = a1 + N1 a2 of plane p, each transformed along v
// (e^{+2 pi i}); thread t keeps image columns q = t + NTH i (i < V) of the
// retained outputs; then per column the S-point DFT over a2 and the twiddle
// e^{+2 pi i a1 k2 / N_u} give Y[p][k2][a1][q].
template <typename R, int NTH, int S, int V>
__global__ __launch_bounds__(NTH) void k_rows_grid_split(const Cx<R> *__restrict__ G, Cx<R> *__restrict__ Y,
                                                         SplitGeom sg, FftDesc fdv,
                                                         const Cx<R> *__restrict__ twv,
                                                         const Cx<R> *__restrict__ twu) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int a1 = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const int hy = sg.npix_y / 2;
    C acc[S][V];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int i = 0; i < V; ++i) acc[k][i] = cmake<C>((R)0, (R)0);
    for (int a2 = 0; a2 < S; ++a2) {
        const C *src = G + ((int64_t)p * sg.nu + a1 + (int64_t)sg.N1 * a2) * sg.nv;
        if (a2 > 0) __syncthreads();          // previous row's outputs read
        lds_fft<false, true, +1, NTH, false>(buf, 1, fdv, twv, [&](int n, int) { return src[n]; }, NoIo{});
        // shift register over the S rows (static register indices): the
        // new row enters at the top, row a2 ends in acc[a2]
#pragma unroll
        for (int k = 0; k < S - 1; ++k)
#pragma unroll
            for (int i = 0; i < V; ++i) acc[k][i] = acc[k + 1][i];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int q = tid + NTH * i;
            C v = cmake<C>((R)0, (R)0);
            if (q < sg.npix_y) {
                int kb = q - hy;                  // output frequency of image column q
                if (kb < 0) kb += sg.nv;
                v = buf[fft_lidx(kb)];
            }
            acc[S - 1][i] = v;
        }
    }
    // S-point DFT over a2, twiddle, store
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int q = tid + NTH * i;
        if (q >= sg.npix_y) continue;
        C v[S];
#pragma unroll
        for (int k = 0; k < S; ++k) v[k] = acc[k][i];
        Dft<S, +1, C>::run(v);
        C *dst = Y + ((int64_t)p * S * sg.N1 + a1) * sg.npix_y + q;
#pragma unroll
        for (int k2 = 0; k2 < S; ++k2) {
            const C w = twu[a1 * k2];                       // e^{-2 pi i a1 k2 / N_u}
            dst[(int64_t)k2 * sg.N1 * sg.npix_y] = cmulconj(v[k2], w);
        }
    }
}

// Gridding, pass 2: block (k2, column block): for every plane of the batch
// the N1-point transforms (e^{+2 pi i}) of columns q0 .. q0 + Q - 1 of
// Y[p][k2][.][q], i.e. grid rows ka = k2 + S k1; the retained rows are
// multiplied by the conjugate w-screen e^{-2 pi i c_j (n - 1)} (eq. Rad1,
// phase reduced in FP64) and their real parts summed over the batch in LDS,
// then added to the image accumulator once (each pixel has one owner).
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_cols_grid_split(const Cx<R> *__restrict__ Y, R *__restrict__ acc,
                                                         const double *__restrict__ nm1, SplitGeom sg, int j_lo,
                                                         int np, FftDesc fd1, const Cx<R> *__restrict__ tw1) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int Q = sg.Q;
    R *sum = reinterpret_cast<R *>(buf + (size_t)fft_lds_len(sg.N1) * Q);   // [N1][Q]
    const int nqb = (sg.npix_y + Q - 1) / Q;
    const int k2 = blockIdx.x / nqb, qb = blockIdx.x - k2 * nqb;
    const int q0 = qb * Q;
    const int kk = min(Q, sg.npix_y - q0);
    const int ne = sg.N1 * Q;
    for (int e = threadIdx.x; e < ne; e += NTH) sum[e] = (R)0;
    for (int p = 0; p < np; ++p) {
        const C *src = Y + ((int64_t)(p * sg.S + k2) * sg.N1) * sg.npix_y + q0;
        const double cj = sg.w0 + (double)(j_lo + p) * sg.dw;
        int Qp = __builtin_amdgcn_readfirstlane(Q);
        asm volatile("" : "+s"(Qp));
        lds_fft<false, true, +1, NTH, true>(
            buf, Qp, fd1, tw1,
            [&](int n, int col) { return col < kk ? src[(int64_t)n * sg.npix_y + col] : cmake<C>((R)0, (R)0); },
            NoIo{});
        for (int e = threadIdx.x; e < ne; e += NTH) {
            const int k1 = e / Q, col = e - k1 * Q;
            const int pp = split_image_row(k2 + sg.S * k1, sg);
            if (pp < 0 || col >= kk) continue;
            const C hv = buf[fft_lidx(k1) * Q + col];
            R val;
            if (sg.do_w) {
                double ph = cj * nm1[(int64_t)pp * sg.npix_y + q0 + col];
                ph -= rint(ph);
                R sn, cs;
                if constexpr (sizeof(R) == 4) sincos_turns_f32(ph, sn, cs);
                else sincospi(2.0 * ph, &sn, &cs);
                val = hv.x * cs + hv.y * sn;      // Re(h * exp(-2 pi i ph))
            } else {
                val = hv.x;
            }
            sum[e] += val;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < ne; e += NTH) {
        const int k1 = e / Q, col = e - k1 * Q;
        const int pp = split_image_row(k2 + sg.S * k1, sg);
        if (pp < 0 || col >= kk) continue;
        acc[(int64_t)pp * sg.npix_y + q0 + col] += sum[e];
    }
}

// Degridding, pass 1: block (k2, column block): for every plane p of the
// batch, the screened image I~ e^{+2 pi i c_j (n - 1)} (eqs. R1-R2) of
// columns q0 .. q0 + Q - 1 at the grid rows ka = k2 + S k1 (zero where ka is
// not a retained row), N1-point transforms (e^{-2 pi i}) and the twiddle
// e^{-2 pi i a1 k2 / N_u}: Y[p][k2][a1][q].
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_cols_degrid_split(const R *__restrict__ itil,
                                                           const double *__restrict__ nm1, Cx<R> *__restrict__ Y,
                                                           SplitGeom sg, int j_lo, int np, FftDesc fd1,
                                                           const Cx<R> *__restrict__ tw1,
                                                           const Cx<R> *__restrict__ twu) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int Q = sg.Q;
    const int nqb = (sg.npix_y + Q - 1) / Q;
    const int k2 = blockIdx.x / nqb, qb = blockIdx.x - k2 * nqb;
    const int q0 = qb * Q;
    const int kk = min(Q, sg.npix_y - q0);
    for (int p = 0; p < np; ++p) {
        const double cj = sg.w0 + (double)(j_lo + p) * sg.dw;
        C *dst = Y + ((int64_t)(p * sg.S + k2) * sg.N1) * sg.npix_y + q0;
        int Qp = __builtin_amdgcn_readfirstlane(Q);
        asm volatile("" : "+s"(Qp));
        if (p > 0) __syncthreads();               // previous plane's last pass done with LDS
        lds_fft<false, false, -1, NTH, true>(
            buf, Qp, fd1, tw1,
            [&](int k1, int col) {
                const int pp = split_image_row(k2 + sg.S * k1, sg);
                if (pp < 0 || col >= kk) return cmake<C>((R)0, (R)0);
                const int64_t e = (int64_t)pp * sg.npix_y + q0 + col;
                const R x = itil[e];
                if (!sg.do_w) return cmake<C>(x, (R)0);
                double ph = cj * nm1[e];
                ph -= rint(ph);
                R sn, cs;
                if constexpr (sizeof(R) == 4) sincos_turns_f32(ph, sn, cs);
                else sincospi(2.0 * ph, &sn, &cs);
                return cmake<C>(x * cs, x * sn);
            },
            [&](int a1, int col, C v, int) {
                if (col < kk) dst[(int64_t)a1 * sg.npix_y + col] = cmul(v, twu[a1 * k2]);
            });
    }
}

// Degridding, pass 2 (S-point stage along u fused with the rows along v).
// Block (a1, p): thread t reads Y[p][k2][a1][q] for its columns
// q = t + NTH i and all k2, forms the S-point DFT over k2 (e^{-2 pi i}),
// which gives rows a = a1 + N1 a2 of the u-transformed screened image; each
// row is placed at the wrapped v positions of a zero row of length N_v,
// transformed along v (e^{-2 pi i}) and written to G[p][a][.].
template <typename R, int NTH, int S, int V>
__global__ __launch_bounds__(NTH) void k_rows_degrid_split(const Cx<R> *__restrict__ Y, Cx<R> *__restrict__ G,
                                                           SplitGeom sg, FftDesc fdv,
                                                           const Cx<R> *__restrict__ twv) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int a1 = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const int hy = sg.npix_y / 2;
    C z[S][V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        const int q = tid + NTH * i;
        C v[S];
        const C *src = Y + ((int64_t)p * S * sg.N1 + a1) * sg.npix_y + q;
#pragma unroll
        for (int k2 = 0; k2 < S; ++k2)
            v[k2] = q < sg.npix_y ? src[(int64_t)k2 * sg.N1 * sg.npix_y] : cmake<C>((R)0, (R)0);
        Dft<S, -1, C>::run(v);
#pragma unroll
        for (int a2 = 0; a2 < S; ++a2) z[a2][i] = v[a2];
    }
    // zero band of the row: v positions npix_y - hy .. N_v - hy - 1 hold no image column
    const int gap0 = sg.npix_y - hy, gap1 = sg.nv - hy;
    for (int a2 = 0; a2 < S; ++a2) {
        if (a2 > 0) __syncthreads();              // previous row's transform done with LDS
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int q = tid + NTH * i;
            if (q < sg.npix_y) {
                int kb = q - hy;                  // grid column of image column q
                if (kb < 0) kb += sg.nv;
                buf[fft_lidx(kb)] = z[0][i];
            }
        }
        for (int b = gap0 + tid; b < gap1; b += NTH) buf[fft_lidx(b)] = cmake<C>((R)0, (R)0);
        // next row moves to the front (static register indices)
#pragma unroll
        for (int k = 0; k < S - 1; ++k)
#pragma unroll
            for (int i = 0; i < V; ++i) z[k][i] = z[k + 1][i];
        __syncthreads();
        C *dst = G + ((int64_t)p * sg.nu + a1 + (int64_t)sg.N1 * a2) * sg.nv;
        lds_fft<true, false, -1, NTH, false>(buf, 1, fdv, twv, NoIo{}, [&](int o, int, C v, int) { dst[o] = v; });
    }
}

}  // namespace wg
