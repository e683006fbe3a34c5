// Apply-time kernels: LDS-tiled gridder, gather degridder, the two FFT
// passes of each direction with the w-screens fused in, and the image-side
// correction/finalisation kernels.
#pragma once
#include "device_common.hpp"
#include "fft_lds.hpp"

namespace wg {

constexpr int kTileCells = 16;            // uv tile edge (cells)
constexpr int kTileArea = kTileCells * kTileCells;

// Arguments shared by the gridder and the degridder.
// Per selected visibility, in sorted order (built once per plan): the
// kernel-local coordinates z in [-1, 1) of the u, v and w kernels and the
// anchor cell/plane: anc.x = i_u | i_v << 16, anc.y = i_w | fold << 31.
template <typename R> struct VisArgs {
    const R *z;                 // [n_active][3] (z_u, z_v, z_w)
    const int2 *anc;            // [n_active]
    const Cx<R> *vsorted;       // gridder input in sorted order, weighted and unfolded
    const uint32_t *tab_lo;     // [tiles][NJ+1], shift alpha-1
    const uint32_t *tab_hi;     // [tiles][NJ+1], shift 0
    const R *coef;              // [degree+1][alpha] kernel polynomial
    int degree;
    int P;                      // planes per batch
    int NJ;                     // batches
    Geom g;
};

// ---------------------------------------------------------------------------
// Gridder (adjoint, eq. Rad2 before the FFT).  One workgroup owns one 16x16
// tile of the grid for the P = alpha planes of batch J and accumulates every
// visibility whose kernel footprint reaches the tile: those anchored in the
// tile itself and in the three neighbouring tiles up/left (a footprint spans
// at most alpha <= 16 cells).  No two workgroups write the same grid cell,
// so the tile is flushed with plain stores, zeros included.
//
// Visibilities are taken in chunks.  Phase 1, one thread per visibility:
// tile-relative anchor, weighted value, the u and v kernel values and the w
// weights rotated onto the batch's plane slots go to LDS.  Phase 2: wave w
// owns quadrant w (8 x 8 cells) of the tile, lane = cell, and holds that
// cell's P plane accumulators in registers; for every staged visibility
// whose footprint meets the quadrant it adds value * ku * kv * kw[slot] to
// each slot.  Every LDS access in phase 2 is a read, so waves never wait on
// each other and need no atomics.
// ---------------------------------------------------------------------------
template <typename R, int ALPHA> struct GridStage {
    static constexpr int CH = 256;                 // visibilities per chunk (one per phase-1 thread)
    static constexpr int S = CH + 1;               // + one zero-weight slot used as padding
    static constexpr size_t bytes = (size_t)S * (3 * ALPHA * sizeof(R) + sizeof(Cx<R>) + sizeof(int2)) +
                                    4 * CH * sizeof(uint16_t) + 64;
};

template <typename R, int ALPHA>
__global__ __launch_bounds__(256) void k_grid(VisArgs<R> a, int J, Cx<R> *__restrict__ G) {
    using C = Cx<R>;
    using ST = GridStage<R, ALPHA>;
    constexpr int CH = ST::CH, S = ST::S;
    constexpr int P = ALPHA;                                   // plane slots (batch size <= alpha)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *s_kw = reinterpret_cast<R *>(smem_raw);                 // [S][P] rotated w weights
    R *s_ku = s_kw + S * P;                                    // [S][ALPHA]
    R *s_kv = s_ku + S * ALPHA;                                // [S][ALPHA]
    C *s_d = reinterpret_cast<C *>(s_kv + S * ALPHA);          // [S]
    int2 *s_anc = reinterpret_cast<int2 *>(s_d + S);           // [S] (la0, lb0)
    uint16_t *s_list = reinterpret_cast<uint16_t *>(s_anc + S);   // [4][CH] per-quadrant lists
    int *s_cnt = reinterpret_cast<int *>(s_list + 4 * CH);     // [4 quadrants][4 waves]

    const Geom &g = a.g;
    const int ntiles = g.ntu * g.ntv;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    if (tile < 0) return;
    const int A = tile / g.ntv, B = tile - (tile / g.ntv) * g.ntv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qa = (wave >> 1) * 8, qb = (wave & 1) * 8;       // quadrant origin
    const int la = qa + (lane >> 3), lb = qb + (lane & 7);     // this lane's cell
    const int j_lo = J * a.P;
    const int j_hi = min(j_lo + a.P, g.nw);
    // the four contributing bins as one concatenated list
    uint32_t b_s0[4], b_end[4];
    uint32_t total = 0;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        int tu = A - 1 + (nb >> 1);
        int tv = B - 1 + (nb & 1);
        if (tu < 0) tu += g.ntu;
        if (tv < 0) tv += g.ntv;
        const int64_t bin = (int64_t)tu * g.ntv + tv;
        const uint32_t s0 = a.tab_lo[bin * (a.NJ + 1) + J];
        const uint32_t s1 = a.tab_hi[bin * (a.NJ + 1) + J + 1];
        const uint32_t n = s1 > s0 ? s1 - s0 : 0u;
        b_s0[nb] = s0;
        total += n;
        b_end[nb] = total;
    }
    // the padding slot contributes nothing
    if (tid == 0) {
        s_d[CH] = cmake<C>((R)0, (R)0);
        s_anc[CH] = make_int2(1 << 20, 1 << 20);
    }
    if (tid < P) s_kw[CH * P + tid] = (R)0;
    if (tid < ALPHA) {
        s_ku[CH * ALPHA + tid] = (R)0;
        s_kv[CH * ALPHA + tid] = (R)0;
    }
    R acc_re[P], acc_im[P];
#pragma unroll
    for (int r = 0; r < P; ++r) acc_re[r] = acc_im[r] = (R)0;
    const unsigned long long lt = (1ull << lane) - 1ull;

    for (uint32_t base = 0; base < total; base += CH) {
        // ---- phase 1: one thread per visibility -------------------------
        const uint32_t pos = base + tid;
        int qmask = 0;
        if (pos < total) {
            int nb = pos < b_end[0] ? 0 : pos < b_end[1] ? 1 : pos < b_end[2] ? 2 : 3;
            const uint32_t s = b_s0[nb] + (pos - (nb ? b_end[nb - 1] : 0u));
            const int2 an = a.anc[s];
            const int iu = an.x & 0xffff, iv = (an.x >> 16) & 0xffff, iw = an.y & 0x7fffffff;
            int la0 = iu - A * kTileCells;
            int lb0 = iv - B * kTileCells;
            if (la0 > g.nu / 2) la0 -= g.nu;
            if (lb0 > g.nv / 2) lb0 -= g.nv;
            s_anc[tid] = make_int2(la0, lb0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int oa = (q >> 1) * 8, ob = (q & 1) * 8;
                if (la0 <= oa + 7 && la0 + ALPHA > oa && lb0 <= ob + 7 && lb0 + ALPHA > ob) qmask |= 1 << q;
            }
            s_d[tid] = a.vsorted[s];
            const R zu = a.z[3 * (size_t)s], zv = a.z[3 * (size_t)s + 1], zw = a.z[3 * (size_t)s + 2];
            R ku[ALPHA], kv[ALPHA], kw[ALPHA];
            kernel_values_z<ALPHA, R>(zu, a.coef, a.degree, ku);
            kernel_values_z<ALPHA, R>(zv, a.coef, a.degree, kv);
#pragma unroll
            for (int i = 0; i < ALPHA; ++i) {
                s_ku[tid * ALPHA + i] = ku[i];
                s_kv[tid * ALPHA + i] = kv[i];
            }
            // plane slot r holds plane j_lo + r; kernel index j - iw
            if (g.do_w) {
                kernel_values_z<ALPHA, R>(zw, a.coef, a.degree, kw);
                const int sh = j_lo - iw;                      // kernel index of slot 0
#pragma unroll
                for (int rr = 0; rr < P; ++rr) {
                    R wv = (R)0;
#pragma unroll
                    for (int i = 0; i < ALPHA; ++i) wv = (i == rr + sh && j_lo + rr < j_hi) ? kw[i] : wv;
                    s_kw[tid * P + rr] = wv;
                }
            } else {
#pragma unroll
                for (int rr = 0; rr < P; ++rr) s_kw[tid * P + rr] = (R)(rr == 0);
            }
        }
        // per-quadrant lists: wave-level ballots, then offsets across waves
        unsigned long long bal[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bal[q] = __ballot((qmask >> q) & 1);
            if (lane == 0) s_cnt[q * 4 + wave] = (int)__popcll(bal[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if ((qmask >> q) & 1) {
                int off = 0;
                for (int w = 0; w < wave; ++w) off += s_cnt[q * 4 + w];
                s_list[q * CH + off + (int)__popcll(bal[q] & lt)] = (uint16_t)tid;
            }
        }
        __syncthreads();
        // ---- phase 2: this wave's quadrant, lanes = cells, 4 visibilities a step
        const int n = s_cnt[wave * 4 + 0] + s_cnt[wave * 4 + 1] + s_cnt[wave * 4 + 2] + s_cnt[wave * 4 + 3];
        const uint16_t *lst = s_list + wave * CH;
        for (int j = 0; j < n; j += 4) {
            int vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) vv[u] = (j + u < n) ? (int)lst[j + u] : CH;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = vv[u];
                const int2 an = s_anc[v];
                const int i = la - an.x, k = lb - an.y;
                const bool act = (unsigned)i < (unsigned)ALPHA && (unsigned)k < (unsigned)ALPHA;
                const int ic = act ? i : 0, kc = act ? k : 0;
                const R wuv = act ? s_ku[v * ALPHA + ic] * s_kv[v * ALPHA + kc] : (R)0;
                const C d = s_d[v];
                const R fr = d.x * wuv, fi = d.y * wuv;
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const R kwv = s_kw[v * P + r];
                    acc_re[r] += fr * kwv;
                    acc_im[r] += fi * kwv;
                }
            }
        }
        __syncthreads();
    }
    const int np = j_hi - j_lo;
    const int64_t cell_off = (int64_t)(A * kTileCells + la) * g.nv + (B * kTileCells + lb);
#pragma unroll
    for (int r = 0; r < P; ++r)
        if (r < np) G[(int64_t)r * g.nu * g.nv + cell_off] = cmake<C>(acc_re[r], acc_im[r]);
}

// ---------------------------------------------------------------------------
// Degridder (forward, bracket of eq. R3).  One workgroup per 16x16 tile and
// batch: the tile plus its (alpha-1)-cell halo of the P planes is staged in
// LDS, then each thread gathers alpha x alpha x (planes in batch) values for
// its visibilities and adds the batch's partial sum to its accumulator.
// ---------------------------------------------------------------------------
template <typename R, int ALPHA>
__global__ __launch_bounds__(256) void k_degrid(VisArgs<R> a, int J, int PD, const Cx<R> *__restrict__ G,
                                                Cx<R> *__restrict__ visacc) {
    using C = Cx<R>;
    constexpr int W = kTileCells + ALPHA - 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *st = reinterpret_cast<C *>(smem_raw);                  // [PD][W][W]
    const Geom &g = a.g;
    const int ntiles = g.ntu * g.ntv;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    if (tile < 0) return;
    const int A = tile / g.ntv, B = tile - (tile / g.ntv) * g.ntv;
    const int64_t bin = tile;
    const uint32_t s0 = a.tab_lo[bin * (a.NJ + 1) + J];
    const uint32_t s1 = a.tab_hi[bin * (a.NJ + 1) + J + 1];
    if (s0 >= s1) return;
    const int tid = threadIdx.x;
    const int j_lo = J * a.P;
    const int j_hi = min(j_lo + a.P, g.nw);
    // planes are staged PD at a time (tile + halo of PD planes in LDS)
    for (int g0 = j_lo; g0 < j_hi; g0 += PD) {
        const int g1 = min(g0 + PD, j_hi);
        const int np = g1 - g0;
        for (int e = tid; e < np * W * W; e += blockDim.x) {
            const int p = e / (W * W), cell = e - p * (W * W);
            const int ra = cell / W, rb = cell - ra * W;
            int ga = A * kTileCells + ra;
            int gb = B * kTileCells + rb;
            if (ga >= g.nu) ga -= g.nu;
            if (gb >= g.nv) gb -= g.nv;
            st[e] = G[((int64_t)(g0 - j_lo + p) * g.nu + ga) * g.nv + gb];
        }
        __syncthreads();
        for (uint32_t s = s0 + tid; s < s1; s += blockDim.x) {
            const int2 an = a.anc[s];
            const int iu = an.x & 0xffff, iv = (an.x >> 16) & 0xffff, iw = an.y & 0x7fffffff;
            const int la0 = iu - A * kTileCells;   // in [0, 16) by the index
            const int lb0 = iv - B * kTileCells;
            if (la0 < 0 || la0 >= kTileCells || lb0 < 0 || lb0 >= kTileCells) continue;
            const int jw0 = g.do_w ? max(iw, g0) : g0;
            const int jw1 = g.do_w ? min(iw + ALPHA, g1) : g1;
            if (jw0 >= jw1) continue;
            const R zu = a.z[3 * (size_t)s], zv = a.z[3 * (size_t)s + 1], zw = a.z[3 * (size_t)s + 2];
            R ku[ALPHA], kv[ALPHA], kw[ALPHA];
            kernel_values_z<ALPHA, R>(zu, a.coef, a.degree, ku);
            kernel_values_z<ALPHA, R>(zv, a.coef, a.degree, kv);
            if (g.do_w) {
                kernel_values_z<ALPHA, R>(zw, a.coef, a.degree, kw);
            } else {
#pragma unroll
                for (int i = 0; i < ALPHA; ++i) kw[i] = (R)(i == 0);
            }
            R sre = 0, sim = 0;
#pragma unroll
            for (int jw = 0; jw < ALPHA; ++jw) {
                const int j = (g.do_w ? iw : g0) + jw;
                if (j < jw0 || j >= jw1) continue;
                const C *pl = st + (j - g0) * (W * W) + la0 * W + lb0;
                R pre = 0, pim = 0;
#pragma unroll
                for (int i = 0; i < ALPHA; ++i) {
                    R rre = 0, rim = 0;
#pragma unroll
                    for (int k = 0; k < ALPHA; ++k) {
                        const C v = pl[i * W + k];
                        rre += kv[k] * v.x;
                        rim += kv[k] * v.y;
                    }
                    pre += ku[i] * rre;
                    pim += ku[i] * rim;
                }
                sre += kw[jw] * pre;
                sim += kw[jw] * pim;
            }
            C old = visacc[s];
            visacc[s] = cmake<C>(old.x + sre, old.y + sim);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FFT passes.  Grid order: rows (contiguous, along v) then columns (along u).
// ---------------------------------------------------------------------------
struct PassGeom {
    int nu, nv, npix_x, npix_y;
    int P, nw;
    int do_w;
    double w0, dw;
};

// Gridding pass 1: row a of plane p: T[p][a][q] = sum_b G[p][a][b] e^{+2 pi i b q'/N_v}
// for the npix_y retained q (q' = q - npix_y/2), i.e. the pruned output.
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_rows_grid(const Cx<R> *__restrict__ G, Cx<R> *__restrict__ T,
                                                   PassGeom pg, FftDesc fd, const Cx<R> *__restrict__ tw) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int a = blockIdx.x, p = blockIdx.y;
    const C *src = G + ((int64_t)p * pg.nu + a) * pg.nv;
    for (int e = threadIdx.x; e < pg.nv; e += NTH) buf[e] = src[e];
    __syncthreads();
    lds_fft<+1>(buf, 1, fd, tw, threadIdx.x, NTH);
    C *dst = T + ((int64_t)p * pg.nu + a) * pg.npix_y;
    const int h = pg.npix_y / 2;
    for (int q = threadIdx.x; q < pg.npix_y; q += NTH) {
        int b = q - h;
        if (b < 0) b += pg.nv;
        dst[q] = buf[b];
    }
}

// Gridding pass 2: K columns q of every plane in the batch, transform along
// u, keep the npix_x retained p, multiply by the conjugate w-screen
// exp(-2 pi i c_j (n - 1)) (eq. Rad1, phase reduced in FP64) and add the
// real part into the image accumulator (owned by this workgroup).
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_cols_grid(const Cx<R> *__restrict__ T, R *__restrict__ acc,
                                                   const double *__restrict__ nm1, PassGeom pg, int K,
                                                   int j_lo, int np, FftDesc fd,
                                                   const Cx<R> *__restrict__ tw) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    // neighbouring column blocks share cache lines: keep them on one XCD
    const int cb = xcd_remap(blockIdx.x, (pg.npix_y + K - 1) / K);
    if (cb < 0) return;
    const int q0 = cb * K;
    const int kk = min(K, pg.npix_y - q0);
    const int h = pg.npix_x / 2;
    for (int p = 0; p < np; ++p) {
        const C *src = T + (int64_t)p * pg.nu * pg.npix_y;
        for (int e = threadIdx.x; e < pg.nu * K; e += NTH) {
            const int a = e / K, col = e - a * K;
            buf[e] = col < kk ? src[(int64_t)a * pg.npix_y + q0 + col] : cmake<C>((R)0, (R)0);
        }
        __syncthreads();
        lds_fft<+1>(buf, K, fd, tw, threadIdx.x, NTH);
        const double cj = pg.w0 + (double)(j_lo + p) * pg.dw;
        for (int e = threadIdx.x; e < pg.npix_x * kk; e += NTH) {
            const int pp = e / kk, col = e - pp * kk;
            int ga = pp - h;
            if (ga < 0) ga += pg.nu;
            const C hv = buf[ga * K + col];
            const int64_t pix = (int64_t)pp * pg.npix_y + q0 + col;
            R val;
            if (pg.do_w) {
                double ph = cj * nm1[pix];
                ph -= rint(ph);
                R sn, cs;
                if constexpr (sizeof(R) == 4) sincospif((float)(2.0 * ph), &sn, &cs);
                else sincospi(2.0 * ph, &sn, &cs);
                val = hv.x * cs + hv.y * sn;      // Re(h * exp(-2 pi i ph))
            } else {
                val = hv.x;
            }
            acc[pix] += val;
        }
        __syncthreads();
    }
}

// Degridding pass A: image row p, for every plane of the batch: screened
// row I~ exp(+2 pi i c_j (n - 1)) (eqs. R1-R2) placed at the wrapped
// positions of a zero row of length N_v, transformed along v (e^{-2 pi i}).
// Output T[p][row][b], all N_v columns.
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_rows_degrid(const R *__restrict__ itil, const double *__restrict__ nm1,
                                                     Cx<R> *__restrict__ T, PassGeom pg, int j_lo, int np,
                                                     FftDesc fd, const Cx<R> *__restrict__ tw) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int row = blockIdx.x;
    const int h = pg.npix_y / 2;
    const R *irow = itil + (int64_t)row * pg.npix_y;
    const double *nrow = nm1 + (int64_t)row * pg.npix_y;
    for (int p = 0; p < np; ++p) {
        const double cj = pg.w0 + (double)(j_lo + p) * pg.dw;
        for (int b = threadIdx.x; b < pg.nv; b += NTH) {
            int q = b < pg.nv - h ? b + h : b - (pg.nv - h);   // inverse of b = (q - h) mod N_v
            C v = cmake<C>((R)0, (R)0);
            if (q >= 0 && q < pg.npix_y && (b < pg.npix_y - h || b >= pg.nv - h)) {
                const R x = irow[q];
                if (pg.do_w) {
                    double ph = cj * nrow[q];
                    ph -= rint(ph);
                    R sn, cs;
                    if constexpr (sizeof(R) == 4) sincospif((float)(2.0 * ph), &sn, &cs);
                    else sincospi(2.0 * ph, &sn, &cs);
                    v = cmake<C>(x * cs, x * sn);
                } else {
                    v = cmake<C>(x, (R)0);
                }
            }
            buf[b] = v;
        }
        __syncthreads();
        lds_fft<-1>(buf, 1, fd, tw, threadIdx.x, NTH);
        C *dst = T + ((int64_t)p * pg.npix_x + row) * pg.nv;
        for (int b = threadIdx.x; b < pg.nv; b += NTH) dst[b] = buf[b];
        __syncthreads();
    }
}

// Degridding pass B: K grid columns b of plane p: the npix_x rows of T are
// placed at wrapped u positions of a zero column of length N_u and
// transformed along u (e^{-2 pi i}); output G[p][a][b] for all a.
template <typename R, int NTH>
__global__ __launch_bounds__(NTH) void k_cols_degrid(const Cx<R> *__restrict__ T, Cx<R> *__restrict__ G,
                                                     PassGeom pg, int K, FftDesc fd,
                                                     const Cx<R> *__restrict__ tw) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    // neighbouring column blocks share cache lines: keep them on one XCD
    const int cb = xcd_remap(blockIdx.x, (pg.nv + K - 1) / K);
    if (cb < 0) return;
    const int b0 = cb * K;
    const int p = blockIdx.y;
    const int kk = min(K, pg.nv - b0);
    const int h = pg.npix_x / 2;
    const C *src = T + (int64_t)p * pg.npix_x * pg.nv;
    for (int e = threadIdx.x; e < pg.nu * K; e += NTH) {
        const int a = e / K, col = e - a * K;
        // a = (pp - h) mod N_u  <=>  pp = a + h (a < npix_x - h) or a - (N_u - h) (a >= N_u - h)
        int pp = -1;
        if (a < pg.npix_x - h) pp = a + h;
        else if (a >= pg.nu - h) pp = a - (pg.nu - h);
        C v = cmake<C>((R)0, (R)0);
        if (pp >= 0 && col < kk) v = src[(int64_t)pp * pg.nv + b0 + col];
        buf[e] = v;
    }
    __syncthreads();
    lds_fft<-1>(buf, K, fd, tw, threadIdx.x, NTH);
    C *dst = G + (int64_t)p * pg.nu * pg.nv;
    for (int e = threadIdx.x; e < pg.nu * kk; e += NTH) {
        const int a = e / kk, col = e - a * kk;
        dst[(int64_t)a * pg.nv + b0 + col] = buf[a * K + col];
    }
}

// ---- image-side elementwise kernels ----------------------------------------
template <typename R>
__global__ void k_scale_image(const R *__restrict__ in, const double *__restrict__ corr, R *__restrict__ out,
                              int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (R)((double)in[e] * corr[e]);
}

template <typename T>
__global__ void k_fill_zero(T *__restrict__ p, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = T{};
}

// Degridding output: undo the fold (conjugate), apply the weights and
// scatter from sorted order to [n_rows][n_chan].
template <typename R>
__global__ void k_degrid_finish(const Cx<R> *__restrict__ visacc, const uint32_t *__restrict__ order,
                                const int2 *__restrict__ anc, const R *__restrict__ wgt, int64_t n_active,
                                Cx<R> *__restrict__ vis) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_active;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = order[s];
        Cx<R> v = visacc[s];
        if (anc[s].y < 0) v.y = -v.y;
        if (wgt) v = cscale(v, wgt[idx]);
        vis[idx] = v;
    }
}

// Gridding input in sorted order: weighted, and conjugated where folded.
template <typename R>
__global__ void k_gather_vis(const Cx<R> *__restrict__ vis, const R *__restrict__ wgt,
                             const uint32_t *__restrict__ order, const int2 *__restrict__ anc, int64_t n_active,
                             Cx<R> *__restrict__ vsorted) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_active;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = order[s];
        Cx<R> v = vis[idx];
        if (wgt) v = cscale(v, wgt[idx]);
        if (anc[s].y < 0) v.y = -v.y;
        vsorted[s] = v;
    }
}

template <typename R>
__global__ void k_zero_masked(const uint8_t *__restrict__ mask, int64_t n, Cx<R> *__restrict__ vis) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        if (!mask[e]) vis[e] = Cx<R>{};
}

}  // namespace wg
