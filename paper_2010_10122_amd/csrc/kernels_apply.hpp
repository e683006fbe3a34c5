// Apply-time kernels: LDS-tiled gridder, gather degridder, the two FFT
// passes of each direction with the w-screens fused in, and the image-side
// correction/finalisation kernels.
#pragma once
#include "device_common.hpp"
#include "fft_lds.hpp"

namespace wg {

constexpr int kTileCells = 16;            // uv tile edge (cells)
constexpr int kTileArea = kTileCells * kTileCells;
#ifndef WG_GRID_ITEM_CAP
#define WG_GRID_ITEM_CAP 512
#endif
constexpr int kGridItemCap = WG_GRID_ITEM_CAP;   // visibilities per gridder work item
constexpr int kDegridItemCap = 512;              // visibilities per degridder work item (one per thread)

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
// tile of the grid for the (at most 8) planes of batch J and accumulates
// every visibility whose kernel footprint reaches the tile: those anchored in
// the tile itself and in the three neighbouring tiles up/left (a footprint
// spans at most alpha <= 16 cells).  No two workgroups write the same grid
// cell, so the tile is flushed with plain stores, zeros included.
//
// Work is dealt in items of at most a fixed number of visibilities (the
// uv coverage is far from uniform: a tile near the origin can hold a hundred
// times the mean), so one launch is made of many similar workgroups.  A tile
// whose list is longer is split over several items: the first writes the
// grid planes, the others write partial tiles to scratch, and k_grid_reduce
// adds those to the planes in item order, so the sum order is fixed.
// ---------------------------------------------------------------------------

// Highest polynomial degree the planner picks for a support of ALPHA cells
// (Sect. 4.2 uses ALPHA + 3); the kernels stage the coefficient table in LDS.
template <int ALPHA> constexpr int kMaxDegree = ALPHA + 3;
template <typename R, int ALPHA> constexpr size_t kCoefBytes = (size_t)(kMaxDegree<ALPHA> + 1) * ALPHA * sizeof(R);

// The w weights of one visibility on the batch's plane slots: slot rr holds
// kernel cell rr + sh (zero outside [0, ALPHA)), for a shift sh in
// [1 - PS, ALPHA - 1].  A barrel shifter over a zero-padded copy: one select
// per element and set bit of the shift, all register indices static.
template <typename R, int ALPHA, int PS>
__device__ __forceinline__ void rotate_w(const R kw[ALPHA], int sh, R out[PS]) {
    constexpr int NE = ALPHA + 2 * (PS - 1);
    R e[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) e[k] = (k >= PS - 1 && k < PS - 1 + ALPHA) ? kw[k - (PS - 1)] : (R)0;
    const int o = sh + PS - 1;                     // in [0, NE - PS]
#pragma unroll
    for (int b = 16; b >= 1; b >>= 1) {
        if (b > NE - PS) continue;
        const bool take = (o & b) != 0;
#pragma unroll
        for (int k = 0; k < NE; ++k) e[k] = take ? (k + b < NE ? e[k + b] : (R)0) : e[k];
    }
#pragma unroll
    for (int rr = 0; rr < PS; ++rr) out[rr] = e[rr];
}

// Block -> work item.  Blocks [0, pad8(n_extra)) take the listed extra items
// (heaviest tiles first in dispatch order, dealt round-robin over the XCDs);
// the following blocks take the first item of every tile, (tile, 0, cap, -1),
// in the XCD-contiguous tile order.  Returns false for padding blocks.
__device__ __forceinline__ bool work_item(const int4 *__restrict__ extra, int n_extra, int ntiles, int cap,
                                          int4 &item) {
    const int pad = (n_extra + 7) & ~7;
    const int b = (int)blockIdx.x;
    if (b < pad) {
        if (b >= n_extra) return false;
        item = extra[b];
        return true;
    }
    const int t = xcd_remap(b - pad, ntiles);
    if (t < 0) return false;
    item = make_int4(t, 0, cap, -1);
    return true;
}

// The visibilities that reach tile (A, B) in batch J: the nine runs of the
// gridder stream (class order) that grid_seg_bin names (the tile's own bin,
// and the parts of the bins up/left whose footprints reach into it), as one
// concatenated list of stream positions.  a.tab_lo / a.tab_hi are the
// stream's (tile, rank) tables.
struct TileBins {
    uint32_t s0[kGridSegs], end[kGridSegs];   // first position, running end of the concatenation
    uint32_t total;
};
template <typename R>
__device__ __forceinline__ TileBins tile_bins(const VisArgs<R> &a, int J, int A, int B) {
    const Geom &g = a.g;
    TileBins tb;
    tb.total = 0;
#pragma unroll
    for (int sg = 0; sg < kGridSegs; ++sg) {
        const int64_t bin = grid_seg_bin(sg, A, B, g.ntu, g.ntv);
        const uint32_t s0 = a.tab_lo[bin * (a.NJ + 1) + J];
        const uint32_t s1 = a.tab_hi[bin * (a.NJ + 1) + J + 1];
        tb.s0[sg] = s0;
        tb.total += s1 > s0 ? s1 - s0 : 0u;
        tb.end[sg] = tb.total;
    }
    return tb;
}
// stream position of entry pos of the concatenation (a select chain, no
// dynamic register indexing)
__device__ __forceinline__ uint32_t tile_bins_pos(const TileBins &tb, uint32_t pos) {
    uint32_t s = tb.s0[0] + pos;
#pragma unroll
    for (int k = 0; k < kGridSegs - 1; ++k) s = pos >= tb.end[k] ? tb.s0[k + 1] + (pos - tb.end[k]) : s;
    return s;
}
// Tile-relative first cell of a footprint and the masks of the tile's rows
// (bm) and columns (cm) of 4 cells it meets.
template <int ALPHA>
__device__ __forceinline__ void footprint_masks(int2 an, int A, int B, const Geom &g, int &la0, int &lb0, int &bm,
                                                int &cm) {
    const int iu = an.x & 0xffff, iv = (an.x >> 16) & 0xffff;
    la0 = iu - A * kTileCells;
    lb0 = iv - B * kTileCells;
    if (la0 > g.nu / 2) la0 -= g.nu;
    if (lb0 > g.nv / 2) lb0 -= g.nv;
    bm = cm = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (la0 <= 4 * q + 3 && la0 + ALPHA > 4 * q) bm |= 1 << q;
        if (lb0 <= 4 * q + 3 && lb0 + ALPHA > 4 * q) cm |= 1 << q;
    }
}
// ---------------------------------------------------------------------------
// The gridder on the matrix cores (FP32 and FP64).  Visibilities are taken
// in chunks; phase 1, one lane per visibility, stages its kernel values,
// operands and footprint masks in LDS; phase 2 is a matrix product per
// 4x4-cell region of the tile.  For the four
// visibilities k of a step and the 16 cells m of a region,
//     D[n][m] += sum_k  dk_k[n] * (ku_k[row m] kv_k[col m]),
// where n = 2 slot + (re, im) and dk_k[n] is the weighted visibility (its
// real or imaginary part) times its w weight on plane slot n / 2; phase 1
// stores the 16 values dk[n] of each visibility, so that a lane reads its
// operand with one LDS read.  That is one v_mfma_f32_16x16x4_f32: lane l supplies
// A[n = l % 16][k] = dk and B[k][m = l % 16] = the uv weight of the cell,
// k = l / 16, and ends holding D[4 (l / 16) + i][l % 16], i.e. cell l % 16
// of planes 2 (l / 16) and 2 (l / 16) + 1.  The u and v kernel rows sit
// back to back with three zeros between them (the zeros after a row are the
// next row's leading ones), so every cell of a region the footprint meets
// indexes a kernel value or a zero.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R> using MfmaAcc = std::conditional_t<sizeof(R) == 4, f32x4, f64x4>;
// D += A B for one 16x16x4 product (FP32 or FP64 matrix cores); lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds 4 values of
// column l % 16 of D: rows 4 (l / 16) + i (FP32) or 4 i + l / 16 (FP64),
// i = 0 .. 3.
__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_16x16x4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Gridder, FP32 on the matrix cores (adjoint, eqs. Rad2 / R2 bracket).
// One 64-lane workgroup per work item (a tile and batch, or a share of a
// long tile list): the wave owns all 16 4x4-cell regions of its tile, 16
// accumulators of 4 values a lane, so no other wave takes part in a chunk.
// Per chunk of 64 visibilities of the tile's nine stream runs: phase 1 one
// lane per visibility (kernel values, rotated w weights, footprint
// masks) into LDS; region lists from the wave's ballots; phase 2 one
// v_mfma_f32_16x16x4_f32 per region and four listed visibilities, two
// regions at a time (see the design notes for the operand layout).  168
// registers: three waves a SIMD (four would spill).  FP64 takes the same
// form with v_mfma_f64_16x16x4_f64 (its D holds the same 16 x 16 layout,
// four values a lane), twice the accumulator registers: two waves a SIMD.
template <typename R, int ALPHA> struct GridStageMx1 {
    static constexpr int CH = 64;
    static constexpr int S = CH + 1;
    static constexpr int KP = ALPHA + 3;
    static constexpr int NKP = (S + 1) * KP + 16;
    static constexpr int NW = 8;                   // plane slots
    static constexpr int ND = 2 * NW;              // A-operand values of a slot (re, im per plane slot)
    static constexpr int LST = CH + 8;             // per-region list: entries + padding
    static constexpr size_t al(size_t x) { return (x + 15) & ~(size_t)15; }
    static constexpr size_t off_kv = al((size_t)NKP * sizeof(R));
    static constexpr size_t off_dk = al(off_kv + (size_t)NKP * sizeof(R));
    static constexpr size_t off_bs = al(off_dk + (size_t)S * ND * sizeof(R));
    static constexpr size_t off_list = al(off_bs + (size_t)S * sizeof(int2));
    static constexpr size_t off_coef = al(off_list + (size_t)16 * LST);
    static constexpr size_t bytes = off_coef + kCoefBytes<R, ALPHA>;
};

template <typename R, int ALPHA, int PS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2)))
void k_grid_mx1(VisArgs<R> a, int J, const int4 *__restrict__ extra, int n_extra, int cap,
                Cx<R> *__restrict__ G, Cx<R> *__restrict__ part) {
    using C = Cx<R>;
    using ST = GridStageMx1<R, ALPHA>;
    constexpr int CH = ST::CH, KP = ST::KP, NW = ST::NW, ND = ST::ND, LST = ST::LST;
    static_assert(PS <= NW, "one w weight per plane slot");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *s_ku = reinterpret_cast<R *>(smem_raw);
    R *s_kv = reinterpret_cast<R *>(smem_raw + ST::off_kv);
    R *s_dk = reinterpret_cast<R *>(smem_raw + ST::off_dk);
    int2 *s_bs = reinterpret_cast<int2 *>(smem_raw + ST::off_bs);
    uint8_t *s_list = reinterpret_cast<uint8_t *>(smem_raw + ST::off_list);
    R *s_coef = reinterpret_cast<R *>(smem_raw + ST::off_coef);

    const Geom &g = a.g;
    int4 item;
    if (!work_item(extra, n_extra, g.ntu * g.ntv, cap, item)) return;
    const int tile = item.x;
    const int A = tile / g.ntv, B = tile - (tile / g.ntv) * g.ntv;
    const int lane = threadIdx.x;
    const int kv_of = lane >> 4, m = lane & 15;
    const int mr = m >> 2, cc = m & 3;
    const int j_lo = J * a.P;
    const int j_hi = min(j_lo + a.P, g.nw);
    const TileBins tb = tile_bins(a, J, A, B);
    const uint32_t first = (uint32_t)item.y;
    const uint32_t last = min(tb.total, first + (uint32_t)item.z);
    struct In {
        int2 an;
        C d;
        R zu, zv, zw;
    };
    auto load_in = [&](uint32_t pos) {
        In r;
        const uint32_t s = tile_bins_pos(tb, pos);
        r.an = a.anc[s];
        r.d = a.vsorted[s];
        r.zu = a.z[3 * (size_t)s];
        r.zv = a.z[3 * (size_t)s + 1];
        r.zw = a.z[3 * (size_t)s + 2];
        return r;
    };
    In in{};
    if (first + lane < last) in = load_in(first + lane);
    for (int e = lane; e < ST::NKP; e += CH) {
        s_ku[e] = (R)0;
        s_kv[e] = (R)0;
    }
    if (lane < ND) s_dk[CH * ND + lane] = (R)0;
    if (lane == 0) s_bs[CH] = make_int2(CH * KP, CH * KP);
    for (int e = lane; e < (a.degree + 1) * ALPHA; e += CH) s_coef[e] = a.coef[e];
    MfmaAcc<R> acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = MfmaAcc<R>{(R)0, (R)0, (R)0, (R)0};
    __syncthreads();

    for (uint32_t base = first; base < last; base += CH) {
        const uint32_t pos = base + lane;
        int bm = 0, cm = 0;
        if (pos < last) {
            const int iw = in.an.y & 0x7fffffff;
            int la0, lb0;
            footprint_masks<ALPHA>(in.an, A, B, g, la0, lb0, bm, cm);
            s_bs[lane] = make_int2(3 + lane * KP - la0, 3 + lane * KP - lb0);
            R ku[ALPHA], kv[ALPHA], kw[ALPHA];
            kernel_values_z3<ALPHA, R>(g.do_w, in.zu, in.zv, in.zw, s_coef, a.degree, ku, kv, kw);
            R *pu = s_ku + 3 + lane * KP;
            R *pv = s_kv + 3 + lane * KP;
#pragma unroll
            for (int i = 0; i < ALPHA; ++i) {
                pu[i] = ku[i];
                pv[i] = kv[i];
            }
            R ws[PS];
            if (g.do_w) {
                rotate_w<R, ALPHA, PS>(kw, j_lo - iw, ws);
            } else {
#pragma unroll
                for (int rr = 0; rr < PS; ++rr) ws[rr] = rr == 0 ? (R)1 : (R)0;
            }
            // the A operand of this slot, once: row n holds the visibility's
            // real or imaginary part times the w weight of a plane slot r
            // (zero past the batch's slots), so that lane l ends with slots
            // 2 (l / 16) and 2 (l / 16) + 1 as (re, im) pairs: n = 2 r + c
            // with the FP32 result layout, n = 4 (2 (r % 2) + c) + r / 2
            // with the FP64 one
            if constexpr (sizeof(R) == 4) {
                C *pd = reinterpret_cast<C *>(s_dk + lane * ND);
#pragma unroll
                for (int r = 0; r < NW; ++r) {
                    const R wr = r < PS ? ws[r < PS ? r : 0] : (R)0;
                    pd[r] = cmake<C>(in.d.x * wr, in.d.y * wr);
                }
            } else {
                R *pd = s_dk + lane * ND;
#pragma unroll
                for (int r = 0; r < NW; ++r) {
                    const R wr = r < PS ? ws[r < PS ? r : 0] : (R)0;
                    pd[4 * (2 * (r % 2)) + r / 2] = in.d.x * wr;
                    pd[4 * (2 * (r % 2) + 1) + r / 2] = in.d.y * wr;
                }
            }
        }
        // region lists from the wave's ballots: region rg holds, in lane
        // order, the slots whose footprint meets it, padded with the zero
        // slot up to a multiple of 4 plus the 4 entries read ahead
        unsigned long long balr[4], balc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            balr[q] = __ballot((bm >> q) & 1);
            balc[q] = __ballot((cm >> q) & 1);
        }
        int cnt[16];
#pragma unroll
        for (int rg = 0; rg < 16; ++rg) {
            const unsigned long long bal = balr[rg >> 2] & balc[rg & 3];
            cnt[rg] = __popcll(bal);
            const int at = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            if ((bm >> (rg >> 2)) & (cm >> (rg & 3)) & 1) s_list[rg * LST + at] = (uint8_t)lane;
        }
        {
            // lanes 4 rg .. 4 rg + 3 pad region rg, two entries each
            const int rg = lane >> 2, k0 = (lane & 3) * 2;
            int n = cnt[0];
#pragma unroll
            for (int q = 1; q < 16; ++q) n = rg == q ? cnt[q] : n;
            const int end = ((n + 3) & ~3) + 4;
            if (n + k0 < end) s_list[rg * LST + n + k0] = (uint8_t)CH;
            if (n + k0 + 1 < end) s_list[rg * LST + n + k0 + 1] = (uint8_t)CH;
        }
        __syncthreads();
        if (base + CH + lane < last) in = load_in(base + CH + lane);
#pragma unroll
        for (int qp = 0; qp < 8; ++qp) {
            const int qa = 2 * qp, qb = 2 * qp + 1;
            const int n4a = (cnt[qa] + 3) & ~3, n4b = (cnt[qb] + 3) & ~3;
            const int n4 = max(n4a, n4b);
            const uint8_t *lsta = s_list + qa * LST + kv_of;
            const uint8_t *lstb = s_list + qb * LST + kv_of;
            const int rowa = 4 * (qa >> 2) + mr, cola = 4 * (qa & 3) + cc;
            const int rowb = 4 * (qb >> 2) + mr, colb = 4 * (qb & 3) + cc;
            unsigned va = lsta[0], vb = lstb[0];
            int2 bsa = s_bs[va], bsb = s_bs[vb];
            for (int j = 0; j < n4; j += 4) {
                const R kua = s_ku[bsa.x + rowa], kva = s_kv[bsa.y + cola];
                const R kub = s_ku[bsb.x + rowb], kvb = s_kv[bsb.y + colb];
                const R ava = s_dk[va * ND + m], avb = s_dk[vb * ND + m];
                unsigned vna = lsta[min(j + 4, n4a)], vnb = lstb[min(j + 4, n4b)];
                int2 bsna = s_bs[vna], bsnb = s_bs[vnb];
                acc[qa] = mfma_16x16x4(ava, kua * kva, acc[qa]);
                acc[qb] = mfma_16x16x4(avb, kub * kvb, acc[qb]);
                asm volatile("" : "+v"(vna), "+v"(bsna.x), "+v"(bsna.y), "+v"(vnb), "+v"(bsnb.x), "+v"(bsnb.y));
                va = vna;
                bsa = bsna;
                vb = vnb;
                bsb = bsnb;
            }
        }
        __syncthreads();
    }
    const int np = j_hi - j_lo;
    const int r0 = 2 * kv_of;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = 4 * (q >> 2) + mr, colw = 4 * (q & 3) + cc;
        C *dst;
        int64_t pstride;
        if (item.w < 0) {
            dst = G + (int64_t)(A * kTileCells + row) * g.nv + (B * kTileCells + colw);
            pstride = (int64_t)g.nu * g.nv;
        } else {
            dst = part + (size_t)item.w * a.P * kTileArea + row * kTileCells + colw;
            pstride = kTileArea;
        }
        if (r0 < np) dst[r0 * pstride] = cmake<C>(acc[q][0], acc[q][1]);
        if (r0 + 1 < np) dst[(r0 + 1) * pstride] = cmake<C>(acc[q][2], acc[q][3]);
    }
}

// Adds the partial tiles of split gridder items to the grid planes, in item
// order.  One workgroup per split tile (tile, first slot, slots), one thread
// per cell.
template <typename R>
__global__ __launch_bounds__(256) void k_grid_reduce(const int4 *__restrict__ red, int n_red, int P, int np,
                                                     Geom g, const Cx<R> *__restrict__ part,
                                                     Cx<R> *__restrict__ G) {
    using C = Cx<R>;
    const int e = blockIdx.x;
    if (e >= n_red) return;
    const int4 r4 = red[e];
    const int tile = r4.x;
    const int A = tile / g.ntv, B = tile - (tile / g.ntv) * g.ntv;
    const int la = threadIdx.x >> 4, lb = threadIdx.x & 15;
    const int64_t cell_off = (int64_t)(A * kTileCells + la) * g.nv + (B * kTileCells + lb);
    for (int r = 0; r < np; ++r) {
        C *gp = G + (int64_t)r * g.nu * g.nv + cell_off;
        C acc = *gp;
        for (int k = 0; k < r4.z; ++k) {
            const C v = part[((size_t)(r4.y + k) * P + r) * kTileArea + threadIdx.x];
            acc.x += v.x;
            acc.y += v.y;
        }
        *gp = acc;
    }
}

// ---------------------------------------------------------------------------
// Degridder (forward, bracket of eq. R3).  One workgroup per work item (a
// run of at most a fixed number of the visibilities anchored in one 16x16
// tile) and batch: the tile plus its (alpha-1)-cell halo of the P planes is
// staged in LDS, then each thread gathers alpha x alpha x (planes in batch)
// values for its visibilities and adds the batch's partial sum to its
// accumulator.
// ---------------------------------------------------------------------------
template <typename R, int ALPHA>
__global__ __launch_bounds__(256) void k_degrid(VisArgs<R> a, int J, int PD, const int4 *__restrict__ extra,
                                                int n_extra, int cap, const Cx<R> *__restrict__ G,
                                                Cx<R> *__restrict__ visacc) {
    using C = Cx<R>;
    constexpr int W = kTileCells + ALPHA - 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *st = reinterpret_cast<C *>(smem_raw);                  // [PD][W][W]
    R *s_coef = reinterpret_cast<R *>(smem_raw + (((size_t)PD * W * W * sizeof(C) + 15) & ~(size_t)15));
    const Geom &g = a.g;
    int4 item;                                                 // (tile, first position, count, -)
    if (!work_item(extra, n_extra, g.ntu * g.ntv, cap, item)) return;
    const int tile = item.x;
    const int A = tile / g.ntv, B = tile - (tile / g.ntv) * g.ntv;
    uint32_t s0, s1;
    if (item.w == -1) {                                        // first item of the tile: its bin's run
        s0 = a.tab_lo[(int64_t)tile * (a.NJ + 1) + J];
        const uint32_t e = a.tab_hi[(int64_t)tile * (a.NJ + 1) + J + 1];
        s1 = e > s0 ? s0 + min(e - s0, (uint32_t)cap) : s0;
    } else {
        s0 = (uint32_t)item.y;
        s1 = s0 + (uint32_t)item.z;
    }
    if (s0 >= s1) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < (a.degree + 1) * ALPHA; e += blockDim.x) s_coef[e] = a.coef[e];
    const int j_lo = J * a.P;
    int j_hi = min(j_lo + a.P, g.nw);
    int j_first = j_lo;
    if (g.do_w) {
        // the run is sorted by first plane: only planes from the first
        // visibility's to the last one's footprint are read
        const int iw0 = a.anc[s0].y & 0x7fffffff, iw1 = a.anc[s1 - 1].y & 0x7fffffff;
        j_first = max(j_lo, iw0);
        j_hi = min(j_hi, iw1 + ALPHA);
    }
    // Staging (FP32) copies window cell c = tid + k * 256 of each plane; its
    // offset within a plane (the window wraps around the grid; N_u * N_v <
    // 2^32 since the anchors hold 16 bits per axis) is formed once per
    // group, not once per plane and cell.
    constexpr int WW = W * W;
    constexpr int KC = (WW + 255) / 256;
    // One visibility per thread and chunk: its inputs are read before the
    // chunk's first barrier, its kernel values once (while the first group
    // of planes is staged), and its sum is kept in registers over the
    // staged groups and added to the accumulator once.
    for (uint32_t c0 = s0; c0 < s1; c0 += blockDim.x) {
        const uint32_t s = c0 + tid;
        bool act = s < s1;
        int2 an = make_int2(0, 0);
        R zu = 0, zv = 0, zw = 0;
        C old = cmake<C>((R)0, (R)0);
        if (act) {
            an = a.anc[s];
            zu = a.z[3 * (size_t)s];
            zv = a.z[3 * (size_t)s + 1];
            zw = a.z[3 * (size_t)s + 2];
            old = visacc[s];
        }
        const int iu = an.x & 0xffff, iv = (an.x >> 16) & 0xffff, iw = an.y & 0x7fffffff;
        const int la0 = iu - A * kTileCells;   // in [0, 16) by the index
        const int lb0 = iv - B * kTileCells;
        act = act && la0 >= 0 && la0 < kTileCells && lb0 >= 0 && lb0 < kTileCells;
        R ku[ALPHA], kv[ALPHA], kw[ALPHA];
        R sre = 0, sim = 0;
        __syncthreads();                       // coefficients staged; previous chunk's readers done
        // planes are staged PD at a time (tile + halo of PD planes in LDS)
        for (int g0 = j_first; g0 < j_hi; g0 += PD) {
            const int g1 = min(g0 + PD, j_hi);
            const int np = g1 - g0;
            if (g0 != j_first) __syncthreads();   // the previous group's readers are done
            if constexpr (sizeof(R) == 8) {
                // FP64: the plain loop (the form below costs registers, and
                // with them a wave per SIMD)
                for (int e = tid; e < np * WW; e += 256) {
                    const int p = e / WW, cell = e - p * WW;
                    const int ra = cell / W, rb = cell - ra * W;
                    int ga = A * kTileCells + ra;
                    int gb = B * kTileCells + rb;
                    if (ga >= g.nu) ga -= g.nu;
                    if (gb >= g.nv) gb -= g.nv;
                    st[e] = G[((int64_t)(g0 - j_lo + p) * g.nu + ga) * g.nv + gb];
                }
            } else {
                uint32_t src_off[KC];
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    const int c = tid + k * 256;
                    const int ra = c / W, rb = c - (c / W) * W;
                    int ga = A * kTileCells + ra;
                    int gb = B * kTileCells + rb;
                    if (ga >= g.nu) ga -= g.nu;
                    if (gb >= g.nv) gb -= g.nv;
                    src_off[k] = (uint32_t)ga * (uint32_t)g.nv + (uint32_t)gb;
                }
                for (int p = 0; p < np; ++p) {
                    const C *plane = G + (int64_t)(g0 - j_lo + p) * g.nu * g.nv;
#pragma unroll
                    for (int k = 0; k < KC; ++k) {
                        const int c = tid + k * 256;
                        if (k < KC - 1 || c < WW) st[p * WW + c] = plane[src_off[k]];
                    }
                }
            }
            if (g0 == j_first && act) {
                kernel_values_z3<ALPHA, R>(g.do_w, zu, zv, zw, s_coef, a.degree, ku, kv, kw);
            }
            __syncthreads();
            const int jw0 = g.do_w ? max(iw, g0) : g0;
            const int jw1 = g.do_w ? min(iw + ALPHA, g1) : g1;
            if (!act || jw0 >= jw1) continue;
            // the gather of one staged plane q with weight wq
            auto plane = [&](int q, R wq) {
                const C *pl = st + q * (W * W) + la0 * W + lb0;
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
                sre += wq * pre;
                sim += wq * pim;
            };
            if constexpr (sizeof(R) == 8) {
                // FP64: the w weights rotated onto the staged planes (slot q
                // holds plane g0 + q, zero where the footprint does not reach
                // it), so that every lane walks the same np planes (measured
                // faster in FP64, slower in FP32, where the lanes of a sorted
                // run share most planes anyway)
                constexpr int PSD = 4;
                R ws[PSD];
                if (g.do_w) {
                    rotate_w<R, ALPHA, PSD>(kw, g0 - iw, ws);
                } else {
#pragma unroll
                    for (int q = 0; q < PSD; ++q) ws[q] = (R)(q == 0);
                }
#pragma unroll
                for (int q = 0; q < PSD; ++q) {
                    if (q >= np) break;
                    plane(q, ws[q]);
                }
            } else {
#pragma unroll
                for (int jw = 0; jw < ALPHA; ++jw) {
                    const int j = (g.do_w ? iw : g0) + jw;
                    if (j < jw0 || j >= jw1) continue;
                    plane(j - g0, kw[jw]);
                }
            }
        }
        if (act) visacc[s] = cmake<C>(old.x + sre, old.y + sim);
    }
}

// ---------------------------------------------------------------------------
// FFT passes.  Grid order: rows (contiguous, along v) then columns (along u).
// ---------------------------------------------------------------------------
// The intermediate T between the two passes of each direction is stored in
// panels of kPanel columns: T[p][c / kPanel][r][c % kPanel] (r the row the
// first pass transformed, c its retained output column).  A panel row is one
// 128-byte line (FP32), so the first pass still writes whole lines, and the
// K <= kPanel columns a column-pass workgroup reads lie in one panel, whose
// rows follow each other in memory (not a 32-byte piece every row stride).
constexpr int kPanel = 16;
__host__ __device__ inline int64_t panel_elems(int cols, int rows) {
    return (int64_t)((cols + kPanel - 1) / kPanel) * rows * kPanel;
}

struct PassGeom {
    int nu, nv, npix_x, npix_y;
    int P, nw;
    int do_w;
    double w0, dw;
};

// Gridding pass 1: row a of plane p: T[p][a][q] = sum_b G[p][a][b] e^{+2 pi i b q'/N_v}
// for the npix_y retained q (q' = q - npix_y/2), i.e. the pruned output.
// The first FFT pass reads the row from HBM, the last writes T.
template <typename R, int NTH, int CAP>
__global__ __launch_bounds__(NTH) void k_rows_grid(const Cx<R> *__restrict__ G, Cx<R> *__restrict__ T,
                                                   PassGeom pg, FftDesc fd, const Cx<R> *__restrict__ tw) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int a = blockIdx.x, p = blockIdx.y;
    const C *src = G + ((int64_t)p * pg.nu + a) * pg.nv;
    // row a of panel 0 of plane p; panel c holds columns c kPanel ..
    C *dst = T + p * panel_elems(pg.npix_y, pg.nu) + (int64_t)a * kPanel;
    const int64_t pstride = (int64_t)pg.nu * kPanel;
    const int h = pg.npix_y / 2;
    lds_fft<false, false, +1, NTH, false, CAP>(
        buf, 1, fd, tw, [&](int n, int) { return src[n]; },
        [&](int o, int, C v, int) {
            // output frequency o holds image column q with o = (q - h) mod N_v
            int q = o + h;
            if (q >= pg.nv) q -= pg.nv;
            if (q < pg.npix_y) dst[(q / kPanel) * pstride + (q % kPanel)] = v;
        });
}

// Gridding pass 2: K columns q of every plane in the batch, transform along
// u, keep the npix_x retained p, multiply by the conjugate w-screen
// exp(-2 pi i c_j (n - 1)) (eq. Rad1, phase reduced in FP64) and add the
// real part into the image accumulator (owned by this workgroup).  The sum
// over the batch's planes stays in LDS and is added to the image once.
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
    // the image pixels of this column block, summed over the batch's planes
    // in LDS behind the FFT buffer (each thread owns pixels e = tid + i * NTH)
    // and added to the image once
    R *sum = reinterpret_cast<R *>(buf + (size_t)fft_lds_len(pg.nu) * K);
    const int ne = pg.npix_x * kk;
    // pixel e of the block is image row pp, column q0 + col (the float
    // quotient is exact for e < 2^20)
    const float rk = 1.0f / (float)kk;
    const int kshift = __builtin_ctz((unsigned)K);   // K is a power of two
    auto pixel = [&](int e, int &pp, int &col) {
        pp = (int)(((float)e + 0.5f) * rk);
        col = e - pp * kk;
    };
    for (int e = threadIdx.x; e < ne; e += NTH) sum[e] = (R)0;
    // n - 1 of this thread's pixels, read once for the batch and held in
    // registers where they fit (kColPix a thread): a column of the n - 1
    // table is a strided read of one 8-byte value per image row, which per
    // plane cost more than the transform at K = 1
    constexpr int kColPix = sizeof(R) == 4 ? 12 : 1;   // FP64: its registers are spoken for
    const bool nm_regs = sizeof(R) == 4 && pg.do_w && ne <= NTH * kColPix;
    double nmr[kColPix];
    if (nm_regs) {
#pragma unroll
        for (int i = 0; i < kColPix; ++i) {
            const int e = threadIdx.x + i * NTH;
            nmr[i] = 0.0;
            if (e < ne) {
                int pp, col;
                pixel(e, pp, col);
                nmr[i] = nm1[(int64_t)pp * pg.npix_y + q0 + col];
            }
        }
    }
    for (int p = 0; p < np; ++p) {
        // the K columns q0 .. lie in one panel (K divides kPanel)
        const C *src = T + p * panel_elems(pg.npix_y, pg.nu) + (int64_t)(q0 / kPanel) * pg.nu * kPanel + q0 % kPanel;
        const double cj = pg.w0 + (double)(j_lo + p) * pg.dw;
        // an opaque copy of K per plane: otherwise every FFT address is
        // hoisted out of the plane loop and held in registers across it
        int Kp = __builtin_amdgcn_readfirstlane(K);
        asm volatile("" : "+s"(Kp));
        lds_fft<false, true, +1, NTH, true>(
            buf, Kp, fd, tw,
            [&](int n, int col) {
                return col < kk ? src[(int64_t)n * kPanel + col] : cmake<C>((R)0, (R)0);
            },
            NoIo{});
        // the screened real part of pixel e (n - 1 given)
        auto screen = [&](int e, int pp, int col, double nmv) {
            // image row pp sits at grid row (pp - h) mod N_u
            int ga = pp - h;
            if (ga < 0) ga += pg.nu;
            const C hv = buf[(fft_lidx(ga) << kshift) + col];
            R val;
            if (pg.do_w) {
                double ph = cj * nmv;
                ph -= rint(ph);
                R sn, cs;
                if constexpr (sizeof(R) == 4) sincos_turns_f32(ph, sn, cs);
                else sincospi(2.0 * ph, &sn, &cs);
                val = hv.x * cs + hv.y * sn;      // Re(h * exp(-2 pi i ph))
            } else {
                val = hv.x;
            }
            sum[e] += val;
        };
        if (nm_regs) {
#pragma unroll
            for (int i = 0; i < kColPix; ++i) {
                const int e = threadIdx.x + i * NTH;
                if (e < ne) {
                    int pp, col;
                    pixel(e, pp, col);
                    screen(e, pp, col, nmr[i]);
                }
            }
        } else {
            for (int e = threadIdx.x; e < ne; e += NTH) {
                int pp, col;
                pixel(e, pp, col);
                screen(e, pp, col, pg.do_w ? nm1[(int64_t)pp * pg.npix_y + q0 + col] : 0.0);
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < ne; e += NTH) {
        int pp, col;
        pixel(e, pp, col);
        acc[(int64_t)pp * pg.npix_y + q0 + col] += sum[e];
    }
}

// Degridding pass A: image row p, one plane of the batch per workgroup: screened
// row I~ exp(+2 pi i c_j (n - 1)) (eqs. R1-R2) placed at the wrapped
// positions of a zero row of length N_v, transformed along v (e^{-2 pi i});
// the last FFT pass writes T[p][row][b], all N_v columns.
template <typename R, int NTH, int CAP>
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
    {
        const int p = blockIdx.y;
        const double cj = pg.w0 + (double)(j_lo + p) * pg.dw;
        // row `row` of panel 0 of plane p; panel c holds grid columns c kPanel ..
        C *dst = T + p * panel_elems(pg.nv, pg.npix_x) + (int64_t)row * kPanel;
        const int64_t pstride = (int64_t)pg.npix_x * kPanel;
        for (int b = threadIdx.x; b < pg.nv; b += NTH) {
            // grid position b holds image column q with b = (q - h) mod N_v
            const int q = b < pg.nv - h ? b + h : b - (pg.nv - h);
            C v = cmake<C>((R)0, (R)0);
            if (q < pg.npix_y && (b < pg.npix_y - h || b >= pg.nv - h)) {
                const R x = irow[q];
                if (pg.do_w) {
                    double ph = cj * nrow[q];
                    ph -= rint(ph);
                    R sn, cs;
                    if constexpr (sizeof(R) == 4) sincos_turns_f32(ph, sn, cs);
                    else sincospi(2.0 * ph, &sn, &cs);
                    v = cmake<C>(x * cs, x * sn);
                } else {
                    v = cmake<C>(x, (R)0);
                }
            }
            buf[fft_lidx(b)] = v;
        }
        __syncthreads();
        lds_fft<true, false, -1, NTH, false, CAP>(buf, 1, fd, tw, NoIo{}, [&](int o, int, C v, int) {
            dst[(o / kPanel) * pstride + (o % kPanel)] = v;
        });
    }
}

// Degridding pass B: K grid columns b of plane p: the npix_x rows of T are
// placed at wrapped u positions of a zero column of length N_u and
// transformed along u (e^{-2 pi i}); output G[p][a][b] for all a.
template <typename R, int NTH, int CAP>
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
    // the K columns b0 .. lie in one panel (K divides kPanel)
    const C *src = T + p * panel_elems(pg.nv, pg.npix_x) + (int64_t)(b0 / kPanel) * pg.npix_x * kPanel + b0 % kPanel;
    C *dst = G + (int64_t)p * pg.nu * pg.nv;
    lds_fft<false, false, -1, NTH, true, CAP>(
        buf, K, fd, tw,
        [&](int a, int col) {
            // a = (pp - h) mod N_u  <=>  pp = a + h (a < npix_x - h) or a - (N_u - h) (a >= N_u - h)
            int pp = -1;
            if (a < pg.npix_x - h) pp = a + h;
            else if (a >= pg.nu - h) pp = a - (pg.nu - h);
            return (pp >= 0 && col < kk) ? src[(int64_t)pp * kPanel + col] : cmake<C>((R)0, (R)0);
        },
        [&](int o, int col, C v, int) {
            if (col < kk) dst[(int64_t)o * pg.nv + b0 + col] = v;
        });
}

// ---- four-step column transform ---------------------------------------------
// Where a whole column of length N = N_u fits a workgroup only once (one
// column per workgroup: every global access a lone 8- or 16-byte piece of a
// cache line), the u transform runs in two passes over the 16-column panels
// of the intermediate, each moving whole panel rows.  With N = n1 n2,
// input index a = n2 s + t and output index k = r + n1 q
// (s, r < n1; t, q < n2):
//   X[r + n1 q] = sum_t w_n2^{t q} w_N^{t r} sum_s x[n2 s + t] w_n1^{s r},
// w_m = exp(DIR 2 pi i / m).  Pass A: for one t, the n1-point transforms
// over s, times w_N^{t r}, into Y[p][panel][r][t][16]; pass B: for one r,
// the n2-point transforms over t.
struct Col4Geom {
    int n, n1, n2;           // N = n1 n2
    int rows_in;             // rows of the pass-A input panels
    int h;                   // pruned input (degridding): row pp sits at a = (pp - h) mod N
    int ncols;               // valid columns (the last panel may be partial)
    int64_t in_plane;        // elements per plane of the input panels
    int64_t y_plane;         // elements per plane of Y
};

// Pass A.  Block (panel * n2 + t, plane).  PRUNED: the input holds only the
// rows_in image rows (degridding), zero elsewhere; otherwise all N rows.
template <typename R, int NTH, int CAP, int DIR, bool PRUNED>
__global__ __launch_bounds__(NTH) void k_col4_a(const Cx<R> *__restrict__ in, Cx<R> *__restrict__ Y,
                                                Col4Geom cg, FftDesc fd1, const Cx<R> *__restrict__ tw1,
                                                const Cx<R> *__restrict__ twn) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int panel = blockIdx.x / cg.n2;
    const int t = blockIdx.x - panel * cg.n2;
    const int p = blockIdx.y;
    const int kk = min(kPanel, cg.ncols - panel * kPanel);
    const C *src = in + p * cg.in_plane + (int64_t)panel * cg.rows_in * kPanel;
    C *dst = Y + p * cg.y_plane + ((int64_t)panel * cg.n + t) * kPanel;
    const int64_t rstride = (int64_t)cg.n2 * kPanel;
    lds_fft<false, false, DIR, NTH, false, CAP>(
        buf, kPanel, fd1, tw1,
        [&](int s, int col) {
            const int a = cg.n2 * s + t;
            int row = a;
            if constexpr (PRUNED) {
                row = -1;
                if (a < cg.rows_in - cg.h) row = a + cg.h;
                else if (a >= cg.n - cg.h) row = a - (cg.n - cg.h);
            }
            return (row >= 0 && col < kk) ? src[(int64_t)row * kPanel + col] : cmake<C>((R)0, (R)0);
        },
        [&](int r, int col, C v, int) {
            const C w = twn[r * t];   // exp(-2 pi i r t / N); r t < N
            dst[(int64_t)r * rstride + col] = DIR < 0 ? cmul(v, w) : cmulconj(v, w);
        });
}

// Pass B, degridding: block (panel * n1 + r, plane); the n2-point
// transforms over t of Y[p][panel][r][.][.] give the grid rows a = r + n1 q of
// the panel's columns, G[p][a][b].
template <typename R, int NTH, int CAP>
__global__ __launch_bounds__(NTH) void k_col4_b_degrid(const Cx<R> *__restrict__ Y, Cx<R> *__restrict__ G,
                                                       Col4Geom cg, int nv, FftDesc fd2,
                                                       const Cx<R> *__restrict__ tw2) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int panel = blockIdx.x / cg.n1;
    const int r = blockIdx.x - panel * cg.n1;
    const int p = blockIdx.y;
    const int b0 = panel * kPanel;
    const int kk = min(kPanel, cg.ncols - b0);
    const C *src = Y + p * cg.y_plane + ((int64_t)panel * cg.n + (int64_t)r * cg.n2) * kPanel;
    C *dst = G + (int64_t)p * cg.n * nv + b0;
    lds_fft<false, false, -1, NTH, false, CAP>(
        buf, kPanel, fd2, tw2, [&](int t, int col) { return src[t * kPanel + col]; },
        [&](int q, int col, C v, int) {
            if (col < kk) dst[(int64_t)(r + cg.n1 * q) * nv + col] = v;
        });
}

// Pass B, gridding: block (panel * n1 + r) over all planes of the batch; the
// n2-point transforms over t give grid rows a = r + n1 q; the retained ones
// (image row pp, a = (pp - h) mod N) are multiplied by the conjugate w-screen
// (eq. Rad1, phase reduced in FP64), their real parts summed over the planes
// in registers and added to the image accumulator once.  Each (pp, column)
// belongs to one block.
template <typename R, int NTH, int CAP>
__global__ __launch_bounds__(NTH) void k_col4_b_grid(const Cx<R> *__restrict__ Y, R *__restrict__ acc,
                                                     const double *__restrict__ nm1, PassGeom pg, Col4Geom cg,
                                                     int j_lo, int np, FftDesc fd2,
                                                     const Cx<R> *__restrict__ tw2) {
    using C = Cx<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int panel = blockIdx.x / cg.n1;
    const int r = blockIdx.x - panel * cg.n1;
    const int q0 = panel * kPanel;
    const int kk = min(kPanel, pg.npix_y - q0);
    const int h = pg.npix_x / 2;
    // output e = tid + i NTH of the block: q = e / 16, column e % 16; its
    // image pixel (flat index, -1 when not retained)
    auto pixel = [&](int i) -> int {
        const int e = threadIdx.x + i * NTH;
        const int q = e >> 4, col = e & (kPanel - 1);
        const int a = r + cg.n1 * q;
        int pp = -1;
        if (e < cg.n2 * kPanel && col < kk) {
            if (a < pg.npix_x - h) pp = a + h;
            else if (a >= cg.n - h) pp = a - (cg.n - h);
        }
        return pp >= 0 ? pp * pg.npix_y + q0 + col : -1;   // npix_x npix_y < 2^31
    };
    double nmv[CAP];
    R sum[CAP];
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        const int px = pixel(i);
        nmv[i] = (px >= 0 && pg.do_w) ? nm1[px] : 0.0;
        sum[i] = (R)0;
    }
    for (int p = 0; p < np; ++p) {
        const C *src = Y + p * cg.y_plane + ((int64_t)panel * cg.n + (int64_t)r * cg.n2) * kPanel;
        const double cj = pg.w0 + (double)(j_lo + p) * pg.dw;
        // an opaque copy of the column count per plane: otherwise every FFT
        // address is hoisted out of the plane loop and held in registers
        int Kp = __builtin_amdgcn_readfirstlane(kPanel);
        asm volatile("" : "+s"(Kp));
        lds_fft<false, true, +1, NTH, false, CAP>(
            buf, Kp, fd2, tw2, [&](int t, int col) { return src[t * kPanel + col]; }, NoIo{});
#pragma unroll
        for (int i = 0; i < CAP; ++i) {
            if (pixel(i) >= 0) {
                const int e = threadIdx.x + i * NTH;
                const C hv = buf[(fft_lidx(e >> 4) << 4) + (e & (kPanel - 1))];
                if (pg.do_w) {
                    double ph = cj * nmv[i];
                    ph -= rint(ph);
                    R sn, cs;
                    if constexpr (sizeof(R) == 4) sincos_turns_f32(ph, sn, cs);
                    else sincospi(2.0 * ph, &sn, &cs);
                    sum[i] += hv.x * cs + hv.y * sn;   // Re(h * exp(-2 pi i ph))
                } else {
                    sum[i] += hv.x;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < CAP; ++i) {
        const int px = pixel(i);
        if (px >= 0) acc[px] += sum[i];
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
__global__ void k_degrid_finish(const Cx<R> *__restrict__ visacc, const uint32_t *__restrict__ inv,
                                const R *__restrict__ wgt, int64_t n_total, Cx<R> *__restrict__ vis) {
    // caller's order out: the writes stay contiguous and the scattered side
    // is the read (a scattered 8-byte write costs a read-modify-write of a
    // whole memory sector)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = inv[i];
        if (e == 0xffffffffu) continue;                    // masked
        Cx<R> v = visacc[e & 0x7fffffffu];
        if (e >> 31) v.y = -v.y;                            // folded: conjugate
        if (wgt) v = cscale(v, wgt[i]);
        vis[i] = v;
    }
}

// Gridding input in sorted order: weighted, and conjugated where folded.
template <typename R>
__global__ void k_gather_vis(const Cx<R> *__restrict__ vis, const R *__restrict__ wgt,
                             const uint32_t *__restrict__ inv, int64_t n_total, Cx<R> *__restrict__ vsorted) {
    // caller's order in, sorted order out: the reads stay contiguous and the
    // scattered side is the write (cheaper than a scattered read)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = inv[i];
        if (e == 0xffffffffu) continue;                    // masked
        Cx<R> v = vis[i];
        if (wgt) v = cscale(v, wgt[i]);
        if (e >> 31) v.y = -v.y;                            // folded: conjugate
        vsorted[e & 0x7fffffffu] = v;
    }
}

template <typename R>
__global__ void k_zero_masked(const uint8_t *__restrict__ mask, int64_t n, Cx<R> *__restrict__ vis) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        if (!mask[e]) vis[e] = Cx<R>{};
}

}  // namespace wg
