// Plan-time kernels: w range, visibility binning keys (Sect. 4.3), stable
// LSD radix sort, per-(tile, batch) range tables, correction factors.
#pragma once
#include "device_common.hpp"

namespace wg {

// ---- w range and active count over selected visibilities -----------------
// |w| after the fold is non-negative, so its IEEE bit pattern orders like an
// unsigned integer and integer atomics give exact min/max.
__global__ void k_wrange(const double *__restrict__ uvw, const double *__restrict__ scale,
                         const uint8_t *__restrict__ mask, int64_t n_rows, int64_t n_chan,
                         int do_w, unsigned long long *out /* [0]=min bits, [1]=max bits, [2]=count */) {
    unsigned long long mn = ~0ull, mx = 0ull, cnt = 0ull;
    const int64_t n = n_rows * n_chan;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (mask && !mask[k]) continue;
        ++cnt;
        if (do_w) {
            int64_t r = k / n_chan;
            int64_t c = k - r * n_chan;
            double w = fabs(uvw[3 * r + 2] * scale[c]);
            unsigned long long b = (unsigned long long)__double_as_longlong(w);
            mn = b < mn ? b : mn;
            mx = b > mx ? b : mx;
        }
    }
    // wave reduction then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long omn = __shfl_down(mn, off, 64);
        unsigned long long omx = __shfl_down(mx, off, 64);
        unsigned long long oc = __shfl_down(cnt, off, 64);
        mn = omn < mn ? omn : mn;
        mx = omx > mx ? omx : mx;
        cnt += oc;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&out[0], mn);
        atomicMax(&out[1], mx);
        atomicAdd(&out[2], cnt);
    }
}

__global__ void k_wrange_init(unsigned long long *out) {
    if (threadIdx.x == 0) {
        out[0] = ~0ull;
        out[1] = 0ull;
        out[2] = 0ull;
    }
}

// ---- binning keys: ((t_u * NTv + t_v) * N_w + t_w), masked -> sentinel ----
__global__ void k_keys(const double *__restrict__ uvw, const double *__restrict__ scale,
                       const uint8_t *__restrict__ mask, int64_t n_rows, Geom g,
                       unsigned long long sentinel, unsigned long long *__restrict__ keys,
                       uint32_t *__restrict__ vals) {
    const int64_t n = n_rows * g.n_chan;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long key = sentinel;
        if (!mask || mask[k]) {
            int64_t r = k / g.n_chan;
            int64_t c = k - r * g.n_chan;
            VisCoord vc = vis_coord(uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], scale[c], g);
            unsigned long long tile = (unsigned long long)(vc.iu >> 4) * (unsigned long long)g.ntv +
                                      (unsigned long long)(vc.iv >> 4);
            key = tile * (unsigned long long)g.nw + (unsigned long long)vc.iw;
        }
        keys[k] = key;
        vals[k] = (uint32_t)k;
    }
}

// ---- stable LSD radix sort, 8-bit digits ----------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const unsigned long long *__restrict__ keys,
                                                        int64_t n, int shift, uint32_t *__restrict__ hist,
                                                        int nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int i = 0; i < kRsItems; ++i) {
        int64_t idx = base + i * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of a uint32 array in tiles of 4096; writes each tile's total.
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4 * kScanThreads;

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *__restrict__ data, int64_t n,
                                                             uint32_t *__restrict__ tile_sums) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    uint32_t v[4];
    uint32_t tsum = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < n) ? data[base + i] : 0u;
        tsum += v[i];
    }
    // inclusive scan of per-thread sums within the wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = tsum;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t s = threadIdx.x < kScanThreads / 64 ? wsum[threadIdx.x] : 0u;
        uint32_t t = s;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(t, off, 64);
            if ((int)threadIdx.x >= off) t += y;
        }
        if (threadIdx.x < kScanThreads / 64) wsum[threadIdx.x] = t - s;   // exclusive
    }
    __syncthreads();
    uint32_t run = wsum[wave] + x - tsum;   // exclusive prefix of this thread
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = wsum[wave] + x;
}

__global__ void k_scan_add(uint32_t *__restrict__ data, int64_t n, const uint32_t *__restrict__ tile_offs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) data[i] += tile_offs[i / kScanTile];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const unsigned long long *__restrict__ kin, const uint32_t *__restrict__ vin,
    unsigned long long *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int nblocks) {
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kRsThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_off[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    running[tid] = 0;
    for (int w = 0; w < kRsThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int i = 0; i < kRsItems; ++i) {
        int64_t idx = (int64_t)blockIdx.x * kRsTile + i * kRsThreads + tid;
        bool valid = idx < n;
        unsigned long long key = valid ? kin[idx] : 0ull;
        uint32_t val = valid ? vin[idx] : 0u;
        uint32_t digit = (uint32_t)((key >> shift) & 255u);
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (digit >> b) & 1u;
            unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = running[digit] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
            uint32_t dst = base_off[digit] + pos;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kRsThreads / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        running[tid] += add;
        __syncthreads();
    }
}

// ---- per-(tile, batch) range tables ----------------------------------------
// Entry e = tile * (NJ + 1) + J holds the first sorted position whose key is
// >= tile * N_w + clamp(J * P - shift, 0, N_w).  With shift = 0 the entry at
// J starts batch J; with shift = alpha - 1 it starts the visibilities whose
// alpha planes reach into batch J.  Each sorted position fills the entries
// whose thresholds lie in (key[s-1], key[s]].
__device__ __forceinline__ unsigned long long tab_count(unsigned long long key, int nw, int P, int NJ,
                                                        int shift) {
    unsigned long long tile = key / (unsigned long long)nw;
    int w = (int)(key - tile * (unsigned long long)nw);
    int j = (w + shift) / P;
    if (j > NJ) j = NJ;
    return tile * (unsigned long long)(NJ + 1) + (unsigned long long)(j + 1);
}

__global__ void k_fill_tab(const unsigned long long *__restrict__ keys, int64_t n_active, int nw, int P,
                           int NJ, int shift, unsigned long long total, uint32_t *__restrict__ tab) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s <= n_active;
         s += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long lo = s == 0 ? 0ull : tab_count(keys[s - 1], nw, P, NJ, shift);
        unsigned long long hi = s == n_active ? total : tab_count(keys[s], nw, P, NJ, shift);
        for (unsigned long long e = lo; e < hi; ++e) tab[e] = (uint32_t)s;
    }
}

// ---- work items -------------------------------------------------------------
// In batch J the gridder of tile t takes, from the gridder stream, the
// visibilities of bin t and those of the bins up/left whose footprints reach
// t (grid_seg_bin).  A list longer than `cap` is dealt as ceil(len/cap)
// items: the first is implied by the launch (one block per tile), the others
// are listed here.  Run twice: emit = 0 counts the extra items per batch into
// cur_*, emit = 1 (cursors cleared, off_* = per-batch list offsets) writes
// them.  Gridder extras get consecutive partial-tile slots (numbered per
// batch), recorded in `red` as (tile, first slot, slots) for the reduction;
// the list order depends on the atomics, the slot order within a tile does
// not.
__device__ __forceinline__ uint32_t bin_len(const uint32_t *__restrict__ tab_lo, const uint32_t *__restrict__ tab_hi,
                                            int64_t bin, int NJ, int J) {
    const uint32_t s0 = tab_lo[bin * (NJ + 1) + J];
    const uint32_t s1 = tab_hi[bin * (NJ + 1) + J + 1];
    return s1 > s0 ? s1 - s0 : 0u;
}

__global__ void k_items(const uint32_t *__restrict__ tab2_lo, const uint32_t *__restrict__ tab2_hi, int ntu,
                        int ntv, int NJ, uint32_t cap_g, int emit, uint32_t *__restrict__ cur_g,
                        uint32_t *__restrict__ cur_r, const uint32_t *__restrict__ off_g,
                        const uint32_t *__restrict__ off_r, int4 *__restrict__ items_g, int4 *__restrict__ red) {
    const int64_t nt = (int64_t)ntu * ntv;
    const int64_t n = nt * NJ;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int J = (int)(e / nt);
        const int t = (int)(e - (int64_t)J * nt);
        const int A = t / ntv, B = t - (t / ntv) * ntv;
        uint32_t cg = 0;
        for (int sg = 0; sg < kGridSegs; ++sg) cg += bin_len(tab2_lo, tab2_hi, grid_seg_bin(sg, A, B, ntu, ntv), NJ, J);
        const uint32_t eg = cg > cap_g ? (cg - 1) / cap_g : 0u;
        if (!eg) continue;
        if (!emit) {
            atomicAdd(&cur_g[J], eg);
            atomicAdd(&cur_r[J], 1u);
            continue;
        }
        const uint32_t b = atomicAdd(&cur_g[J], eg);
        for (uint32_t k = 1; k <= eg; ++k) {
            const uint32_t first = k * cap_g;
            items_g[off_g[J] + b + k - 1] = make_int4(t, (int)first, (int)min(cap_g, cg - first), (int)(b + k - 1));
        }
        const uint32_t r = atomicAdd(&cur_r[J], 1u);
        red[off_r[J] + r] = make_int4(t, (int)b, (int)eg, 0);
    }
}

// ---- gridder stream in edge-class order ------------------------------------
// The gridder of tile (A, B) takes its own bin and, from the bins up/left of
// it, only the visibilities whose footprints reach into it.  A visibility
// anchored at tile-relative first cell (la, lb) reaches the next tile down
// when la + alpha - 1 >= 16 and the next tile right when lb + alpha - 1 >= 16.
// Rank within a tile: 0 interior, 1 right only, 2 both, 3 down only, so that
// the ranks a neighbour needs ({1, 2} from the left, {2, 3} from above, {2}
// diagonally) are contiguous.
__device__ __forceinline__ int edge_rank(int2 an, int alpha) {
    const int la = (an.x & 0xffff) & 15, lb = ((an.x >> 16) & 0xffff) & 15;
    const bool down = la + alpha - 1 >= 16, right = lb + alpha - 1 >= 16;
    return down ? (right ? 2 : 3) : (right ? 1 : 0);
}

// Keys of the gridder stream for the sorted positions s of the index:
// ((tile * 4 + rank) * N_w + first plane); values s.  A stable sort of these
// keeps the index order within each (tile, rank, plane).
__global__ void k_class_keys(const unsigned long long *__restrict__ keys, const int2 *__restrict__ anc,
                             int64_t n_active, int nw, int alpha, unsigned long long *__restrict__ keys2,
                             uint32_t *__restrict__ vals2) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_active;
         s += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = keys[s];
        const unsigned long long tile = k / (unsigned long long)nw;
        const unsigned long long iw = k - tile * (unsigned long long)nw;
        const int rank = edge_rank(anc[s], alpha);
        keys2[s] = (tile * 4ull + (unsigned long long)rank) * (unsigned long long)nw + iw;
        vals2[s] = (uint32_t)s;
    }
}

// The gridder stream: coordinates and anchors in class order, and the map
// from the caller's order to class-order positions (fold bit on top, all
// ones for masked visibilities, filled beforehand).
template <typename R>
__global__ void k_class_stream(const uint32_t *__restrict__ perm2, const uint32_t *__restrict__ order,
                               const R *__restrict__ z, const int2 *__restrict__ anc, int64_t n_active,
                               R *__restrict__ z2, int2 *__restrict__ anc2, uint32_t *__restrict__ inv2) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_active;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = perm2[t];
        z2[3 * t] = z[3 * (int64_t)s];
        z2[3 * t + 1] = z[3 * (int64_t)s + 1];
        z2[3 * t + 2] = z[3 * (int64_t)s + 2];
        const int2 a = anc[s];
        anc2[t] = a;
        inv2[order[s]] = (uint32_t)t | (a.y < 0 ? 0x80000000u : 0u);
    }
}

// ---- degridder work items -------------------------------------------------
// The degridder takes the visibilities of one bin (index order).  A run
// longer than `cap` is dealt as ceil(len/cap) items; the first is implied by
// the launch (one block per tile), the others are listed as (tile, first
// position, count, 0).  Run twice like k_items: emit = 0 counts, emit = 1
// writes at per-batch offsets off.
__global__ void k_items_deg(const uint32_t *__restrict__ tab_lo, const uint32_t *__restrict__ tab_hi, int ntu,
                            int ntv, int NJ, uint32_t cap, int emit, uint32_t *__restrict__ cur,
                            const uint32_t *__restrict__ off, int4 *__restrict__ items) {
    const int64_t nt = (int64_t)ntu * ntv;
    const int64_t n = nt * NJ;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int J = (int)(e / nt);
        const int t = (int)(e - (int64_t)J * nt);
        const uint32_t len = bin_len(tab_lo, tab_hi, t, NJ, J);
        const uint32_t ex = len > cap ? (len - 1) / cap : 0u;
        if (!ex) continue;
        const uint32_t b = atomicAdd(&cur[J], ex);
        if (!emit) continue;
        const uint32_t s0 = tab_lo[(int64_t)t * (NJ + 1) + J];
        for (uint32_t k = 1; k <= ex; ++k) {
            const uint32_t first = k * cap;
            items[off[J] + b + k - 1] = make_int4(t, (int)(s0 + first), (int)min(cap, len - first), 0);
        }
    }
}

// order2[stream position] = caller's linear index, from the caller-order map
__global__ void k_stream_order(const uint32_t *__restrict__ inv2, int64_t n_total, uint32_t *__restrict__ order2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t e = inv2[i];
        if (e != 0xffffffffu) order2[e & 0x7fffffffu] = (uint32_t)i;
    }
}

// ---- inverse permutation ----------------------------------------------------
// inv[r * n_chan + c] = sorted position | fold << 31 for selected
// visibilities, ~0 for masked ones (filled beforehand), so that gridding can
// read its input in the caller's order and scatter it to sorted order.
__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t value) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = value;
}

__global__ void k_inv_order(const uint32_t *__restrict__ order, const int2 *__restrict__ anc, int64_t n_active,
                            uint32_t *__restrict__ inv) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_active;
         s += (int64_t)gridDim.x * blockDim.x)
        inv[order[s]] = (uint32_t)s | (anc[s].y < 0 ? 0x80000000u : 0u);
}

// ---- per sorted visibility: kernel-local coordinates and anchors ------------
// z = 2 (first cell - coordinate + alpha/2) - 1 in [-1, 1) for u, v and w
// (the shared local variable of the alpha polynomial pieces), anchors packed
// as anc.x = i_u | i_v << 16, anc.y = i_w | fold << 31.
template <typename R>
__global__ void k_vis_prep(const double *__restrict__ uvw, const double *__restrict__ scale,
                           const uint32_t *__restrict__ order, int64_t n_active, Geom g, R *__restrict__ z,
                           int2 *__restrict__ anc) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n_active;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = order[s];
        const int64_t r = idx / g.n_chan;
        const int64_t c = idx - r * g.n_chan;
        const VisCoord vc = vis_coord(uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], scale[c], g);
        z[3 * s] = (R)(2.0 * (vc.ou + g.half) - 1.0);
        z[3 * s + 1] = (R)(2.0 * (vc.ov + g.half) - 1.0);
        z[3 * s + 2] = (R)(g.do_w ? 2.0 * (vc.ow + g.half) - 1.0 : 0.0);
        anc[s] = make_int2(vc.iu | (vc.iv << 16), vc.iw | (vc.flip ? (int)0x80000000u : 0));
    }
}

// ---- n - 1 and the correction 1 / (n Psi) per pixel ------------------------
// Psi = psi(p'/N_u) psi(q'/N_v) psi((n-1) dw) (Sect. 2), psi by quadrature with
// precomputed nodes t_i and weights wphi_i = w_i phi(t_i) on [0, alpha/2].
__global__ void k_corr(int npix_x, int npix_y, double pixsize_x, double pixsize_y, int do_w, double dw,
                       const double *__restrict__ psix, const double *__restrict__ psiy,
                       const double *__restrict__ qt, const double *__restrict__ qw, int nq,
                       double *__restrict__ nm1_out, double *__restrict__ corr_out) {
    const int64_t npix = (int64_t)npix_x * npix_y;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npix;
         e += (int64_t)gridDim.x * blockDim.x) {
        int p = (int)(e / npix_y), q = (int)(e - (int64_t)p * npix_y);
        double l = (double)(p - npix_x / 2) * pixsize_x;
        double m = (double)(q - npix_y / 2) * pixsize_y;
        double rho = l * l + m * m;
        double n = sqrt(1.0 - rho);
        double nm1 = -rho / (1.0 + n);
        double psi = psix[p] * psiy[q];
        if (do_w) {
            double k = nm1 * dw;
            double acc = 0.0;
            for (int i = nq - 1; i >= 0; --i) acc += qw[i] * cos(kTwoPi * k * qt[i]);
            psi *= 2.0 * acc;
        }
        nm1_out[e] = nm1;
        corr_out[e] = 1.0 / (n * psi);
    }
}

}  // namespace wg
