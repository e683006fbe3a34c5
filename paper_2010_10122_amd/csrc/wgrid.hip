// wgrid: C-ABI implementation (plan construction and the two apply calls).
// See include/wgrid.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/wgrid.h"
#include "host_math.hpp"
#include "kernels_apply.hpp"
#include "kernels_index.hpp"
#include "plan_internal.hpp"
#include "vis_launch.hpp"

using namespace wg;

namespace {

thread_local std::string g_last_hip;

bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    g_last_hip = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

#define HIP_TRY(call)                                   \
    do {                                                \
        if (!hip_ok((call), #call)) return WG_EHIP;     \
    } while (0)

#define LAUNCH_CHECK(what)                                              \
    do {                                                                \
        if (!hip_ok(hipGetLastError(), what)) return WG_EHIP;           \
    } while (0)

// Device allocations of one plan, through the caller's allocator if given.
// Optional per-kernel timing: while a profiler is attached to the calling
// host thread, every launch of the apply pipeline is bracketed by a pair of
// HIP events on the launch stream.  Events come from a pool and are read
// (synchronising on them) only by wg_profiler_read.
}  // namespace

struct wg_profiler {
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[WG_KIND_COUNT] = {};
    int64_t launches[WG_KIND_COUNT] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // timing only: no system-scope fence at the event (that fence writes
        // back and invalidates the caches at every kernel boundary, which
        // both slows the next kernel and adds to the measured interval)
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
    void drain() {
        for (Rec &r : pending) {
            float ms = 0.f;
            if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                total_ms[r.kind] += ms;
                launches[r.kind] += 1;
            } else {
                (void)hipGetLastError();
            }
            if (r.a) pool.push_back(r.a);
            if (r.b) pool.push_back(r.b);
        }
        pending.clear();
    }
};

namespace {

thread_local wg_profiler *g_prof = nullptr;

// Scope guard recording one launch of `kind` on `st` when profiling.
struct ProfScope {
    wg_profiler *p;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    ProfScope(int k, hipStream_t s) : p(g_prof), kind(k), st(s) {
        if (p) {
            a = p->get();
            b = p->get();
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (p) {
            if (b) (void)hipEventRecord(b, st);
            p->pending.push_back({kind, a, b});
        }
    }
};

int64_t grid_blocks(int64_t n, int threads, int64_t cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    return std::max<int64_t>(1, std::min(b, cap));
}

// Radices of the passes: greedy over the register DFTs, largest first, so
// that few passes (LDS exchanges) remain; the largest radix goes last (its
// outputs are stored straight to the destination).
void make_fft_desc(int n, FftDesc &d) {
    d.n = n;
    d.npass = 0;
    int m = n;
    while (m > 1 && d.npass < kFftMaxPass) {
        int pick = 0;
        for (int r : {16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2})
            if (m % r == 0) {
                pick = r;
                break;
            }
        if (!pick) break;
        d.radix[d.npass++] = pick;
        m /= pick;
    }
    std::reverse(d.radix, d.radix + d.npass);
}

// the length a descriptor transforms (its radices' product)
int fft_desc_len(const FftDesc &d) {
    int n = 1;
    for (int s = 0; s < d.npass; ++s) n *= d.radix[s];
    return n;
}

// exp(-2 pi i t / N) with the angle folded into [0, pi/4] so that the library
// sin/cos see a small, exactly scaled argument.
void twiddles(int n, std::vector<double> &re, std::vector<double> &im) {
    re.resize(n);
    im.resize(n);
    for (int t = 0; t < n; ++t) {
        // angle fraction f = t/n of a full turn; use octant symmetry on 8t vs n
        long long k8 = 8LL * t;
        int oct = (int)(k8 / n);            // 0..7
        long long rem = k8 - (long long)oct * n;   // in [0, n)
        // angle inside the octant, in [0, pi/4)
        double a = (M_PI / 4.0) * (double)rem / (double)n;
        double c = std::cos(a), s = std::sin(a);
        double cr, sr;   // cos and sin of (oct * pi/4 + a)
        const double r2 = 0.70710678118654752440;
        switch (oct) {
            case 0: cr = c; sr = s; break;
            case 1: cr = r2 * (c - s); sr = r2 * (c + s); break;
            case 2: cr = -s; sr = c; break;
            case 3: cr = -r2 * (c + s); sr = r2 * (c - s); break;
            case 4: cr = -c; sr = -s; break;
            case 5: cr = -r2 * (c - s); sr = -r2 * (c + s); break;
            case 6: cr = s; sr = -c; break;
            default: cr = r2 * (c + s); sr = -r2 * (c - s); break;
        }
        re[t] = cr;
        im[t] = -sr;
    }
}

}  // namespace


namespace {


template <typename R> int build_plan_tables(wg_plan *p, const std::vector<double> &coefd,
                                            const std::vector<double> &twu_re, const std::vector<double> &twu_im,
                                            const std::vector<double> &twv_re, const std::vector<double> &twv_im) {
    using C = Cx<R>;
    std::vector<R> cr(coefd.size());
    for (size_t i = 0; i < coefd.size(); ++i) cr[i] = (R)coefd[i];
    const hipStream_t st = p->stream;
    p->coef = p->mem.get(cr.size() * sizeof(R));
    if (!p->coef) return WG_ENOMEM;
    HIP_TRY(hipMemcpyAsync(p->coef, cr.data(), cr.size() * sizeof(R), hipMemcpyHostToDevice, st));
    std::vector<C> tu(twu_re.size()), tv(twv_re.size());
    for (size_t i = 0; i < tu.size(); ++i) { tu[i].x = (R)twu_re[i]; tu[i].y = (R)twu_im[i]; }
    for (size_t i = 0; i < tv.size(); ++i) { tv[i].x = (R)twv_re[i]; tv[i].y = (R)twv_im[i]; }
    p->tw_u = p->mem.get(tu.size() * sizeof(C));
    p->tw_v = p->mem.get(tv.size() * sizeof(C));
    if (!p->tw_u || !p->tw_v) return WG_ENOMEM;
    HIP_TRY(hipMemcpyAsync(p->tw_u, tu.data(), tu.size() * sizeof(C), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->tw_v, tv.data(), tv.size() * sizeof(C), hipMemcpyHostToDevice, st));
    // four-step sub-lengths: exp(-2 pi i t / n_k) = exp(-2 pi i (t N / n_k) / N),
    // the same values as the length-N table
    std::vector<C> t1, t2;
    if (p->col4) {
        t1.resize(p->n1);
        t2.resize(p->n2);
        for (int t = 0; t < p->n1; ++t) t1[t] = tu[(size_t)t * p->n2];
        for (int t = 0; t < p->n2; ++t) t2[t] = tu[(size_t)t * p->n1];
        p->tw_n1 = p->mem.get(t1.size() * sizeof(C));
        p->tw_n2 = p->mem.get(t2.size() * sizeof(C));
        if (!p->tw_n1 || !p->tw_n2) return WG_ENOMEM;
        HIP_TRY(hipMemcpyAsync(p->tw_n1, t1.data(), t1.size() * sizeof(C), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(p->tw_n2, t2.data(), t2.size() * sizeof(C), hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));   // the host vectors must outlive the copies
    return WG_OK;
}

// Stable LSD radix sort of (keys, vals) on the low `bits` bits.
// The sorted result is left in (keys, vals); scratch is released before return.
int radix_sort(wg_plan *p, unsigned long long *const keys_io, uint32_t *const vals_io, int64_t n, int bits,
               hipStream_t st) {
    if (n <= 1) return WG_OK;
    unsigned long long *keys = keys_io;
    uint32_t *vals = vals_io;
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    const int64_t hist_n = 256LL * nblocks;
    unsigned long long *k2 = (unsigned long long *)p->mem.get(n * sizeof(unsigned long long));
    uint32_t *v2 = (uint32_t *)p->mem.get(n * sizeof(uint32_t));
    uint32_t *hist = (uint32_t *)p->mem.get(hist_n * sizeof(uint32_t));
    // scan scratch: one level of tile sums per recursion level
    std::vector<int64_t> lens;
    std::vector<uint32_t *> levels;
    int64_t len = hist_n;
    bool ok = k2 && v2 && hist;
    while (ok && len > 1) {
        int64_t nt = (len + kScanTile - 1) / kScanTile;
        uint32_t *buf = (uint32_t *)p->mem.get(std::max<int64_t>(nt, 1) * sizeof(uint32_t));
        if (!buf) { ok = false; break; }
        levels.push_back(buf);
        lens.push_back(len);
        len = nt;
        if (nt == 1) break;
    }
    int rc = ok ? WG_OK : WG_ENOMEM;
    for (int shift = 0; rc == WG_OK && shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kRsThreads), 0, st, keys, n, shift, hist, nblocks);
        // multi-level exclusive scan of hist
        uint32_t *data = hist;
        for (size_t lv = 0; lv < levels.size(); ++lv) {
            int64_t ln = lens[lv];
            int64_t nt = (ln + kScanTile - 1) / kScanTile;
            hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kScanThreads), 0, st, data, ln, levels[lv]);
            data = levels[lv];
        }
        for (size_t lv = levels.size(); lv-- > 0;) {
            uint32_t *below = lv == 0 ? hist : levels[lv - 1];
            int64_t ln = lens[lv];
            if ((ln + kScanTile - 1) / kScanTile > 1)
                hipLaunchKernelGGL(k_scan_add, dim3((unsigned)grid_blocks(ln, 256, 1LL << 30)), dim3(256), 0, st,
                                   below, ln, levels[lv]);
        }
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, st, keys, vals, k2, v2, n, shift,
                           hist, nblocks);
        if (!hip_ok(hipGetLastError(), "radix sort")) rc = WG_EHIP;
        std::swap(keys, k2);
        std::swap(vals, v2);
    }
    if (rc == WG_OK && keys != keys_io) {   // odd pass count: copy back
        if (!hip_ok(hipMemcpyAsync(keys_io, keys, n * sizeof(unsigned long long), hipMemcpyDeviceToDevice, st),
                    "radix sort copy") ||
            !hip_ok(hipMemcpyAsync(vals_io, vals, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st),
                    "radix sort copy"))
            rc = WG_EHIP;
        std::swap(keys, k2);
        std::swap(vals, v2);
    }
    if (rc == WG_OK && !hip_ok(hipStreamSynchronize(st), "radix sort sync")) rc = WG_EHIP;
    p->mem.put(k2 == keys_io ? keys : k2);
    p->mem.put(v2 == vals_io ? vals : v2);
    p->mem.put(hist);
    for (uint32_t *b : levels) p->mem.put(b);
    return rc;
}

// Gridder stream (see k_class_keys): keys (tile * 4 + edge rank) * N_w +
// first plane of the sorted positions, stably sorted; range tables per
// (tile, rank, batch); coordinates, anchors and the caller-order map in the
// new order.  Needs the index (keys, order, tables), zc and anc.
int build_class_stream(wg_plan *p, hipStream_t st, int bits) {
    const Geom &g = p->g;
    const int64_t nact = std::max<int64_t>(p->n_active, 1);
    const size_t sr = p->precision == WG_F32 ? 4 : 8;
    const unsigned long long tab2_n = (unsigned long long)g.ntu * g.ntv * 4ull * (unsigned long long)(p->NJ + 1);
    p->tab2_lo = (uint32_t *)p->mem.get(tab2_n * sizeof(uint32_t));
    p->tab2_hi = (uint32_t *)p->mem.get(tab2_n * sizeof(uint32_t));
    p->zc2 = p->mem.get(nact * 3 * sr);
    p->anc2 = (int2 *)p->mem.get(nact * sizeof(int2));
    p->inv2 = (uint32_t *)p->mem.get(std::max<int64_t>(p->n_total, 1) * sizeof(uint32_t));
    unsigned long long *keys2 = (unsigned long long *)p->mem.get(nact * sizeof(unsigned long long));
    uint32_t *perm2 = (uint32_t *)p->mem.get(nact * sizeof(uint32_t));
    if (!p->tab2_lo || !p->tab2_hi || !p->zc2 || !p->anc2 || !p->inv2 || !keys2 || !perm2) return WG_ENOMEM;
    const unsigned grid = (unsigned)grid_blocks(p->n_active, 256, 1 << 20);
    if (p->n_total > 0)
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 20)), dim3(256), 0, st,
                           p->inv2, p->n_total, 0xffffffffu);
    int rc = WG_OK;
    if (p->n_active > 0) {
        hipLaunchKernelGGL(k_class_keys, dim3(grid), dim3(256), 0, st, p->keys, p->anc, p->n_active, g.nw, g.alpha,
                           keys2, perm2);
        LAUNCH_CHECK("k_class_keys");
        rc = radix_sort(p, keys2, perm2, p->n_active, bits + 2, st);
        if (rc != WG_OK) return rc;
        if (p->precision == WG_F32)
            hipLaunchKernelGGL(k_class_stream<float>, dim3(grid), dim3(256), 0, st, perm2, p->order,
                               (const float *)p->zc, p->anc, p->n_active, (float *)p->zc2, p->anc2, p->inv2);
        else
            hipLaunchKernelGGL(k_class_stream<double>, dim3(grid), dim3(256), 0, st, perm2, p->order,
                               (const double *)p->zc, p->anc, p->n_active, (double *)p->zc2, p->anc2, p->inv2);
        LAUNCH_CHECK("k_class_stream");
    }
    hipLaunchKernelGGL(k_fill_tab, dim3((unsigned)grid_blocks(p->n_active + 1, 256, 1 << 20)), dim3(256), 0, st,
                       keys2, p->n_active, g.nw, p->P, p->NJ, p->alpha - 1, tab2_n, p->tab2_lo);
    hipLaunchKernelGGL(k_fill_tab, dim3((unsigned)grid_blocks(p->n_active + 1, 256, 1 << 20)), dim3(256), 0, st,
                       keys2, p->n_active, g.nw, p->P, p->NJ, 0, tab2_n, p->tab2_hi);
    LAUNCH_CHECK("k_fill_tab (class)");
    HIP_TRY(hipStreamSynchronize(st));
    p->mem.put(keys2);
    p->mem.put(perm2);
    return rc;
}

// Extra work items of every batch (gridder: k_items over the gridder
// stream; degridder: k_items_deg over the index): count, lay out per batch,
// emit.  Leaves
// xg/xd/xr and their per-batch offsets in the plan.
int build_items(wg_plan *p, hipStream_t st) {
    const int NJ = p->NJ;
    const int64_t n = (int64_t)p->g.ntu * p->g.ntv * NJ;
    uint32_t *cur = (uint32_t *)p->mem.get((size_t)6 * NJ * sizeof(uint32_t));
    if (!cur) return WG_ENOMEM;
    uint32_t *cur_g = cur, *cur_d = cur + NJ, *cur_r = cur + 2 * NJ;
    uint32_t *doff = cur + 3 * NJ;
    const unsigned nb = (unsigned)grid_blocks(n, 256, 1 << 16);
    hipLaunchKernelGGL(k_fill_zero<uint32_t>, dim3((unsigned)grid_blocks(6 * NJ, 256, 1024)), dim3(256), 0, st, cur,
                       (int64_t)6 * NJ);
    hipLaunchKernelGGL(k_items, dim3(nb), dim3(256), 0, st, p->tab2_lo, p->tab2_hi, p->g.ntu, p->g.ntv, NJ,
                       (uint32_t)kGridItemCap, 0, cur_g, cur_r, nullptr, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_items_deg, dim3(nb), dim3(256), 0, st, p->tab_lo, p->tab_hi, p->g.ntu, p->g.ntv, NJ,
                       (uint32_t)kDegridItemCap, 0, cur_d, nullptr, nullptr);
    LAUNCH_CHECK("k_items");
    std::vector<uint32_t> cnt((size_t)3 * NJ);
    HIP_TRY(hipMemcpyAsync(cnt.data(), cur, cnt.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    p->xg_off.assign(NJ + 1, 0);
    p->xd_off.assign(NJ + 1, 0);
    p->xr_off.assign(NJ + 1, 0);
    p->max_slots = 0;
    for (int J = 0; J < NJ; ++J) {
        p->xg_off[J + 1] = p->xg_off[J] + cnt[J];
        p->xd_off[J + 1] = p->xd_off[J] + cnt[NJ + J];
        p->xr_off[J + 1] = p->xr_off[J] + cnt[2 * NJ + J];
        p->max_slots = std::max(p->max_slots, (int)cnt[J]);
    }
    const uint32_t ng = p->xg_off[NJ], nd = p->xd_off[NJ], nr = p->xr_off[NJ];
    p->xg = (int4 *)p->mem.get(std::max<size_t>(ng, 1) * sizeof(int4));
    p->xd = (int4 *)p->mem.get(std::max<size_t>(nd, 1) * sizeof(int4));
    p->xr = (int4 *)p->mem.get(std::max<size_t>(nr, 1) * sizeof(int4));
    if (!p->xg || !p->xd || !p->xr) return WG_ENOMEM;
    if (ng + nd > 0) {
        std::vector<uint32_t> offs((size_t)3 * NJ);
        for (int J = 0; J < NJ; ++J) {
            offs[J] = p->xg_off[J];
            offs[NJ + J] = p->xd_off[J];
            offs[2 * NJ + J] = p->xr_off[J];
        }
        HIP_TRY(hipMemcpyAsync(doff, offs.data(), offs.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_fill_zero<uint32_t>, dim3((unsigned)grid_blocks(3 * NJ, 256, 1024)), dim3(256), 0, st,
                           cur, (int64_t)3 * NJ);
        hipLaunchKernelGGL(k_items, dim3(nb), dim3(256), 0, st, p->tab2_lo, p->tab2_hi, p->g.ntu, p->g.ntv, NJ,
                           (uint32_t)kGridItemCap, 1, cur_g, cur_r, doff, doff + 2 * NJ, p->xg, p->xr);
        hipLaunchKernelGGL(k_items_deg, dim3(nb), dim3(256), 0, st, p->tab_lo, p->tab_hi, p->g.ntu, p->g.ntv, NJ,
                           (uint32_t)kDegridItemCap, 1, cur_d, doff + NJ, p->xd);
        if (!hip_ok(hipGetLastError(), "k_items")) return WG_EHIP;
        HIP_TRY(hipStreamSynchronize(st));   // the host offsets buffer must outlive the copy
    }
    p->mem.put(cur);
    p->index_bytes += (size_t)(std::max<uint32_t>(ng, 1) + std::max<uint32_t>(nd, 1) + std::max<uint32_t>(nr, 1)) *
                      sizeof(int4);
    return WG_OK;
}

int validate(const wg_plan_desc *d) {
    if (!d) return WG_EINVAL;
    if (d->n_rows < 0 || d->n_chan < 1) return WG_EINVAL;
    if ((d->n_rows > 0 && !d->uvw) || !d->freq) return WG_EINVAL;
    if ((unsigned long long)d->n_rows * (unsigned long long)d->n_chan >= (1ULL << 31)) return WG_EINVAL;
    if (d->npix_x < 32 || d->npix_y < 32 || (d->npix_x & 1) || (d->npix_y & 1)) return WG_EINVAL;
    if (!(d->pixsize_x > 0.0) || !(d->pixsize_y > 0.0)) return WG_EINVAL;
    if (d->precision != WG_F32 && d->precision != WG_F64) return WG_EINVAL;
    if (!(d->epsilon <= 0.1)) return WG_EINVAL;
    if (d->precision == WG_F32 && !(d->epsilon >= 1e-5)) return WG_EINVAL;
    if (d->precision == WG_F64 && !(d->epsilon > 2e-13)) return WG_EINVAL;
    if ((d->alloc == nullptr) != (d->free == nullptr)) return WG_EINVAL;
    if (d->alpha != 0 || d->sigma != 0.0) {
        if (!find_row(d->alpha, d->sigma)) return WG_EINVAL;
    }
    if (d->planes_per_batch < 0) return WG_EINVAL;
    double l = (double)(0 - d->npix_x / 2) * d->pixsize_x;
    double m = (double)(0 - d->npix_y / 2) * d->pixsize_y;
    if (!(l * l + m * m < 1.0)) return WG_EINVAL;
    return WG_OK;
}

// Workspace layout of one apply call (byte offsets into the caller's
// workspace) for a given number of partial-tile slots of the gridder.
size_t plan_layout(wg_plan *p, int64_t slots) {
    const Geom &g = p->g;
    const size_t sc = p->precision == WG_F32 ? 8 : 16;
    const size_t sr = sc / 2;
    const int64_t npix = (int64_t)g.npix_x * g.npix_y;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    p->off_G = off;
    off = align(off + (size_t)p->P * g.nu * g.nv * sc);
    p->off_G2 = off;                   // the second plane buffer of the pipeline
    off = align(off + (size_t)p->P * g.nu * g.nv * sc);
    p->off_T = off;
    off = align(off + (size_t)p->P * std::max(panel_elems(g.npix_y, g.nu), panel_elems(g.nv, g.npix_x)) * sc);
    p->off_Y = off;                    // the four-step intermediate
    if (p->col4)
        off = align(off + (size_t)p->P * std::max(panel_elems(g.nv, g.nu), panel_elems(g.npix_y, g.nu)) * sc);
    p->off_acc = off;
    off = align(off + (size_t)npix * sr);
    p->off_itil = off;
    off = align(off + (size_t)npix * sr);
    p->off_vacc = off;
    off = align(off + (size_t)std::max<int64_t>(p->n_active, 1) * sc);
    p->off_part = off;
    off = align(off + (size_t)slots * p->P * kTile * kTile * sc);
    p->ws_bytes = off;
    return off;
}

// Device bytes the plan holds once built (resident) and at most during
// construction (peak), from the geometry alone.  Work-item lists, whose
// length depends on the binning, are bounded by their largest possible size.
void plan_footprint(const wg_plan *p, size_t &resident, size_t &peak) {
    const Geom &g = p->g;
    const size_t sc = p->precision == WG_F32 ? 8 : 16;
    const size_t sr = sc / 2;
    const uint64_t npix = (uint64_t)g.npix_x * g.npix_y;
    const uint64_t ntot = (uint64_t)std::max<int64_t>(p->n_total, 1);
    const uint64_t nact = (uint64_t)std::max<int64_t>(p->n_active, 1);
    const uint64_t ntiles = (uint64_t)g.ntu * g.ntv;
    const uint64_t tab_n = ntiles * (uint64_t)(p->NJ + 1);
    const uint64_t span = (uint64_t)((p->alpha - 1 + p->P - 1) / p->P + 1);   // batches a visibility meets
    const uint64_t items = 3 * (4 * nact * span / (uint64_t)kDegridItemCap + (uint64_t)p->NJ) + 3;
    resident = (size_t)(p->desc.n_chan * 8 + (uint64_t)(p->alpha + 4) * p->alpha * sr +
                        (uint64_t)(g.nu + g.nv) * sc +
                        2 * npix * 8 + ntot * (8 + 4 + 4 + 4) + 2 * tab_n * 4 * 5 + 2 * nact * (3 * sr + 8) +
                        items * 16 + (p->col4 ? (uint64_t)(p->n1 + p->n2) * sc + 512 : 0));
    // construction also holds the radix-sort scratch (second key and value
    // buffers, histograms, scan levels) and small host-table copies
    const uint64_t nblocks = (ntot + kRsTile - 1) / kRsTile;
    const uint64_t sort = ntot * 12 + 256 * nblocks * 4 * 2 + 4096 + nact * 24;   // index sort; class keys + sort
    const uint64_t tables = (uint64_t)(g.npix_x + g.npix_y) * 8 + 2 * 1024 * 8 + (uint64_t)6 * p->NJ * 4;
    peak = resident + (size_t)(sort + tables);
}

// w range and number of selected visibilities (one reduction on the
// device, read back synchronously on the plan's stream).  scale: device
// [n_chan] freq / c.
int plan_wrange(const wg_plan_desc &d, DevMem &mem, const double *scale, int do_w, hipStream_t st,
                int64_t &n_active, double &wmin, double &wmax) {
    const int64_t n_total = d.n_rows * d.n_chan;
    unsigned long long *red = (unsigned long long *)mem.get(3 * sizeof(unsigned long long));
    if (!red) return WG_ENOMEM;
    if (n_total > 0)
        hipLaunchKernelGGL(k_wrange_init, dim3(1), dim3(64), 0, st, red);
    if (n_total > 0)
        hipLaunchKernelGGL(k_wrange, dim3((unsigned)grid_blocks(n_total, 256, 4096)), dim3(256), 0, st, d.uvw,
                           scale, d.mask, d.n_rows, d.n_chan, do_w, red);
    unsigned long long hred[3] = {~0ull, 0ull, 0ull};
    int rc = WG_OK;
    if (!hip_ok(hipGetLastError(), "k_wrange")) rc = WG_EHIP;
    if (rc == WG_OK && n_total > 0 &&
        (!hip_ok(hipMemcpyAsync(hred, red, sizeof(hred), hipMemcpyDeviceToHost, st), "w range copy") ||
         !hip_ok(hipStreamSynchronize(st), "w range sync")))
        rc = WG_EHIP;
    mem.put(red);
    if (rc != WG_OK) return rc;
    n_active = (int64_t)hred[2];
    if (do_w && n_active > 0) {
        std::memcpy(&wmin, &hred[0], sizeof(double));
        std::memcpy(&wmax, &hred[1], sizeof(double));
    } else {
        wmin = wmax = 0.0;
    }
    return WG_OK;
}

// Channel scale freq / c, computed on the host (one IEEE division) and
// uploaded; the frequencies are checked to be positive.
int plan_scale(const wg_plan_desc &d, DevMem &mem, hipStream_t st, double *&scale_dev) {
    std::vector<double> freq(d.n_chan), scale(d.n_chan);
    HIP_TRY(hipMemcpyAsync(freq.data(), d.freq, d.n_chan * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t c = 0; c < d.n_chan; ++c) {
        if (!(freq[c] > 0.0)) return WG_EINVAL;
        scale[c] = freq[c] / kC;
    }
    scale_dev = (double *)mem.get(d.n_chan * sizeof(double));
    if (!scale_dev) return WG_ENOMEM;
    HIP_TRY(hipMemcpyAsync(scale_dev, scale.data(), d.n_chan * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // the host vector must outlive the copy
    return WG_OK;
}

// Host planning once the w range and the active count are known: kernel
// choice (Sect. 4.1), polynomial degree (Sect. 4.2), grid and plane geometry
// (Sect. 2), batching and FFT descriptors.  No device work.
int plan_host(wg_plan *p) {
    const wg_plan_desc &d = p->desc;
    if (d.alpha) {
        p->alpha = d.alpha;
        p->sigma = d.sigma;
        p->predicted = predict_seconds(d.alpha, d.sigma, d.precision, p->do_w, d.npix_x, d.npix_y,
                                       max_abs_nm1(d.npix_x, d.npix_y, d.pixsize_x, d.pixsize_y),
                                       p->n_active, p->wmin, p->wmax);
    } else if (select_kernel(d.epsilon, d.precision, p->do_w, d.npix_x, d.npix_y, d.pixsize_x, d.pixsize_y,
                             p->n_active, p->wmin, p->wmax, &p->alpha, &p->sigma, &p->predicted) != 0) {
        return WG_EUNSUPPORTED;
    }
    const KernelRow *row = find_row(p->alpha, p->sigma);
    p->beta = row->beta;
    p->mu = row->mu;
    p->eps_k = row->eps;
    p->degree = choose_degree(p->alpha, p->beta, p->mu, p->eps_k, d.precision);
    if (p->degree > p->alpha + 3) return WG_EUNSUPPORTED;   // the kernels' LDS table holds alpha + 4 rows
    {
        std::vector<double> c;
        kernel_poly(p->alpha, p->beta, p->mu, p->degree, c);
        p->poly_err = kernel_poly_max_error(p->alpha, p->beta, p->mu, p->degree, c);
    }
    p->amp = rounding_amplification(p->alpha, p->sigma, p->do_w, d.npix_x, d.npix_y, d.pixsize_x, d.pixsize_y);
    p->round_err = rounding_error(p->alpha, p->sigma, d.precision, p->do_w, d.npix_x, d.npix_y, d.pixsize_x,
                                  d.pixsize_y);

    // geometry (Sect. 2)
    Geom &g = p->g;
    g.nu = grid_size(p->sigma, d.npix_x);
    g.nv = grid_size(p->sigma, d.npix_y);
    g.ntu = g.nu / kTile;
    g.ntv = g.nv / kTile;
    g.npix_x = d.npix_x;
    g.npix_y = d.npix_y;
    g.alpha = p->alpha;
    g.do_w = p->do_w;
    g.half = 0.5 * p->alpha;
    g.pixsize_x = d.pixsize_x;
    g.pixsize_y = d.pixsize_y;
    g.n_chan = d.n_chan;
    if (p->do_w) {
        g.dw = 1.0 / (2.0 * p->sigma * max_abs_nm1(d.npix_x, d.npix_y, d.pixsize_x, d.pixsize_y));
        g.w0 = p->wmin - g.dw * (p->alpha - 1) * 0.5;
        g.nw = (int)std::ceil((p->wmax - p->wmin) / g.dw) + p->alpha;
    } else {
        g.dw = 1.0;
        g.w0 = 0.0;
        g.nw = 1;
    }
    const size_t sc = d.precision == WG_F32 ? 8 : 16;
    const size_t sr = sc / 2;
    // FFT length limit: one transform line must fit in LDS
    const size_t lds_cap = 160 * 1024;
    if ((size_t)std::max(g.nu, g.nv) * sc > lds_cap || std::max(g.nu, g.nv) > max_grid(d.precision))
        return WG_EUNSUPPORTED;
    // columns per workgroup in the strided passes: as many as fit about
    // 144 KB of LDS (the gridding column pass also keeps npix_x * K image
    // sums there) and the values one column-pass workgroup transforms, N K:
    // FP32 <= 12288 (1024 threads x 12), FP64 <= 6144 (256 threads x
    // kFftMaxC), the same bounds that cap N itself
    const int64_t col_values = d.precision == WG_F32 ? 12288 : 6144;
    p->k_cols = 1;
    while (p->k_cols < 8 && (size_t)(fft_lds_len(g.nu) * sc + d.npix_x * sr) * (2 * p->k_cols) <= 144 * 1024 &&
           (int64_t)g.nu * 2 * p->k_cols <= col_values)
        p->k_cols *= 2;
    p->k_cols_d = p->k_cols;
    // four-step column transform where the one-pass form keeps at most two
    // columns per workgroup (its row pieces are then 16 or 32 bytes; at four
    // FP32 columns the one-pass form measured faster), or when asked for:
    // N_u = n1 n2 with both
    // factors in [17, 128] (16-column panels of n_k values fit 256 threads x
    // 8, and each sub-length takes at least two FFT passes), as close to
    // sqrt(N_u) as the factors allow
    p->col4 = 0;
    if (d.column_transform < 0 || d.column_transform > 2) return WG_EINVAL;
    if (d.column_transform == 2 || (d.column_transform == 0 && p->k_cols <= 2)) {
        int best = 0;
        for (int a = 17; a <= 128; ++a) {
            if (g.nu % a != 0 || g.nu / a < 17 || g.nu / a > 128) continue;
            FftDesc f1, f2;
            make_fft_desc(a, f1);
            make_fft_desc(g.nu / a, f2);
            if (fft_desc_len(f1) != a || fft_desc_len(f2) != g.nu / a) continue;
            if (!best || std::abs(a - g.nu / a) < std::abs(best - g.nu / best)) best = a;
        }
        if (best) {
            p->col4 = 1;
            p->n1 = best;
            p->n2 = g.nu / best;
            make_fft_desc(p->n1, p->fft_n1);
            make_fft_desc(p->n2, p->fft_n2);
        } else if (d.column_transform == 2) {
            return WG_EUNSUPPORTED;
        }
    }
    // planes per batch: P = alpha (a visibility's alpha planes then meet at
    // most two batches), at most the 8 plane slots of the matrix-core
    // gridders (the 16 rows of their 16 x 16 products, re and im per slot);
    // the degridder stages the batch's planes a group at a time
    const int max_slots = 8;
    p->P = d.planes_per_batch > 0 ? std::min(d.planes_per_batch, p->alpha) : p->alpha;
    p->P = std::min(std::min(p->P, max_slots), g.nw);
    p->NJ = (g.nw + p->P - 1) / p->P;
    make_fft_desc(g.nu, p->fft_u);
    make_fft_desc(g.nv, p->fft_v);
    return WG_OK;
}

void *scratch_for_device(int dev);

int plan_build(wg_plan *p) {
    const wg_plan_desc &d = p->desc;
    hipStream_t st = p->stream;
    HIP_TRY(hipGetDevice(&p->device));
    // the apply pipeline's side stream (default priority) and events
    HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    for (hipEvent_t &e : p->ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // set-up of the allocation-free entry point on this device (its scratch
    // address, looked up once per device); a failure is reported by that
    // entry point, not here
    if (!scratch_for_device(p->device)) (void)hipGetLastError();
    p->precision = d.precision;
    p->do_w = d.do_wgridding ? 1 : 0;
    p->n_total = d.n_rows * d.n_chan;
    int rc = plan_scale(d, p->mem, st, p->scale);
    if (rc != WG_OK) return rc;
    rc = plan_wrange(d, p->mem, p->scale, p->do_w, st, p->n_active, p->wmin, p->wmax);
    if (rc != WG_OK) return rc;
    rc = plan_host(p);
    if (rc != WG_OK) return rc;
    const Geom &g = p->g;
    const size_t sc = d.precision == WG_F32 ? 8 : 16;
    const size_t sr = sc / 2;

    // host tables: polynomial, psi on the pixel axes, quadrature nodes, twiddles
    std::vector<double> coef_id;
    kernel_poly(p->alpha, p->beta, p->mu, p->degree, coef_id);
    std::vector<double> coefd((size_t)(p->degree + 1) * p->alpha);   // degree-major
    for (int i = 0; i < p->alpha; ++i)
        for (int k = 0; k <= p->degree; ++k)
            coefd[(size_t)k * p->alpha + i] = coef_id[(size_t)i * (p->degree + 1) + k];
    std::vector<double> qt, qw;
    psi_nodes(p->alpha, p->beta, p->mu, qt, qw);
    std::vector<double> psix(d.npix_x), psiy(d.npix_y);
    for (int i = 0; i < d.npix_x; ++i) psix[i] = psi_eval((double)(i - d.npix_x / 2) / g.nu, qt, qw);
    for (int i = 0; i < d.npix_y; ++i) psiy[i] = psi_eval((double)(i - d.npix_y / 2) / g.nv, qt, qw);
    std::vector<double> tur, tui, tvr, tvi;
    twiddles(g.nu, tur, tui);
    twiddles(g.nv, tvr, tvi);
    rc = d.precision == WG_F32 ? build_plan_tables<float>(p, coefd, tur, tui, tvr, tvi)
                               : build_plan_tables<double>(p, coefd, tur, tui, tvr, tvi);
    if (rc != WG_OK) return rc;

    // correction factors
    const int64_t npix = (int64_t)d.npix_x * d.npix_y;
    p->nm1 = (double *)p->mem.get(npix * sizeof(double));
    p->corr = (double *)p->mem.get(npix * sizeof(double));
    double *dpx = (double *)p->mem.get(d.npix_x * sizeof(double));
    double *dpy = (double *)p->mem.get(d.npix_y * sizeof(double));
    double *dqt = (double *)p->mem.get(qt.size() * sizeof(double));
    double *dqw = (double *)p->mem.get(qw.size() * sizeof(double));
    if (!p->nm1 || !p->corr || !dpx || !dpy || !dqt || !dqw) return WG_ENOMEM;
    HIP_TRY(hipMemcpyAsync(dpx, psix.data(), psix.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dpy, psiy.data(), psiy.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dqt, qt.data(), qt.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dqw, qw.data(), qw.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // host vectors live until here
    hipLaunchKernelGGL(k_corr, dim3((unsigned)grid_blocks(npix, 256, 1 << 20)), dim3(256), 0, st, d.npix_x,
                       d.npix_y, d.pixsize_x, d.pixsize_y, p->do_w, g.dw, dpx, dpy, dqt, dqw, (int)qt.size(),
                       p->nm1, p->corr);
    LAUNCH_CHECK("k_corr");

    // visibility index: keys, stable sort, batch tables
    const unsigned long long ntiles = (unsigned long long)g.ntu * g.ntv;
    const unsigned long long sentinel = ntiles * (unsigned long long)g.nw;
    int bits = 1;
    while (bits < 64 && (sentinel >> bits) != 0) ++bits;
    const int64_t nkeys = std::max<int64_t>(p->n_total, 1);
    p->keys = (unsigned long long *)p->mem.get(nkeys * sizeof(unsigned long long));
    p->order = (uint32_t *)p->mem.get(nkeys * sizeof(uint32_t));
    if (!p->keys || !p->order) return WG_ENOMEM;
    if (p->n_total > 0) {
        hipLaunchKernelGGL(k_keys, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 20)), dim3(256), 0, st, d.uvw,
                           p->scale, d.mask, d.n_rows, g, sentinel, p->keys, p->order);
        LAUNCH_CHECK("k_keys");
        rc = radix_sort(p, p->keys, p->order, p->n_total, bits, st);
        if (rc != WG_OK) return rc;
    }
    const unsigned long long tab_n = ntiles * (unsigned long long)(p->NJ + 1);
    p->tab_lo = (uint32_t *)p->mem.get(tab_n * sizeof(uint32_t));
    p->tab_hi = (uint32_t *)p->mem.get(tab_n * sizeof(uint32_t));
    if (!p->tab_lo || !p->tab_hi) return WG_ENOMEM;
    hipLaunchKernelGGL(k_fill_tab, dim3((unsigned)grid_blocks(p->n_active + 1, 256, 1 << 20)), dim3(256), 0, st,
                       p->keys, p->n_active, g.nw, p->P, p->NJ, p->alpha - 1, tab_n, p->tab_lo);
    hipLaunchKernelGGL(k_fill_tab, dim3((unsigned)grid_blocks(p->n_active + 1, 256, 1 << 20)), dim3(256), 0, st,
                       p->keys, p->n_active, g.nw, p->P, p->NJ, 0, tab_n, p->tab_hi);
    LAUNCH_CHECK("k_fill_tab");
    // sorted per-visibility stream: kernel-local coordinates and anchors
    const int64_t nact = std::max<int64_t>(p->n_active, 1);
    p->zc = p->mem.get(nact * 3 * sr);
    p->anc = (int2 *)p->mem.get(nact * sizeof(int2));
    if (!p->zc || !p->anc) return WG_ENOMEM;
    if (p->n_active > 0) {
        if (d.precision == WG_F32)
            hipLaunchKernelGGL(k_vis_prep<float>, dim3((unsigned)grid_blocks(p->n_active, 256, 1 << 20)), dim3(256), 0,
                               st, d.uvw, p->scale, p->order, p->n_active, g, (float *)p->zc, p->anc);
        else
            hipLaunchKernelGGL(k_vis_prep<double>, dim3((unsigned)grid_blocks(p->n_active, 256, 1 << 20)), dim3(256),
                               0, st, d.uvw, p->scale, p->order, p->n_active, g, (double *)p->zc, p->anc);
        LAUNCH_CHECK("k_vis_prep");
    }
    // inverse permutation (caller's order -> sorted position and fold bit)
    p->inv = (uint32_t *)p->mem.get(std::max<int64_t>(p->n_total, 1) * sizeof(uint32_t));
    if (!p->inv) return WG_ENOMEM;
    if (p->n_total > 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 20)), dim3(256), 0, st,
                           p->inv, p->n_total, 0xffffffffu);
        if (p->n_active > 0)
            hipLaunchKernelGGL(k_inv_order, dim3((unsigned)grid_blocks(p->n_active, 256, 1 << 20)), dim3(256), 0,
                               st, p->order, p->anc, p->n_active, p->inv);
        LAUNCH_CHECK("k_inv_order");
    }
    // gridder stream: the index re-sorted by (tile, edge rank, first plane)
    rc = build_class_stream(p, st, bits);
    if (rc != WG_OK) return rc;
    // work items: lists of the gridder and degridder beyond the item cap
    rc = build_items(p, st);
    if (rc != WG_OK) return rc;
    p->index_bytes += nkeys * (sizeof(unsigned long long) + sizeof(uint32_t)) + 6 * tab_n * sizeof(uint32_t) +
                      2 * nact * (3 * sr + sizeof(int2)) + 2 * std::max<int64_t>(p->n_total, 1) * sizeof(uint32_t);
    HIP_TRY(hipStreamSynchronize(st));
    p->mem.put(dpx);
    p->mem.put(dpy);
    p->mem.put(dqt);
    p->mem.put(dqw);

    plan_layout(p, p->max_slots);
    return WG_OK;
}

// ---- apply ------------------------------------------------------------------

template <typename R>
void launch_vis_kernel(bool gridding, const wg_plan *p, const VisArgs<R> &va, int J, Cx<R> *G, Cx<R> *vacc,
                       Cx<R> *part, hipStream_t st) {
    switch (p->alpha) {
#define CASE(A)                                                          \
    case A:                                                              \
        launch_vis<R, A>(gridding, p, va, J, G, vacc, part, st);         \
        break;
        CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15)
        CASE(16)
#undef CASE
        default: break;
    }
}

template <typename R, int NTH> struct FftLaunch {
    template <int CAP>
    static void rows_grid(const wg_plan *p, const Cx<R> *G, Cx<R> *T, const PassGeom &pg, int np, hipStream_t st) {
        hipLaunchKernelGGL((k_rows_grid<R, NTH, CAP>), dim3(p->g.nu, np), dim3(NTH), fft_lds_len(p->g.nv) * sizeof(Cx<R>), st, G, T,
                           pg, p->fft_v, (const Cx<R> *)p->tw_v);
    }
    static void cols_grid(const wg_plan *p, const Cx<R> *T, R *acc, const PassGeom &pg, int j_lo, int np,
                          hipStream_t st) {
        const int K = p->k_cols;
        const int nb = ((p->g.npix_y + K - 1) / K + 7) / 8 * 8;
        const size_t lds = (size_t)fft_lds_len(p->g.nu) * K * sizeof(Cx<R>) + (size_t)p->g.npix_x * K * sizeof(R);
        hipLaunchKernelGGL((k_cols_grid<R, NTH>), dim3(nb), dim3(NTH), lds, st, T,
                           acc, p->nm1, pg, K, j_lo, np, p->fft_u, (const Cx<R> *)p->tw_u);
    }
    template <int CAP>
    static void rows_degrid(const wg_plan *p, const R *itil, Cx<R> *T, const PassGeom &pg, int j_lo, int np,
                            hipStream_t st) {
        hipLaunchKernelGGL((k_rows_degrid<R, NTH, CAP>), dim3(p->g.npix_x, np), dim3(NTH), fft_lds_len(p->g.nv) * sizeof(Cx<R>), st,
                           itil, p->nm1, T, pg, j_lo, np, p->fft_v, (const Cx<R> *)p->tw_v);
    }
    template <int CAP>
    static void cols_degrid(const wg_plan *p, const Cx<R> *T, Cx<R> *G, const PassGeom &pg, int np,
                            hipStream_t st) {
        const int K = p->k_cols_d;
        const int nb = ((p->g.nv + K - 1) / K + 7) / 8 * 8;
        hipLaunchKernelGGL((k_cols_degrid<R, NTH, CAP>), dim3(nb, np), dim3(NTH), (size_t)fft_lds_len(p->g.nu) * K * sizeof(Cx<R>),
                           st, T, G, pg, K, p->fft_u, (const Cx<R> *)p->tw_u);
    }
};

// Four-step column transform: 256 threads, 8 values a thread (16-column
// panels of n1, n2 <= 128 values).
template <typename R> struct Col4Launch {
    static constexpr int NTH = 256, CAP = 8;
    static Col4Geom geom(const wg_plan *p, bool gridding) {
        const Geom &g = p->g;
        Col4Geom cg;
        cg.n = g.nu;
        cg.n1 = p->n1;
        cg.n2 = p->n2;
        cg.rows_in = gridding ? g.nu : g.npix_x;
        cg.h = gridding ? 0 : g.npix_x / 2;
        cg.ncols = gridding ? g.npix_y : g.nv;
        cg.in_plane = gridding ? panel_elems(g.npix_y, g.nu) : panel_elems(g.nv, g.npix_x);
        cg.y_plane = panel_elems(cg.ncols, g.nu);
        return cg;
    }
    static int panels(const Col4Geom &cg) { return (cg.ncols + kPanel - 1) / kPanel; }
    static void pass_a(const wg_plan *p, bool gridding, const Cx<R> *in, Cx<R> *Y, int np, hipStream_t st) {
        const Col4Geom cg = geom(p, gridding);
        const dim3 grid(panels(cg) * cg.n2, np);
        const size_t lds = (size_t)fft_lds_len(cg.n1) * kPanel * sizeof(Cx<R>);
        if (gridding)
            hipLaunchKernelGGL((k_col4_a<R, NTH, CAP, +1, false>), grid, dim3(NTH), lds, st, in, Y, cg, p->fft_n1,
                               (const Cx<R> *)p->tw_n1, (const Cx<R> *)p->tw_u);
        else
            hipLaunchKernelGGL((k_col4_a<R, NTH, CAP, -1, true>), grid, dim3(NTH), lds, st, in, Y, cg, p->fft_n1,
                               (const Cx<R> *)p->tw_n1, (const Cx<R> *)p->tw_u);
    }
    static void pass_b_degrid(const wg_plan *p, const Cx<R> *Y, Cx<R> *G, int np, hipStream_t st) {
        const Col4Geom cg = geom(p, false);
        hipLaunchKernelGGL((k_col4_b_degrid<R, NTH, CAP>), dim3(panels(cg) * cg.n1, np), dim3(NTH),
                           (size_t)fft_lds_len(cg.n2) * kPanel * sizeof(Cx<R>), st, Y, G, cg, p->g.nv, p->fft_n2,
                           (const Cx<R> *)p->tw_n2);
    }
    static void pass_b_grid(const wg_plan *p, const Cx<R> *Y, R *acc, const PassGeom &pg, int j_lo, int np,
                            hipStream_t st) {
        const Col4Geom cg = geom(p, true);
        hipLaunchKernelGGL((k_col4_b_grid<R, NTH, CAP>), dim3(panels(cg) * cg.n1), dim3(NTH),
                           (size_t)fft_lds_len(cg.n2) * kPanel * sizeof(Cx<R>), st, Y, acc, p->nm1, pg, cg, j_lo, np,
                           p->fft_n2, (const Cx<R> *)p->tw_n2);
    }
};

// Row transforms (K = 1, N up to the LDS limit): FP32 256/1024 threads,
// FP64 256/512.  Column transforms: FP32 256/1024 (the wide workgroup keeps
// 16 waves on the CU that its LDS allows), FP64 256.  Each choice keeps a
// thread at <= kFftMaxC values without spills.
#define DISPATCH_ROWS(n, EXPR_T)                                       \
    do {                                                               \
        if ((n) <= 256 * 12) {                                         \
            constexpr int NTH = 256, CAP = 12;                         \
            EXPR_T;                                                    \
        } else if ((n) <= 256 * kFftMaxC) {                            \
            constexpr int NTH = 256, CAP = 0;                          \
            EXPR_T;                                                    \
        } else {                                                       \
            constexpr int NTH = sizeof(R) == 4 ? 1024 : 512, CAP = 0;  \
            EXPR_T;                                                    \
        }                                                              \
    } while (0)
#define DISPATCH_COLS(n, EXPR_T)                                       \
    do {                                                               \
        if (sizeof(R) == 8 || (n) <= 256 * kFftMaxC) {                 \
            constexpr int NTH = 256;                                   \
            EXPR_T;                                                    \
        } else {                                                       \
            constexpr int NTH = sizeof(R) == 4 ? 1024 : 256;           \
            EXPR_T;                                                    \
        }                                                              \
    } while (0)

#define DISPATCH_COLS_D(n, EXPR_T)                                     \
    do {                                                               \
        if (sizeof(R) == 8 || (n) <= 256 * kFftMaxC) {                 \
            constexpr int NTH = 256, CAP = 0;                          \
            EXPR_T;                                                    \
        } else {                                                       \
            constexpr int NTH = sizeof(R) == 4 ? 1024 : 256, CAP = 0;  \
            EXPR_T;                                                    \
        }                                                              \
    } while (0)

template <typename R>
int apply(const wg_plan *p, bool gridding, const void *in, const void *wgt, void *out, void *ws, size_t ws_bytes,
          hipStream_t st) {
    using C = Cx<R>;
    if (!ws || ws_bytes < p->ws_bytes) return WG_EINVAL;
    std::lock_guard<std::mutex> lock(p->enqueue_mu);
    const Geom &g = p->g;
    const wg_plan_desc &d = p->desc;
    unsigned char *w = (unsigned char *)ws;
    C *Gbuf[2] = {(C *)(w + p->off_G), (C *)(w + p->off_G2)};
    C *T = (C *)(w + p->off_T);
    C *Y = (C *)(w + p->off_Y);
    R *acc = (R *)(w + p->off_acc);
    R *itil = (R *)(w + p->off_itil);
    C *vacc = (C *)(w + p->off_vacc);
    C *part = (C *)(w + p->off_part);
    const int64_t npix = (int64_t)g.npix_x * g.npix_y;

    // degridder: the index order; gridder: the class-ordered stream
    VisArgs<R> va;
    va.z = (const R *)p->zc;
    va.anc = p->anc;
    va.vsorted = nullptr;
    va.tab_lo = p->tab_lo;
    va.tab_hi = p->tab_hi;
    va.coef = (const R *)p->coef;
    va.degree = p->degree;
    va.P = p->P;
    va.NJ = p->NJ;
    va.g = g;
    VisArgs<R> vg = va;
    vg.z = (const R *)p->zc2;
    vg.anc = p->anc2;
    vg.vsorted = vacc;              // gridding: the ordered input lives where degridding accumulates
    vg.tab_lo = p->tab2_lo;
    vg.tab_hi = p->tab2_hi;
    PassGeom pg{g.nu, g.nv, g.npix_x, g.npix_y, p->P, g.nw, g.do_w, g.w0, g.dw};

    if (gridding) {
        {
            ProfScope ps(WG_KIND_IMAGE, st);
            hipLaunchKernelGGL(k_fill_zero<R>, dim3((unsigned)grid_blocks(npix, 256, 1 << 16)), dim3(256), 0, st, acc,
                               npix);
        }
        if (p->n_active > 0) {
            {
                ProfScope ps(WG_KIND_VIS, st);
                hipLaunchKernelGGL(k_gather_vis<R>, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 16)), dim3(256),
                                   0, st, (const C *)in, (const R *)wgt, p->inv2, p->n_total, vacc);
            }
            // Two streams (one while a profiler is attached, so that each
            // timed launch runs alone): the gridder of batch J (side stream)
            // fills plane buffer J mod 2 while the FFT passes of batch J - 1
            // (caller's stream) read the other one; the image sums stay in
            // batch order on the caller's stream.
            hipStream_t sd = g_prof ? st : p->side;
            hipEvent_t e_start = p->ev[0], e_vis[2] = {p->ev[1], p->ev[2]}, e_rows[2] = {p->ev[3], p->ev[4]};
            HIP_TRY(hipEventRecord(e_start, st));
            HIP_TRY(hipStreamWaitEvent(sd, e_start, 0));
            for (int J = 0; J < p->NJ; ++J) {
                const int j_lo = J * p->P;
                const int np = std::min(p->P, g.nw - j_lo);
                const int b = J & 1;
                C *G = Gbuf[b];
                // buffer b is free once the row pass of batch J - 2 has read it
                if (J >= 2) HIP_TRY(hipStreamWaitEvent(sd, e_rows[b], 0));
                {
                    ProfScope ps(WG_KIND_GRID, sd);
                    launch_vis_kernel<R>(true, p, vg, J, G, nullptr, part, sd);
                }
                HIP_TRY(hipEventRecord(e_vis[b], sd));
                HIP_TRY(hipStreamWaitEvent(st, e_vis[b], 0));
                {
                    ProfScope ps(WG_KIND_FFT_ROWS_GRID, st);
                    DISPATCH_ROWS(g.nv, (FftLaunch<R, NTH>::template rows_grid<CAP>(p, G, T, pg, np, st)));
                }
                HIP_TRY(hipEventRecord(e_rows[b], st));
                {
                    ProfScope ps(WG_KIND_FFT_COLS_GRID, st);
                    if (p->col4) {
                        Col4Launch<R>::pass_a(p, true, T, Y, np, st);
                        Col4Launch<R>::pass_b_grid(p, Y, acc, pg, j_lo, np, st);
                    } else {
                        DISPATCH_COLS(g.nu * p->k_cols, (FftLaunch<R, NTH>::cols_grid(p, T, acc, pg, j_lo, np, st)));
                    }
                }
            }
            // every side-stream launch precedes the last batch's event, which
            // the caller's stream has waited for
        }
        {
            ProfScope ps(WG_KIND_IMAGE, st);
            hipLaunchKernelGGL(k_scale_image<R>, dim3((unsigned)grid_blocks(npix, 256, 1 << 16)), dim3(256), 0, st,
                               acc, p->corr, (R *)out, npix);
        }
    } else {
        if (p->n_total > 0 && d.mask) {
            ProfScope ps(WG_KIND_VIS, st);
            hipLaunchKernelGGL(k_zero_masked<R>, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 16)), dim3(256), 0,
                               st, d.mask, p->n_total, (C *)out);
        }
        if (p->n_active > 0) {
            {
                ProfScope ps(WG_KIND_IMAGE, st);
                hipLaunchKernelGGL(k_scale_image<R>, dim3((unsigned)grid_blocks(npix, 256, 1 << 16)), dim3(256), 0, st,
                                   (const R *)in, p->corr, itil, npix);
            }
            {
                ProfScope ps(WG_KIND_VIS, st);
                hipLaunchKernelGGL(k_fill_zero<C>, dim3((unsigned)grid_blocks(p->n_active, 256, 1 << 16)), dim3(256),
                                   0, st, vacc, p->n_active);
            }
            // Two streams (one while a profiler is attached): the FFT passes
            // of batch J (caller's stream) fill plane buffer J mod 2 while the
            // degridder of batch J - 1 (side stream) reads the other one; the
            // visibility sums stay in batch order on the side stream.
            hipStream_t sd = g_prof ? st : p->side;
            hipEvent_t e_start = p->ev[0], e_fft[2] = {p->ev[1], p->ev[2]}, e_vis[2] = {p->ev[3], p->ev[4]};
            hipEvent_t e_end = p->ev[5];
            HIP_TRY(hipEventRecord(e_start, st));
            HIP_TRY(hipStreamWaitEvent(sd, e_start, 0));
            for (int J = 0; J < p->NJ; ++J) {
                const int j_lo = J * p->P;
                const int np = std::min(p->P, g.nw - j_lo);
                const int b = J & 1;
                C *G = Gbuf[b];
                {
                    ProfScope ps(WG_KIND_FFT_ROWS_DEGRID, st);
                    DISPATCH_ROWS(g.nv, (FftLaunch<R, NTH>::template rows_degrid<CAP>(p, itil, T, pg, j_lo, np, st)));
                }
                {
                    ProfScope ps(WG_KIND_FFT_COLS_DEGRID, st);
                    if (p->col4) Col4Launch<R>::pass_a(p, false, T, Y, np, st);
                    // buffer b is free once the degridder of batch J - 2 has read it
                    if (J >= 2) HIP_TRY(hipStreamWaitEvent(st, e_vis[b], 0));
                    if (p->col4) {
                        Col4Launch<R>::pass_b_degrid(p, Y, G, np, st);
                    } else {
                        DISPATCH_COLS_D(g.nu * p->k_cols_d,
                                        (FftLaunch<R, NTH>::template cols_degrid<CAP>(p, T, G, pg, np, st)));
                    }
                }
                HIP_TRY(hipEventRecord(e_fft[b], st));
                HIP_TRY(hipStreamWaitEvent(sd, e_fft[b], 0));
                {
                    ProfScope ps(WG_KIND_DEGRID, sd);
                    launch_vis_kernel<R>(false, p, va, J, G, vacc, nullptr, sd);
                }
                HIP_TRY(hipEventRecord(e_vis[b], sd));
            }
            HIP_TRY(hipEventRecord(e_end, sd));
            HIP_TRY(hipStreamWaitEvent(st, e_end, 0));
            {
                ProfScope ps(WG_KIND_VIS, st);
                hipLaunchKernelGGL(k_degrid_finish<R>, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 16)), dim3(256),
                                   0, st, vacc, p->inv, (const R *)wgt, p->n_total, (C *)out);
            }
        }
    }
    if (!hip_ok(hipGetLastError(), gridding ? "wg_grid launch" : "wg_degrid launch")) return WG_EHIP;
    return WG_OK;
}

}  // namespace

// ---- fixed scratch of the allocation-free entry point -----------------------
// One statically sized device array per GPU (its own copy on each device the
// library runs on, held until the process ends).  Host code never uses the
// array's name as an address: the device address of this device's copy is
// looked up once per device with hipGetSymbolAddress and kept here.
constexpr size_t kScratchBytes = WG_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on the first call on
// the device, with that device current); nullptr on failure.
void *scratch_for_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

int wg_plan_create(const wg_plan_desc *desc, wg_plan **out) {
    if (!out) return WG_EINVAL;
    *out = nullptr;
    int rc = validate(desc);
    if (rc != WG_OK) return rc;
    wg_plan *p = new (std::nothrow) wg_plan();
    if (!p) return WG_ENOMEM;
    p->desc = *desc;
    p->stream = (hipStream_t)desc->stream;
    p->mem.alloc = desc->alloc;
    p->mem.free = desc->free;
    p->mem.ctx = desc->alloc_ctx;
    rc = plan_build(p);
    if (rc != WG_OK) {
        (void)hipStreamSynchronize(p->stream);
        wg_plan_destroy(p);
        return rc;
    }
    *out = p;
    return WG_OK;
}

int wg_plan_destroy(wg_plan *p) {
    if (!p) return WG_OK;
    for (hipEvent_t &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->side) (void)hipStreamDestroy(p->side);
    p->mem.release_all();
    delete p;
    return WG_OK;
}

int wg_degrid(const wg_plan *p, const void *dirty, const void *wgt, void *vis, void *workspace,
              size_t workspace_bytes, void *stream) {
    if (!p || !dirty || (!vis && p->n_total > 0)) return WG_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return p->precision == WG_F32 ? apply<float>(p, false, dirty, wgt, vis, workspace, workspace_bytes, st)
                                  : apply<double>(p, false, dirty, wgt, vis, workspace, workspace_bytes, st);
}

int wg_grid(const wg_plan *p, const void *vis, const void *wgt, void *dirty, void *workspace,
            size_t workspace_bytes, void *stream) {
    if (!p || !dirty || (!vis && p->n_total > 0)) return WG_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    return p->precision == WG_F32 ? apply<float>(p, true, vis, wgt, dirty, workspace, workspace_bytes, st)
                                  : apply<double>(p, true, vis, wgt, dirty, workspace, workspace_bytes, st);
}

int wg_apply_noalloc(const wg_plan *p, int adjoint, const void *in, const void *wgt, void *out, void *stream) {
    if (!p || !in || (!out && (adjoint || p->n_total > 0))) return WG_EINVAL;
    if (p->ws_bytes > kScratchBytes) return WG_ESCRATCH;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return WG_EINVAL;
    void *ws = scratch_for_device(dev);
    if (!ws) return WG_EHIP;
    hipStream_t st = (hipStream_t)stream;
    const bool grid = adjoint != 0;
    return p->precision == WG_F32 ? apply<float>(p, grid, in, wgt, out, ws, kScratchBytes, st)
                                  : apply<double>(p, grid, in, wgt, out, ws, kScratchBytes, st);
}

int wg_plan_info(const wg_plan *p, wg_plan_info_t *info) {
    if (!p || !info) return WG_EINVAL;
    std::memset(info, 0, sizeof(*info));
    const Geom &g = p->g;
    info->alpha = p->alpha;
    info->sigma = p->sigma;
    info->beta = p->beta;
    info->mu = p->mu;
    info->eps_kernel = p->eps_k;
    info->poly_degree = p->degree;
    info->nu = g.nu;
    info->nv = g.nv;
    info->nw = g.nw;
    info->dw = g.dw;
    info->w0 = g.w0;
    info->wmin = p->wmin;
    info->wmax = p->wmax;
    info->npix_x = g.npix_x;
    info->npix_y = g.npix_y;
    info->precision = p->precision;
    info->do_wgridding = p->do_w;
    info->n_rows = p->desc.n_rows;
    info->n_chan = p->desc.n_chan;
    info->n_vis = p->n_active;
    info->planes_per_batch = p->P;
    info->tile = kTile;
    const double sc = p->precision == WG_F32 ? 8.0 : 16.0, sr = sc / 2;
    const double nvis = (double)p->n_active;
    const double planes = (double)g.nw * ((double)g.nu * g.nv * sc * 2.0 + (double)g.nu * g.npix_y * sc * 2.0 +
                                          2.0 * (double)g.npix_x * g.npix_y * sr);
    const double vis_b = nvis * (sc + 4.0) + (double)p->desc.n_rows * 24.0;
    info->bytes_grid = planes + vis_b;
    info->bytes_degrid = planes + vis_b;
    info->predicted_seconds = p->predicted;
    info->plan_bytes = p->mem.total;
    info->index_bytes = p->index_bytes;
    info->workspace_bytes = p->ws_bytes;
    info->extra_items_grid = p->xg_off.empty() ? 0 : p->xg_off.back();
    info->extra_items_degrid = p->xd_off.empty() ? 0 : p->xd_off.back();
    info->rounding_error = p->round_err;
    info->amplification = p->amp;
    info->poly_error = p->poly_err;
    info->column_transform = p->col4 ? 2 : 1;
    info->col_n1 = p->col4 ? p->n1 : 0;
    info->col_n2 = p->col4 ? p->n2 : 0;
    info->col_k = p->k_cols;
    return WG_OK;
}

int wg_plan_estimate(const wg_plan_desc *desc, size_t *plan_bytes, size_t *peak_bytes, size_t *workspace_bytes) {
    int rc = validate(desc);
    if (rc != WG_OK) return rc;
    wg_plan *p = new (std::nothrow) wg_plan();
    if (!p) return WG_ENOMEM;
    p->desc = *desc;
    p->stream = (hipStream_t)desc->stream;
    p->mem.alloc = desc->alloc;
    p->mem.free = desc->free;
    p->mem.ctx = desc->alloc_ctx;
    p->precision = desc->precision;
    p->do_w = desc->do_wgridding ? 1 : 0;
    p->n_total = desc->n_rows * desc->n_chan;
    rc = plan_scale(*desc, p->mem, p->stream, p->scale);
    if (rc == WG_OK) rc = plan_wrange(*desc, p->mem, p->scale, p->do_w, p->stream, p->n_active, p->wmin, p->wmax);
    if (rc == WG_OK) rc = plan_host(p);
    if (rc == WG_OK) {
        size_t res = 0, peak = 0;
        plan_footprint(p, res, peak);
        // partial-tile slots of the gridder: at most one per item beyond the
        // first of a tile, and a batch deals at most 4 n_active visibility visits
        const int64_t slots = 4 * std::max<int64_t>(p->n_active, 1) / kGridItemCap + 1;
        const size_t ws = plan_layout(p, slots);
        if (plan_bytes) *plan_bytes = res;
        if (peak_bytes) *peak_bytes = peak;
        if (workspace_bytes) *workspace_bytes = ws;
    }
    delete p;   // releases the temporaries
    return rc;
}

size_t wg_workspace_bytes(const wg_plan *p) { return p ? p->ws_bytes : 0; }
size_t wg_plan_bytes(const wg_plan *p) { return p ? p->mem.total : 0; }

int wg_plan_index(const wg_plan *p, void *keys, void *order, void *stream) {
    if (!p) return WG_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (p->n_active == 0) return WG_OK;
    if (keys)
        HIP_TRY(hipMemcpyAsync(keys, p->keys, p->n_active * sizeof(unsigned long long), hipMemcpyDeviceToDevice, st));
    if (order)
        HIP_TRY(hipMemcpyAsync(order, p->order, p->n_active * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    return WG_OK;
}

int wg_plan_grid_order(const wg_plan *p, void *order2, void *stream) {
    if (!p || (!order2 && p->n_active > 0)) return WG_EINVAL;
    if (p->n_active == 0) return WG_OK;
    hipLaunchKernelGGL(k_stream_order, dim3((unsigned)grid_blocks(p->n_total, 256, 1 << 20)), dim3(256), 0,
                       (hipStream_t)stream, p->inv2, p->n_total, (uint32_t *)order2);
    LAUNCH_CHECK("k_stream_order");
    return WG_OK;
}

int wg_profiler_create(wg_profiler **out) {
    if (!out) return WG_EINVAL;
    *out = new (std::nothrow) wg_profiler();
    return *out ? WG_OK : WG_ENOMEM;
}

int wg_profiler_destroy(wg_profiler *p) {
    if (!p) return WG_OK;
    if (g_prof == p) g_prof = nullptr;
    p->drain();
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    delete p;
    return WG_OK;
}

int wg_profiler_attach(wg_profiler *p) {
    g_prof = p;
    return WG_OK;
}

int wg_profiler_read(wg_profiler *p, int kind, double *total_ms, int64_t *launches) {
    if (!p || kind < 0 || kind >= WG_KIND_COUNT) return WG_EINVAL;
    p->drain();
    if (total_ms) *total_ms = p->total_ms[kind];
    if (launches) *launches = p->launches[kind];
    return WG_OK;
}

int wg_profiler_reset(wg_profiler *p) {
    if (!p) return WG_EINVAL;
    p->drain();
    for (int k = 0; k < WG_KIND_COUNT; ++k) {
        p->total_ms[k] = 0.0;
        p->launches[k] = 0;
    }
    return WG_OK;
}

const char *wg_kernel_kind_name(int kind) {
    static const char *names[WG_KIND_COUNT] = {"grid", "degrid", "fft_rows_grid", "fft_cols_grid",
                                               "fft_rows_degrid", "fft_cols_degrid", "image", "vis"};
    return kind >= 0 && kind < WG_KIND_COUNT ? names[kind] : "unknown";
}

const char *wg_strerror(int code) {
    switch (code) {
        case WG_OK: return "ok";
        case WG_EINVAL: return "invalid argument";
        case WG_ENOMEM: return "out of device memory";
        case WG_EHIP: {
            static thread_local std::string s;
            s = "HIP error: " + g_last_hip;
            return s.c_str();
        }
        case WG_EUNSUPPORTED: return "unsupported request (no printed kernel reaches epsilon, or grid too large)";
        case WG_ESCRATCH: return "the plan's workspace exceeds the fixed scratch of wg_apply_noalloc";
        default: return "unknown error";
    }
}

int wg_grid_size(double sigma, int npix) {
    if (!(sigma > 1.0) || npix < 1) return WG_EINVAL;
    return grid_size(sigma, npix);
}

int wg_kernel_params(int alpha, double sigma, double *eps_k, double *beta, double *mu) {
    const KernelRow *r = find_row(alpha, sigma);
    if (!r) return WG_EINVAL;
    if (eps_k) *eps_k = r->eps;
    if (beta) *beta = r->beta;
    if (mu) *mu = r->mu;
    return WG_OK;
}

int wg_select_kernel(double epsilon, int precision, int do_wgridding, int npix_x, int npix_y, double pixsize_x,
                     double pixsize_y, int64_t n_vis, double wmin, double wmax, int *alpha, double *sigma) {
    if (!alpha || !sigma || npix_x < 1 || npix_y < 1 || !(pixsize_x > 0) || !(pixsize_y > 0)) return WG_EINVAL;
    if (precision != WG_F32 && precision != WG_F64) return WG_EINVAL;
    if (precision == WG_F32 && !(epsilon >= 1e-5)) return WG_EINVAL;
    if (precision == WG_F64 && !(epsilon > 2e-13)) return WG_EINVAL;
    if (select_kernel(epsilon, precision, do_wgridding ? 1 : 0, npix_x, npix_y, pixsize_x, pixsize_y, n_vis, wmin,
                      wmax, alpha, sigma, nullptr) != 0)
        return WG_EUNSUPPORTED;
    return WG_OK;
}

int wg_kernel_poly(int alpha, double sigma, int precision, double *coeffs, int cap, int *degree) {
    const KernelRow *r = find_row(alpha, sigma);
    if (!r || !degree) return WG_EINVAL;
    int deg = choose_degree(alpha, r->beta, r->mu, r->eps, precision);
    std::vector<double> c;
    kernel_poly(alpha, r->beta, r->mu, deg, c);
    *degree = deg;
    if (coeffs) {
        int n = std::min<int>(cap, (int)c.size());
        for (int i = 0; i < n; ++i) coeffs[i] = c[i];
    }
    return WG_OK;
}

int wg_kernel_search(int alpha, double sigma, double *beta, double *mu, double *eps) {
    if (alpha < 2 || alpha > 16 || !(sigma > 1.0 && sigma <= 4.0) || !beta || !mu) return WG_EINVAL;
    double b = *beta, m = *mu;
    const double e = kernel_search(alpha, sigma, &b, &m);
    *beta = b;
    *mu = m;
    if (eps) *eps = e;
    return WG_OK;
}

int wg_kernel_map_error(int alpha, double sigma, double beta, double mu, double *eps) {
    if (alpha < 2 || alpha > 16 || !(sigma > 1.0 && sigma <= 4.0) || !(beta > 0.0) || !(mu > 0.0) || !eps)
        return WG_EINVAL;
    *eps = map_error_sup(alpha, sigma, beta, mu);
    return WG_OK;
}

int wg_kernel_table(int index, int *alpha, double *sigma, double *eps, double *beta, double *mu, int *printed) {
    const std::vector<KernelRow> &t = planner_table();
    if (index < 0 || index >= (int)t.size()) return WG_EINVAL;
    const KernelRow &r = t[index];
    if (alpha) *alpha = r.alpha;
    if (sigma) *sigma = r.sigma;
    if (eps) *eps = r.eps;
    if (beta) *beta = r.beta;
    if (mu) *mu = r.mu;
    if (printed) *printed = is_printed(r.alpha, r.sigma) ? 1 : 0;
    return WG_OK;
}

int wg_kernel_psi(int alpha, double sigma, const double *k, int n, double *out) {
    const KernelRow *r = find_row(alpha, sigma);
    if (!r || (n > 0 && (!k || !out))) return WG_EINVAL;
    std::vector<double> qt, qw;
    psi_nodes(alpha, r->beta, r->mu, qt, qw);
    for (int i = 0; i < n; ++i) out[i] = psi_eval(k[i], qt, qw);
    return WG_OK;
}

}  // extern "C"
