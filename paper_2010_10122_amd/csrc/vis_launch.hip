// Gridder and degridder launches of one kernel support, WG_ALPHA cells
// (set by the build, once per support).
#include "vis_launch.hpp"

#include <algorithm>

#ifndef WG_ALPHA
#error "build with -DWG_ALPHA=<support>"
#endif

namespace wg {

// blocks of a vis-kernel launch: the extra items (padded to a multiple of
// 8) and then one block per tile (padded likewise)
inline unsigned item_blocks(const wg_plan *p, uint32_t n_extra) {
    const int nt = p->g.ntu * p->g.ntv;
    return (unsigned)(((n_extra + 7) & ~7u) + (((unsigned)nt + 7) & ~7u));
}

template <typename R, int ALPHA> struct Launch {
    template <int PS>
    static void grid_mx(const wg_plan *p, const VisArgs<R> &va, int J, Cx<R> *G, Cx<R> *part, hipStream_t st) {
        const uint32_t ne = p->xg_off[J + 1] - p->xg_off[J];
        const size_t lds = GridStageMx1<R, ALPHA>::bytes;
        hipLaunchKernelGGL((k_grid_mx1<R, ALPHA, PS>), dim3(item_blocks(p, ne)), dim3(64), lds, st, va, J,
                           p->xg + p->xg_off[J], (int)ne, kGridItemCap, G, part);
    }
    static void grid(const wg_plan *p, const VisArgs<R> &va, int J, Cx<R> *G, Cx<R> *part, hipStream_t st) {
        // matrix cores in every case; with a single plane (no w term) 14 of
        // their 16 plane-value rows idle, and still the form measured faster
        // than register FMAs (Sect. 6.2 shape: FP64 339 against 462 ms, FP32
        // 55.7 against 69.0 ms a call)
        if (p->P > 4)
            grid_mx<8>(p, va, J, G, part, st);
        else
            grid_mx<4>(p, va, J, G, part, st);
        // partial tiles of split items, added in item order
        const uint32_t nr = p->xr_off[J + 1] - p->xr_off[J];
        if (nr > 0) {
            const int np = std::min(p->P, p->g.nw - J * p->P);
            hipLaunchKernelGGL(k_grid_reduce<R>, dim3(nr), dim3(kTileArea), 0, st, p->xr + p->xr_off[J], (int)nr,
                               p->P, np, p->g, (const Cx<R> *)part, G);
        }
    }
    static void degrid(const wg_plan *p, const VisArgs<R> &va, int J, const Cx<R> *G, Cx<R> *vacc,
                       hipStream_t st) {
        const uint32_t ne = p->xd_off[J + 1] - p->xd_off[J];
        const int W = kTileCells + ALPHA - 1;
        // planes staged at a time: about 20 KiB of tile + halo, so that
        // eight workgroups (32 waves) share a CU; the kernel values are
        // evaluated once per staged group (measured: 4 planes of 8 at a time
        // beat all 8 at once, 0.49 vs 0.57 ms)
        const int pd = std::max(1, std::min(p->P, (int)(20 * 1024 / ((size_t)W * W * sizeof(Cx<R>)))));
        const size_t lds = (((size_t)pd * W * W * sizeof(Cx<R>) + 15) & ~(size_t)15) + kCoefBytes<R, ALPHA>;
        hipLaunchKernelGGL((k_degrid<R, ALPHA>), dim3(item_blocks(p, ne)), dim3(256), lds, st, va, J, pd,
                           p->xd + p->xd_off[J], (int)ne, kDegridItemCap, G, vacc);
    }
};

template <typename R, int ALPHA>
void launch_vis(bool gridding, const wg_plan *p, const VisArgs<R> &va, int J, Cx<R> *G, Cx<R> *vacc, Cx<R> *part,
                hipStream_t st) {
    if (gridding) Launch<R, ALPHA>::grid(p, va, J, G, part, st);
    else Launch<R, ALPHA>::degrid(p, va, J, G, vacc, st);
}

template void launch_vis<float, WG_ALPHA>(bool, const wg_plan *, const VisArgs<float> &, int, float2 *, float2 *,
                                          float2 *, hipStream_t);
template void launch_vis<double, WG_ALPHA>(bool, const wg_plan *, const VisArgs<double> &, int, double2 *,
                                           double2 *, double2 *, hipStream_t);

}  // namespace wg
