// Launches of the split (four-step) u-axis FFT passes.
#include "fft_split.hpp"
#include "kernels_fft_split.hpp"

namespace wg {

namespace {
SplitGeom split_geom(const wg_plan *p) {
    SplitGeom sg;
    sg.nu = p->g.nu;
    sg.nv = p->g.nv;
    sg.npix_x = p->g.npix_x;
    sg.npix_y = p->g.npix_y;
    sg.S = p->split_S;
    sg.N1 = p->g.nu / p->split_S;
    sg.Q = p->split_Q;
    sg.do_w = p->g.do_w;
    sg.w0 = p->g.w0;
    sg.dw = p->g.dw;
    return sg;
}
constexpr int kColThreads = 256;   // workgroup of the N1-point passes
}  // namespace

// The (S, V) pairs the planner picks: FP32 (16, 1), (16, 2), (8, 4);
// FP64 (16, 1), (8, 2), (4, 4).
#define WG_SPLIT_CASES(R, LAUNCH)                                                  \
    switch (p->split_S * 8 + p->split_V) {                                         \
        case 16 * 8 + 1: LAUNCH(R, 16, 1); break;                                  \
        case 16 * 8 + 2: if constexpr (sizeof(R) == 4) { LAUNCH(R, 16, 2); } break; \
        case 8 * 8 + 4: if constexpr (sizeof(R) == 4) { LAUNCH(R, 8, 4); } break;   \
        case 8 * 8 + 2: if constexpr (sizeof(R) == 8) { LAUNCH(R, 8, 2); } break;   \
        case 4 * 8 + 4: if constexpr (sizeof(R) == 8) { LAUNCH(R, 4, 4); } break;   \
        default: break;                                                            \
    }

template <typename R> void split_rows_grid(const wg_plan *p, const Cx<R> *G, Cx<R> *Y, int np, hipStream_t st) {
    const SplitGeom sg = split_geom(p);
    const size_t lds = (size_t)fft_lds_len(sg.nv) * sizeof(Cx<R>);
#define LAUNCH(RR, SS, VV)                                                                                    \
    hipLaunchKernelGGL((k_rows_grid_split<RR, kSplitThreads, SS, VV>), dim3(sg.N1, np), dim3(kSplitThreads), \
                       lds, st, G, Y, sg, p->fft_v, (const Cx<RR> *)p->tw_v, (const Cx<RR> *)p->tw_u)
    WG_SPLIT_CASES(R, LAUNCH)
#undef LAUNCH
}

template <typename R>
void split_cols_grid(const wg_plan *p, const Cx<R> *Y, R *acc, int j_lo, int np, hipStream_t st) {
    const SplitGeom sg = split_geom(p);
    const int nqb = (sg.npix_y + sg.Q - 1) / sg.Q;
    const size_t lds = (size_t)fft_lds_len(sg.N1) * sg.Q * sizeof(Cx<R>) + (size_t)sg.N1 * sg.Q * sizeof(R);
    hipLaunchKernelGGL((k_cols_grid_split<R, kColThreads>), dim3(sg.S * nqb), dim3(kColThreads), lds, st, Y, acc,
                       p->nm1, sg, j_lo, np, p->fft_u1, (const Cx<R> *)p->tw_u1);
}

template <typename R>
void split_cols_degrid(const wg_plan *p, const R *itil, Cx<R> *Y, int j_lo, int np, hipStream_t st) {
    const SplitGeom sg = split_geom(p);
    const int nqb = (sg.npix_y + sg.Q - 1) / sg.Q;
    const size_t lds = (size_t)fft_lds_len(sg.N1) * sg.Q * sizeof(Cx<R>);
    hipLaunchKernelGGL((k_cols_degrid_split<R, kColThreads>), dim3(sg.S * nqb), dim3(kColThreads), lds, st, itil,
                       p->nm1, Y, sg, j_lo, np, p->fft_u1, (const Cx<R> *)p->tw_u1, (const Cx<R> *)p->tw_u);
}

template <typename R> void split_rows_degrid(const wg_plan *p, const Cx<R> *Y, Cx<R> *G, int np, hipStream_t st) {
    const SplitGeom sg = split_geom(p);
    const size_t lds = (size_t)fft_lds_len(sg.nv) * sizeof(Cx<R>);
#define LAUNCH(RR, SS, VV)                                                                                      \
    hipLaunchKernelGGL((k_rows_degrid_split<RR, kSplitThreads, SS, VV>), dim3(sg.N1, np), dim3(kSplitThreads), \
                       lds, st, Y, G, sg, p->fft_v, (const Cx<RR> *)p->tw_v)
    WG_SPLIT_CASES(R, LAUNCH)
#undef LAUNCH
}

#define WG_INSTANTIATE_SPLIT(R)                                                                 \
    template void split_rows_grid<R>(const wg_plan *, const Cx<R> *, Cx<R> *, int, hipStream_t); \
    template void split_cols_grid<R>(const wg_plan *, const Cx<R> *, R *, int, int, hipStream_t); \
    template void split_cols_degrid<R>(const wg_plan *, const R *, Cx<R> *, int, int, hipStream_t); \
    template void split_rows_degrid<R>(const wg_plan *, const Cx<R> *, Cx<R> *, int, hipStream_t);
WG_INSTANTIATE_SPLIT(float)
WG_INSTANTIATE_SPLIT(double)

}  // namespace wg
