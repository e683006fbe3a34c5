// Launches of the split (four-step) u-axis FFT passes; see
// kernels_fft_split.hpp.  Compiled in a translation unit of their own.
#pragma once
#include "plan_internal.hpp"

namespace wg {

constexpr int kSplitThreads = 1024;   // workgroup of the fused row passes

// Gridding: rows along v with the S-point u stage (G -> Y), then the
// N1-point u transforms with screen and image accumulation (Y -> acc).
template <typename R> void split_rows_grid(const wg_plan *p, const Cx<R> *G, Cx<R> *Y, int np, hipStream_t st);
template <typename R>
void split_cols_grid(const wg_plan *p, const Cx<R> *Y, R *acc, int j_lo, int np, hipStream_t st);
// Degridding: screened-image N1-point u transforms (itil -> Y), then the
// S-point u stage with the rows along v (Y -> G).
template <typename R>
void split_cols_degrid(const wg_plan *p, const R *itil, Cx<R> *Y, int j_lo, int np, hipStream_t st);
template <typename R> void split_rows_degrid(const wg_plan *p, const Cx<R> *Y, Cx<R> *G, int np, hipStream_t st);

#define WG_DECLARE_SPLIT(R)                                                                            \
    extern template void split_rows_grid<R>(const wg_plan *, const Cx<R> *, Cx<R> *, int, hipStream_t); \
    extern template void split_cols_grid<R>(const wg_plan *, const Cx<R> *, R *, int, int, hipStream_t); \
    extern template void split_cols_degrid<R>(const wg_plan *, const R *, Cx<R> *, int, int, hipStream_t); \
    extern template void split_rows_degrid<R>(const wg_plan *, const Cx<R> *, Cx<R> *, int, hipStream_t);
WG_DECLARE_SPLIT(float)
WG_DECLARE_SPLIT(double)
#undef WG_DECLARE_SPLIT

}  // namespace wg
