// Gridder / degridder launches per kernel support.  Each support's kernels
// are compiled in a translation unit of their own (vis_launch.hip built with
// -DWG_ALPHA=N), so that the thirteen supports build in parallel.
#pragma once
#include "kernels_apply.hpp"
#include "plan_internal.hpp"

namespace wg {

// Run the gridder (gridding = true: scatter the batch's visibilities onto
// its planes, eq. Rad2) or the degridder (gather from the planes into the
// visibility accumulators, eq. R3) for batch J of plan p on stream st.
template <typename R, int ALPHA>
void launch_vis(bool gridding, const wg_plan *p, const VisArgs<R> &va, int J, Cx<R> *G, Cx<R> *vacc, Cx<R> *part,
                hipStream_t st);

#define WG_DECLARE_SUPPORT(A)                                                                                \
    extern template void launch_vis<float, A>(bool, const wg_plan *, const VisArgs<float> &, int, float2 *,  \
                                              float2 *, float2 *, hipStream_t);                               \
    extern template void launch_vis<double, A>(bool, const wg_plan *, const VisArgs<double> &, int, double2 *, \
                                               double2 *, double2 *, hipStream_t);
WG_DECLARE_SUPPORT(4) WG_DECLARE_SUPPORT(5) WG_DECLARE_SUPPORT(6) WG_DECLARE_SUPPORT(7) WG_DECLARE_SUPPORT(8)
WG_DECLARE_SUPPORT(9) WG_DECLARE_SUPPORT(10) WG_DECLARE_SUPPORT(11) WG_DECLARE_SUPPORT(12) WG_DECLARE_SUPPORT(13)
WG_DECLARE_SUPPORT(14) WG_DECLARE_SUPPORT(15) WG_DECLARE_SUPPORT(16)
#undef WG_DECLARE_SUPPORT

}  // namespace wg
