/*
 * wgrid -- w-gridding radio-interferometry measurement operator for AMD
 * MI355X (gfx950), after Arras, Reinecke, Westermann & Ensslin,
 * "Efficient wide-field radio interferometry response" (arXiv:2010.10122).
 *
 * C ABI.  All array arguments are plain pointers: "device" means HIP device
 * memory of the current device, "host" means ordinary host memory.  Every
 * array is C-contiguous, row-major.  No call throws; every int-returning
 * call returns WG_OK (0) or a negative WG_E* code, and wg_strerror() turns a
 * code into text (for WG_EHIP it includes the last HIP error seen).
 *
 * Operators (Sect. 2, eq. 3; Sect. 3.1):
 *   degridding  R   : real image [npix_x][npix_y] -> visibilities [n_rows][n_chan]
 *                     d_k = sum_lm I_lm / n_lm exp(-2 pi i [u_k l + v_k m - w_k (n_lm - 1)])
 *   gridding    R^H : visibilities -> real image, the adjoint with the real part
 *                     taken (Sect. 5, direct adjoint; Sect. 5.1, adjointness)
 * computed approximately to a requested accuracy epsilon by w-gridding:
 * convolution with the modified ES kernel (eq. semicircle2) on an
 * oversampled uv grid and on a stack of w-planes, 2-D FFTs per plane,
 * w-screens and the correction 1/(n Psi) (eqs. R1-R3, Rad1-Rad2).
 *
 * Coordinates: pixel (p, q) has l = (p - npix_x/2) * pixsize_x and
 * m = (q - npix_y/2) * pixsize_y (Sect. 2, sets L and M); the x axis pairs
 * with u.  Effective coordinates are uvw[r] * freq[c] / 299792458 (Sect. 2).
 */
#ifndef WGRID_H
#define WGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define WG_OK            0
#define WG_EINVAL       -1   /* invalid argument (see each call)                      */
#define WG_ENOMEM       -2   /* an allocation failed                                  */
#define WG_EHIP         -3   /* a HIP runtime call or kernel launch failed            */
#define WG_EUNSUPPORTED -4   /* valid request outside what this library implements   */
#define WG_ESCRATCH     -5   /* workspace larger than the allocation-free scratch     */

/* Size of the fixed device scratch behind wg_apply_noalloc (per GPU). */
#define WG_SCRATCH_BYTES ((size_t)128 << 20)

/* ---- precision --------------------------------------------------------- */
#define WG_F32 0   /* complex64 visibilities, float32 image (epsilon >= 1e-5)      */
#define WG_F64 1   /* complex128 visibilities, float64 image (epsilon > 2e-13)     */

/* Optional caller allocator for device memory (e.g. a framework's caching
 * allocator).  alloc returns NULL on failure.  Both NULL -> hipMalloc/hipFree. */
typedef void *(*wg_alloc_fn)(void *ctx, size_t bytes);
typedef void (*wg_free_fn)(void *ctx, void *ptr);

typedef struct wg_plan wg_plan;   /* opaque, immutable after creation */

/* Plan description: the problem statement of the paper's interface
 * (Appendix B: uvw, freq, mask, npix, pixsize, epsilon, do_wstacking) plus
 * the precision the operator runs in. */
typedef struct {
    const double  *uvw;          /* device [n_rows][3], baseline coordinates in metres
                                    (may be NULL when n_rows == 0)                     */
    const double  *freq;         /* device [n_chan], channel frequencies in Hz (> 0)    */
    const uint8_t *mask;         /* device [n_rows][n_chan] or NULL; !=0 selects        */
    int64_t        n_rows;       /* >= 0                                                */
    int64_t        n_chan;       /* >= 1; n_rows * n_chan < 2^31                        */
    int            npix_x;       /* image size, even and >= 32 (Appendix B)             */
    int            npix_y;
    double         pixsize_x;    /* pixel size in radians, > 0                          */
    double         pixsize_y;
    double         epsilon;      /* requested accuracy (relative L2)                    */
    int            precision;    /* WG_F32 or WG_F64                                    */
    int            do_wgridding; /* 0: w treated as zero (narrow field), else w-gridding */
    int            alpha;        /* 0 = automatic; else force kernel support (4..16)    */
    double         sigma;        /* 0 = automatic; else force oversampling (a row of the
                                    planner's table, see wg_kernel_table)               */
    int            planes_per_batch; /* 0 = automatic; w-planes processed per batch,
                                        capped at alpha and at 8                        */
    int            column_transform; /* 0 = automatic; 1 = one pass (K whole columns
                                        per workgroup); 2 = four-step (N_u = n1 n2,
                                        two passes over 16-column panels).  Automatic
                                        takes the four-step where one pass would hold
                                        at most two columns per workgroup.  Results
                                        agree to rounding.                            */
    void          *stream;       /* hipStream_t used for plan construction (NULL = 0)   */
    wg_alloc_fn    alloc;        /* optional device allocator (both or neither)         */
    wg_free_fn     free;
    void          *alloc_ctx;
} wg_plan_desc;

/* Create a plan.  Chooses the kernel (alpha, sigma, beta, mu) from the
 * Appendix-A tables with the cost model of Sect. 4.1 unless forced, derives
 * the grid size N = good_size(ceil(sigma n)) (Sect. 2), the w-plane spacing
 * dw = 1/(2 sigma max|n-1|), the first plane w_o and the plane count N_w
 * (Sect. 2, eq. wcirc), builds the piecewise-polynomial kernel (Sect. 4.2),
 * the correction factors and the visibility index (Sect. 4.3) on the device.
 * Synchronises the stream a few times (w range, index sizes) and returns
 * when the plan is complete.
 * The uvw/freq/mask arrays are read during creation and again by every
 * apply call: they must stay alive and unchanged while the plan is used.
 * Errors: WG_EINVAL for NULL desc/out/uvw/freq, odd or < 32 npix, pixsize
 *   <= 0, epsilon outside (2e-13, 0.1] (FP64) or [1e-5, 0.1] (FP32), a forced
 *   (alpha, sigma) not in the tables, any pixel with l^2 + m^2 >= 1,
 *   n_rows * n_chan >= 2^31; WG_EUNSUPPORTED when no printed kernel reaches
 *   epsilon or the grid exceeds the FFT size limit; WG_ENOMEM, WG_EHIP. */
int wg_plan_create(const wg_plan_desc *desc, wg_plan **out);

/* Destroy a plan and release its device memory.  No apply call using the
 * plan may still be running on any stream.  Without allocator callbacks the
 * memory goes back through hipFree (which waits for the device); with them,
 * every block is handed to the free callback at once.  NULL is accepted. */
int wg_plan_destroy(wg_plan *plan);

/* Footprint of the plan wg_plan_create would build for desc, without
 * building it (for admission by memory: Sect. 4.3 index, Sect. 2 geometry).
 * Runs the w-range reduction on desc->stream and synchronises it once;
 * every other step is host planning.  Outputs (each may be NULL):
 *   plan_bytes       upper bound of wg_plan_bytes of the built plan
 *   peak_bytes       upper bound of the device bytes held while it is built
 *                    (plan_bytes plus the sort scratch)
 *   workspace_bytes  upper bound of wg_workspace_bytes (loose: the gridder's
 *                    partial-tile scratch depends on the binning; use the
 *                    built plan's exact figure to admit apply calls)
 * Errors as wg_plan_create (WG_EINVAL, WG_EUNSUPPORTED, WG_ENOMEM, WG_EHIP). */
int wg_plan_estimate(const wg_plan_desc *desc, size_t *plan_bytes, size_t *peak_bytes,
                     size_t *workspace_bytes);

/* Degridding (forward, eq. R3 with R1, R2): vis = wgt * R(dirty).
 *   dirty     device [npix_x][npix_y] float32 (WG_F32) or float64 (WG_F64)
 *   wgt       device [n_rows][n_chan] real of the same precision, or NULL;
 *             multiplies the output (Appendix B)
 *   vis       device [n_rows][n_chan] complex (interleaved re, im); fully
 *             overwritten, masked entries are set to 0
 *   workspace device scratch of at least wg_workspace_bytes(plan) bytes
 *   stream    hipStream_t (NULL = default stream); the call is asynchronous.
 *             Its kernels run on this stream and on a second stream the plan
 *             owns (the visibility kernels overlap the FFT passes of the
 *             neighbouring w-batch); the second stream forks from and joins
 *             back into this one, so the call is ordered on `stream` like a
 *             single-stream call, also under HIP graph capture.
 * Errors: WG_EINVAL for NULL plan/dirty/vis or a short workspace; WG_EHIP. */
int wg_degrid(const wg_plan *plan, const void *dirty, const void *wgt, void *vis,
              void *workspace, size_t workspace_bytes, void *stream);

/* Gridding (adjoint, eqs. Rad1-Rad2): dirty = Re R^H (wgt * vis).
 *   vis       device [n_rows][n_chan] complex; masked entries are ignored
 *   wgt       device real [n_rows][n_chan] or NULL; multiplies the input
 *   dirty     device [npix_x][npix_y] real; fully overwritten
 * Other arguments and errors as wg_degrid.  Concurrent calls on one plan are
 * safe when each uses its own workspace and output (their work on the
 * plan's second stream runs one call after the other). */
int wg_grid(const wg_plan *plan, const void *vis, const void *wgt, void *dirty,
            void *workspace, size_t workspace_bytes, void *stream);

/* Allocation-free apply, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operators, kernels and results as wg_degrid (adjoint = 0:
 * in = dirty image, out = visibilities) and wg_grid (adjoint != 0: in =
 * visibilities, out = dirty image), with the same layouts, weights and
 * masks, but the workspace is a fixed static device array of
 * WG_SCRATCH_BYTES per GPU instead of a caller buffer.  The call makes no
 * allocation of any kind; the first call on a device looks up that
 * device's scratch address once.  The plan's device must be current.
 * Every call on a GPU shares that GPU's scratch and leaves its contents
 * behind (each call clears what it needs): calls that overlap in time on one
 * GPU (different streams or host threads) race and give wrong results.
 * Errors: WG_ESCRATCH when wg_workspace_bytes(plan) > WG_SCRATCH_BYTES;
 * WG_EINVAL for NULL plan/in/out or another device current; WG_EHIP. */
int wg_apply_noalloc(const wg_plan *plan, int adjoint, const void *in, const void *wgt, void *out,
                     void *stream);

/* Plan summary (host struct, filled by wg_plan_info). */
typedef struct {
    int     alpha;            /* kernel support in cells                             */
    double  sigma, beta, mu;  /* oversampling and modified-ES parameters (App. A)     */
    double  eps_kernel;       /* tabulated kernel accuracy eps_k                      */
    int     poly_degree;      /* degree of the per-cell kernel polynomials            */
    int     nu, nv;           /* oversampled grid size (u pairs with x)               */
    int     nw;               /* number of w-planes                                   */
    double  dw, w0;           /* w-plane spacing and first plane (wavelengths)        */
    double  wmin, wmax;       /* range of |w| over selected visibilities              */
    int     npix_x, npix_y;
    int     precision, do_wgridding;
    int64_t n_rows, n_chan;
    int64_t n_vis;            /* selected (unmasked) visibilities                     */
    int     planes_per_batch; /* w-planes per batch in the apply pipeline             */
    int     tile;             /* uv tile edge of the index (cells)                    */
    double  bytes_grid;       /* algorithmic HBM bytes of one wg_grid call            */
    double  bytes_degrid;     /* algorithmic HBM bytes of one wg_degrid call          */
    double  predicted_seconds;/* cost-model estimate of one apply                     */
    size_t  plan_bytes;       /* device bytes held by the plan                        */
    size_t  index_bytes;      /* of which visibility index                            */
    size_t  workspace_bytes;  /* per apply call                                       */
    int64_t extra_items_grid; /* gridder work items beyond one per tile, all batches  */
    int64_t extra_items_degrid;/* likewise for the degridder                          */
    double  rounding_error;   /* estimated relative rounding error of one apply in the
                                 plan's precision: 1.2 ulp x amplification          */
    double  amplification;    /* rms over the image of Psi(0)/Psi: the factor by which
                                 the correction 1/(n Psi) (Sect. 2) magnifies errors
                                 made on the grid                                    */
    double  poly_error;       /* largest |polynomial - phi| over the alpha cells of the
                                 piecewise kernel (Sect. 4.2), evaluated in FP64      */
    int     column_transform; /* 1 = one pass, 2 = four-step (see wg_plan_desc)      */
    int     col_n1, col_n2;   /* four-step factors of nu (0 for one pass)             */
    int     col_k;            /* columns per workgroup of the one-pass form           */
} wg_plan_info_t;

int    wg_plan_info(const wg_plan *plan, wg_plan_info_t *info);
size_t wg_workspace_bytes(const wg_plan *plan);
size_t wg_plan_bytes(const wg_plan *plan);

/* Copy the visibility index (sorted order) into caller device buffers:
 *   keys  [n_vis] uint64: ((t_u * NTv + t_v) * nw + t_w), t_u = i_u/tile,
 *         t_v = i_v/tile, t_w = first w-plane of the visibility (Sect. 4.3)
 *   order [n_vis] uint32: linear index r*n_chan + c, ascending within a key.
 * Either pointer may be NULL.  Asynchronous on ``stream``. */
int wg_plan_index(const wg_plan *plan, void *keys, void *order, void *stream);

/* The gridder's own visibility order (derived from the index of Sect. 4.3):
 * order2[t] (device uint32 [n_vis]) = linear index r*n_chan + c of the
 * visibility at position t.  The order is by (tile, edge rank, first
 * plane): within a 16x16 tile, rank 0 = footprint inside the tile, 1 =
 * reaching the next tile along v only, 2 = along both u and v, 3 = along u
 * only (the next tile meaning the one with the tile index plus one, cyclic);
 * ties keep the index order.  Asynchronous on ``stream``. */
int wg_plan_grid_order(const wg_plan *plan, void *order2, void *stream);

const char *wg_strerror(int code);

/* ---- per-kernel timing ----------------------------------------------------
 * A profiler attached to the calling host thread brackets every kernel
 * launch of wg_grid / wg_degrid with a pair of HIP events on the launch
 * stream and accumulates the elapsed time per kernel kind.  Attaching adds
 * two event records per launch and runs every launch on the caller's stream
 * (the plan's second stream is left out, so each timed kernel runs alone);
 * it changes no result.  A profiler is
 * owned by the caller and must not be shared between host threads. */
#define WG_KIND_GRID             0   /* LDS-tile gridder                        */
#define WG_KIND_DEGRID           1   /* gather degridder                        */
#define WG_KIND_FFT_ROWS_GRID    2   /* gridding FFT pass 1 (rows)              */
#define WG_KIND_FFT_COLS_GRID    3   /* gridding FFT pass 2 + screen + accumulate */
#define WG_KIND_FFT_ROWS_DEGRID  4   /* degridding screen + FFT pass 1 (rows)   */
#define WG_KIND_FFT_COLS_DEGRID  5   /* degridding FFT pass 2 (columns)         */
#define WG_KIND_IMAGE            6   /* image-side correction and clearing      */
#define WG_KIND_VIS              7   /* visibility-side finishing and clearing  */
#define WG_KIND_COUNT            8

typedef struct wg_profiler wg_profiler;
int wg_profiler_create(wg_profiler **out);
int wg_profiler_destroy(wg_profiler *prof);
/* Attach prof to the calling host thread (NULL detaches). */
int wg_profiler_attach(wg_profiler *prof);
/* Totals for one kind since creation or the last reset; waits for the
 * recorded events to complete. */
int wg_profiler_read(wg_profiler *prof, int kind, double *total_ms, int64_t *launches);
int wg_profiler_reset(wg_profiler *prof);
const char *wg_kernel_kind_name(int kind);

/* ---- host-only helpers (no device needed) -------------------------------
 * These expose pieces of the host planner for inspection and testing. */

/* Smallest N >= ceil(sigma * npix) that is a multiple of the tile edge (16)
 * and has no prime factor above 7 (Sect. 2: N = ceil(sigma n), rounded up
 * for the FFT).  Returns N, or WG_EINVAL. */
int wg_grid_size(double sigma, int npix);

/* Modified-ES parameters of a row of the planner's table (Appendix A where
 * printed, else the searched row).  Returns WG_EINVAL when (alpha, sigma) is
 * not in the table. */
int wg_kernel_params(int alpha, double sigma, double *eps_k, double *beta, double *mu);

/* Kernel choice for a problem (Sect. 4.1): for each support the smallest
 * printed sigma with factor * eps_k <= epsilon (factor 3 with w-gridding,
 * 2 without), then the least predicted cost.  n_vis and the |w| range drive
 * the cost model.  Returns WG_OK, WG_EINVAL or WG_EUNSUPPORTED. */
int wg_select_kernel(double epsilon, int precision, int do_wgridding, int npix_x, int npix_y,
                     double pixsize_x, double pixsize_y, int64_t n_vis, double wmin,
                     double wmax, int *alpha, double *sigma);

/* Piecewise-polynomial kernel (Sect. 4.2): for cell i (0 <= i < alpha) and
 * z in [-1, 1] the kernel at t = -alpha/2 + i + (z + 1)/2 is
 * sum_d coeffs[i*(degree+1) + d] * z^d.  Fills at most cap doubles;
 * *degree receives the degree.  Interpolation at Chebyshev roots. */
int wg_kernel_poly(int alpha, double sigma, int precision, double *coeffs, int cap, int *degree);

/* Two-parameter kernel search of Sect. 3.2: the (beta, mu) of the modified
 * ES kernel (eq. semicircle2) that minimise the supremum over the retained
 * band 0 <= x <= 1/(2 sigma) of the map error function l(x) (eq. maperror),
 * for support alpha (2..16 cells) and oversampling sigma (1 < sigma <= 4).
 * On input, *beta and *mu > 0 add a starting point (e.g. the optimum of a
 * neighbouring sigma) to the search's own; 0 adds none.  eps (may be NULL)
 * receives the supremum at the result.  Host only; takes seconds.
 * Errors: WG_EINVAL. */
int wg_kernel_search(int alpha, double sigma, double *beta, double *mu, double *eps);

/* Supremum of the map error function (eq. maperror) over the retained band
 * for given kernel parameters (host only).  Errors: WG_EINVAL. */
int wg_kernel_map_error(int alpha, double sigma, double beta, double mu, double *eps);

/* Row `index` (0-based) of the planner's kernel table, sorted by alpha then
 * sigma: the printed Appendix-A rows and, for the (alpha, sigma) pairs the
 * paper does not print, rows of wg_kernel_search generated at build time.
 * printed receives 1 for an Appendix-A row.  Any output may be NULL.
 * Returns WG_EINVAL past the end. */
int wg_kernel_table(int index, int *alpha, double *sigma, double *eps, double *beta, double *mu, int *printed);

/* Fourier transform of the kernel, psi(k) = int phi(t) cos(2 pi k t) dt, at
 * n points (host arrays). */
int wg_kernel_psi(int alpha, double sigma, const double *k, int n, double *out);

#ifdef __cplusplus
}
#endif
#endif /* WGRID_H */
