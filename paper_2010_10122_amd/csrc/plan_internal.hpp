// Internal declarations shared by the translation units of libwgrid: the
// plan object behind the opaque wg_plan handle and its device-memory
// bookkeeping.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <unordered_map>
#include <mutex>
#include <vector>

#include "../../include/wgrid.h"
#include "device_common.hpp"
#include "fft_lds.hpp"

namespace wg {

// Device allocations of one plan, through the caller's allocator if given.
struct DevMem {
    wg_alloc_fn alloc = nullptr;
    wg_free_fn free = nullptr;
    void *ctx = nullptr;
    size_t total = 0;                          // bytes currently held
    std::unordered_map<void *, size_t> sizes;
    void *get(size_t bytes) {
        if (bytes == 0) bytes = 16;
        void *p = nullptr;
        if (alloc) {
            p = alloc(ctx, bytes);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p) {
            total += bytes;
            sizes[p] = bytes;
        }
        return p;
    }
    void put(void *p) {
        if (!p) return;
        auto it = sizes.find(p);
        if (it != sizes.end()) {
            total -= it->second;
            sizes.erase(it);
        }
        if (free) free(ctx, p);
        else (void)hipFree(p);
    }
    // every allocation still held (plan teardown, and the error paths of
    // plan construction, which may stop between an allocation and its release)
    void release_all() {
        for (auto &kv : sizes) {
            if (free) free(ctx, kv.first);
            else (void)hipFree(kv.first);
        }
        sizes.clear();
        total = 0;
    }
    ~DevMem() { release_all(); }
};

}  // namespace wg

struct wg_plan {
    wg_plan_desc desc;
    wg::DevMem mem;
    hipStream_t stream = nullptr;
    int device = 0;
    // kernel
    int alpha = 0, degree = 0, precision = 0, do_w = 0;
    double sigma = 0, beta = 0, mu = 0, eps_k = 0;
    double poly_err = 0;      // largest |polynomial - kernel| over the cells (FP64 evaluation)
    double amp = 0;           // rms over the image of Psi(0) / Psi (rounding amplification)
    double round_err = 0;     // estimated relative rounding error of one apply
    // geometry
    wg::Geom g{};
    int P = 1, NJ = 1;
    int64_t n_total = 0, n_active = 0;
    double wmin = 0, wmax = 0, predicted = 0;
    wg::FftDesc fft_u{}, fft_v{};
    int k_cols = 1;     // columns per workgroup in the strided passes
    int k_cols_d = 1;   // the same for the degridding column pass
    // four-step column transform (N_u = n1 n2) in place of the one-pass
    // column transforms, with its two sub-length transforms and tables
    int col4 = 0, n1 = 0, n2 = 0;
    wg::FftDesc fft_n1{}, fft_n2{};
    void *tw_n1 = nullptr, *tw_n2 = nullptr;   // complex R
    // device arrays
    double *scale = nullptr;           // [n_chan]
    void *coef = nullptr;              // [degree+1][alpha] R
    void *tw_u = nullptr, *tw_v = nullptr;   // complex R
    double *nm1 = nullptr, *corr = nullptr;  // [npix_x][npix_y]
    unsigned long long *keys = nullptr;
    uint32_t *order = nullptr;
    uint32_t *tab_lo = nullptr, *tab_hi = nullptr;
    void *zc = nullptr;                // [n_active][3] R: kernel-local coordinates
    int2 *anc = nullptr;               // [n_active] anchors and fold bit
    uint32_t *inv = nullptr;           // [n_total] sorted position | fold << 31, ~0 if masked
    // gridder stream: the same visibilities ordered by (tile, edge rank,
    // first plane), with its (tile * 4 + rank, batch) range tables
    uint32_t *tab2_lo = nullptr, *tab2_hi = nullptr;   // [tiles * 4][NJ+1]
    void *zc2 = nullptr;               // [n_active][3] R
    int2 *anc2 = nullptr;              // [n_active]
    uint32_t *inv2 = nullptr;          // [n_total] stream position | fold << 31, ~0 if masked
    // extra work items per batch (lists longer than the item cap); offsets into
    // the device lists, [NJ + 1] each
    std::vector<uint32_t> xg_off, xd_off, xr_off;
    int4 *xg = nullptr, *xd = nullptr, *xr = nullptr;
    int max_slots = 0;                 // partial tiles of the gridder in one batch
    size_t index_bytes = 0;
    size_t ws_bytes = 0;
    // workspace layout (byte offsets)
    size_t off_G = 0, off_G2 = 0, off_T = 0, off_Y = 0, off_acc = 0, off_vacc = 0, off_itil = 0, off_part = 0;
    // the two-stream apply pipeline: a side stream for the visibility
    // kernels and its events (created with the plan), and a lock that keeps
    // one call's enqueue sequence whole when several host threads share the
    // plan
    hipStream_t side = nullptr;
    hipEvent_t ev[6] = {};
    mutable std::mutex enqueue_mu;
};
