// Host-side planner mathematics (no device code):
//   * the Appendix-A kernel tables (modified ES kernel, alpha in {4,7,8,12,16});
//   * FFT-friendly grid sizes (Sect. 2, N = ceil(sigma n));
//   * the kernel phi (eq. semicircle2) and its Fourier transform psi by
//     tanh-sinh quadrature (psi as used by eq. approxw, 2*pi*k convention);
//   * piecewise-polynomial kernel coefficients from interpolation at
//     Chebyshev roots (Sect. 4.2);
//   * the kernel-selection cost model (Sect. 4.1).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <vector>

namespace wg {

// Appendix A, "Kernel parameters": {alpha, sigma, eps, beta, mu}.
static const KernelRow kPrinted[] = {
    { 4, 1.15, 0.025654879, 1.3873426689, 0.5436851297},
    { 4, 1.2, 0.013809249, 1.3008419165, 0.5902137484},
    { 4, 1.25, 0.0085840685, 1.3274088935, 0.5953499486},
    { 4, 1.3, 0.0057322498, 1.3617063353, 0.5965631622},
    { 4, 1.35, 0.0042494419, 1.384549988, 0.5990241291},
    { 4, 1.4, 0.0033459552, 1.4405325088, 0.5924776015},
    { 4, 1.45, 0.0028187359, 1.4635220066, 0.5929442711},
    { 4, 1.5, 0.0023843943, 1.5539689162, 0.5772217314},
    { 4, 1.55, 0.0020343796, 1.5991008653, 0.5721765215},
    { 4, 1.6, 0.0017143851, 1.6581546365, 0.5644747137},
    { 4, 1.65, 0.0014730848, 1.7135331415, 0.5572788589},
    { 4, 1.7, 0.0012554492, 1.7464330378, 0.5548742415},
    { 4, 1.75, 0.0010610904, 1.7887326906, 0.5509877716},
    { 4, 1.8, 0.00090885567, 1.8122309426, 0.5502273972},
    { 4, 1.85, 0.0007757401, 1.8304451327, 0.550396716},
    { 4, 1.9, 0.0006740398, 1.8484487383, 0.5502376937},
    { 4, 1.95, 0.00058655391, 1.8742215688, 0.5489738941},
    { 4, 2.0, 0.00051911189, 1.90694363, 0.5468009434},
    { 7, 1.15, 0.00078476028, 1.5248706519, 0.5288306317},
    { 7, 1.2, 0.00027127166, 1.5739348793, 0.5287992619},
    { 7, 1.25, 0.00012594628, 1.6245240723, 0.527921777},
    { 7, 1.3, 7.0214545e-05, 1.6835745981, 0.5257484101},
    { 7, 1.35, 4.1972457e-05, 1.7343424414, 0.5239793844},
    { 7, 1.4, 2.378019e-05, 1.7845017738, 0.5224266045},
    { 7, 1.45, 1.3863408e-05, 1.8180597789, 0.5221834768},
    { 7, 1.5, 9.1605353e-06, 1.868082272, 0.5206277502},
    { 7, 1.55, 6.479159e-06, 1.9188980015, 0.5183134674},
    { 7, 1.6, 4.6544571e-06, 1.9536166143, 0.5178695891},
    { 7, 1.65, 3.5489761e-06, 1.9786267068, 0.5178430252},
    { 7, 1.7, 2.7030348e-06, 2.0027666534, 0.5178577604},
    { 7, 1.75, 2.0533894e-06, 2.0289949199, 0.5176300336},
    { 7, 1.8, 1.6069122e-06, 2.0596412946, 0.5167551932},
    { 7, 1.85, 1.2936794e-06, 2.0720606842, 0.5178747891},
    { 7, 1.9, 1.0768664e-06, 2.090898174, 0.5181009847},
    { 7, 1.95, 9.0890421e-07, 2.1086185697, 0.5184537843},
    { 7, 2.0, 7.7488775e-07, 2.1278284187, 0.5186377792},
    { 8, 1.15, 0.00026818611, 1.568124649, 0.5223052481},
    { 8, 1.2, 7.8028732e-05, 1.620926145, 0.5219287175},
    { 8, 1.25, 2.7460918e-05, 1.6851585171, 0.519925059},
    { 8, 1.3, 1.3421658e-05, 1.7442373315, 0.5182155619},
    { 8, 1.35, 7.5158217e-06, 1.7876782642, 0.5176319503},
    { 8, 1.4, 4.2472384e-06, 1.8294321912, 0.5171860211},
    { 8, 1.45, 2.5794802e-06, 1.871691821, 0.5161733611},
    { 8, 1.5, 1.6131994e-06, 1.9213040541, 0.5145350888},
    { 8, 1.55, 1.0974814e-06, 1.9637229131, 0.5134005827},
    { 8, 1.6, 7.531955e-07, 2.0002761373, 0.5128849282},
    { 8, 1.65, 5.5097346e-07, 2.0275645736, 0.5127082324},
    { 8, 1.7, 4.0136726e-07, 2.0498410409, 0.5130237662},
    { 8, 1.75, 2.906467e-07, 2.073158517, 0.5131757153},
    { 8, 1.8, 2.1834922e-07, 2.0907418726, 0.5136046561},
    { 8, 1.85, 1.6329905e-07, 2.1164552354, 0.5133333878},
    { 8, 1.9, 1.2828598e-07, 2.126157016, 0.5143004427},
    { 8, 1.95, 1.0171134e-07, 2.1363206613, 0.515235491},
    { 8, 2.0, 8.1881369e-08, 2.1397013368, 0.5166895497},
    {12, 1.15, 2.7535895e-06, 1.6661837519, 0.5098172147},
    {12, 1.2, 5.2570038e-07, 1.7294557459, 0.5089239596},
    {12, 1.25, 1.378658e-07, 1.7698182384, 0.5099240718},
    {12, 1.3, 4.4329167e-08, 1.8092042442, 0.510607427},
    {12, 1.35, 1.7038991e-08, 1.8619112597, 0.5093832337},
    {12, 1.4, 6.5438748e-09, 1.9069147481, 0.5089479889},
    {12, 1.45, 2.9874764e-09, 1.9318398074, 0.5098082325},
    {12, 1.5, 1.4920459e-09, 1.9628483155, 0.5100985753},
    {12, 1.55, 8.0989276e-10, 2.0129847811, 0.5085327805},
    {12, 1.6, 4.1660575e-10, 2.0517921747, 0.5079102398},
    {12, 1.65, 2.3539727e-10, 2.06983884, 0.5085131064},
    {12, 1.7, 1.3497289e-10, 2.0887365361, 0.5090417146},
    {12, 1.75, 8.3256938e-11, 2.106955733, 0.5095920671},
    {12, 1.8, 5.8834619e-11, 2.1359415217, 0.5091887069},
    {12, 1.9, 2.6412908e-11, 2.2006369514, 0.5075889699},
    {12, 1.95, 1.7189689e-11, 2.2146741638, 0.5080017404},
    {12, 2.0, 1.2174796e-11, 2.2431392199, 0.5075191177},
    {16, 1.3, 1.1509596e-10, 1.7892839755, 0.5122877693},
    {16, 1.35, 3.2440049e-11, 1.8914441282, 0.5063521839},
    {16, 1.4, 8.4329616e-12, 1.9296369098, 0.5065170208},
    {16, 1.45, 3.1161739e-12, 1.9674735425, 0.5063244338},
    {16, 1.5, 1.2100308e-12, 2.0130787701, 0.5055587965},
    {16, 1.55, 4.6082202e-13, 2.0438032614, 0.5056309683},
    {16, 1.6, 1.7883238e-13, 2.0329561822, 0.5089045671},
    {16, 1.65, 9.2853815e-14, 2.0494514743, 0.5103582604},
    {16, 1.7, 5.6614567e-14, 2.0925119791, 0.5083767402},
    {16, 1.75, 2.875391e-14, 2.1461524027, 0.5062037834},
    {16, 1.8, 1.6578982e-14, 2.1490040175, 0.508272183},
    {16, 1.85, 1.1782751e-14, 2.1811826814, 0.5072570059},
    {16, 1.9, 8.9196865e-15, 2.1981176583, 0.5075840871},
    {16, 1.95, 6.6530006e-15, 2.234001135, 0.5060133105},
    {16, 2.0, 5.0563492e-15, 2.2621631913, 0.5056924675},
};

// Rows of the library's own search of the map error (Sect. 3.2) for every
// support 4..16 and sigma 1.15..2.00, generated by gen_kernel_table.py.
static const KernelRow kSearched[] = {
#include "kernel_table_search.inc"
    {0, 0.0, 0.0, 0.0, 0.0}   // end marker
};

const int kSupports[kNumSupports] = {4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};

bool is_printed(int alpha, double sigma) {
    for (const KernelRow &r : kPrinted)
        if (r.alpha == alpha && std::fabs(r.sigma - sigma) < 1e-9) return true;
    return false;
}

// The planner's table: the printed rows, and the searched rows of the
// (alpha, sigma) pairs the paper does not print; sorted by alpha, then sigma.
const std::vector<KernelRow> &planner_table() {
    static const std::vector<KernelRow> table = [] {
        std::vector<KernelRow> t(std::begin(kPrinted), std::end(kPrinted));
        for (const KernelRow &r : kSearched)
            if (r.alpha > 0 && !is_printed(r.alpha, r.sigma)) t.push_back(r);
        std::sort(t.begin(), t.end(), [](const KernelRow &a, const KernelRow &b) {
            return a.alpha != b.alpha ? a.alpha < b.alpha : a.sigma < b.sigma;
        });
        return t;
    }();
    return table;
}

const KernelRow *find_row(int alpha, double sigma) {
    for (const KernelRow &r : planner_table())
        if (r.alpha == alpha && std::fabs(r.sigma - sigma) < 1e-9) return &r;
    return nullptr;
}

const KernelRow *smallest_feasible(int alpha, double eps, double factor) {
    for (const KernelRow &r : planner_table())
        if (r.alpha == alpha && factor * r.eps <= eps) return &r;   // rows ascend in sigma
    return nullptr;
}

int good_size(long long nmin) {
    if (nmin < 1) nmin = 1;
    long long n = ((nmin + kTile - 1) / kTile) * kTile;
    for (;; n += kTile) {
        long long m = n;
        for (int p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        if (m == 1) return (int)n;
    }
}

int grid_size(double sigma, int npix) { return good_size((long long)std::ceil(sigma * npix)); }

double es_kernel(double t, int alpha, double beta, double mu) {
    double x = 2.0 * t / alpha;
    double s = 1.0 - x * x;
    if (s < 0.0) return 0.0;
    return std::exp(alpha * beta * (std::pow(s, mu) - 1.0));
}

// Tanh-sinh quadrature on [0, alpha/2]: t = (alpha/4)(1 + tanh((pi/2) sinh(x))).
// The substitution clusters nodes at both ends, which absorbs the
// (alpha/2 - t)^mu behaviour of the kernel at the edge of its support.
void psi_nodes(int alpha, double beta, double mu, std::vector<double> &t, std::vector<double> &w) {
    const double h = 1.0 / 64.0;
    const double half = 0.5 * alpha;
    const double hp = 0.5 * M_PI;
    t.clear();
    w.clear();
    for (int k = -256; k <= 256; ++k) {
        double x = k * h;
        double sh = std::sinh(x), ch = std::cosh(x);
        double u = hp * sh;
        double th = std::tanh(u);
        double sech2 = 1.0 / (std::cosh(u) * std::cosh(u));
        double tt = 0.5 * half * (1.0 + th);
        double wt = 0.5 * half * hp * ch * sech2 * h;
        if (wt < 1e-300 || tt <= 0.0 || tt >= half) continue;
        t.push_back(tt);
        w.push_back(wt * es_kernel(tt, alpha, beta, mu));
    }
}

double psi_eval(double k, const std::vector<double> &t, const std::vector<double> &wphi) {
    // psi(k) = 2 int_0^{alpha/2} phi(t) cos(2 pi k t) dt; summed from the small
    // terms (edge) to the large ones for accuracy.
    long double acc = 0.0L;
    for (size_t i = t.size(); i-- > 0;) acc += (long double)wphi[i] * std::cos(2.0 * M_PI * k * t[i]);
    return (double)(2.0L * acc);
}

// Monomial coefficients, per cell, of the interpolant of the kernel through
// the degree+1 Chebyshev roots of the cell mapped to z in [-1, 1].
void kernel_poly(int alpha, double beta, double mu, int degree, std::vector<double> &coeffs) {
    const int n = degree + 1;
    coeffs.assign((size_t)alpha * n, 0.0);
    std::vector<long double> z(n), f(n), a(n);
    for (int j = 0; j < n; ++j) z[j] = std::cos(M_PI * (j + 0.5L) / n);
    for (int i = 0; i < alpha; ++i) {
        for (int j = 0; j < n; ++j) {
            double t = -0.5 * alpha + i + 0.5 * ((double)z[j] + 1.0);
            f[j] = es_kernel(t, alpha, beta, mu);
        }
        // Chebyshev coefficients by the discrete orthogonality at the roots
        for (int m = 0; m < n; ++m) {
            long double s = 0.0L;
            for (int j = 0; j < n; ++j) s += f[j] * std::cos((long double)M_PI * m * (j + 0.5L) / n);
            a[m] = s * 2.0L / n;
        }
        a[0] *= 0.5L;
        // expand sum_m a_m T_m(z) in powers of z via T_{m+1} = 2 z T_m - T_{m-1}
        std::vector<long double> tm1(n, 0.0L), tm(n, 0.0L), mono(n, 0.0L);
        tm1[0] = 1.0L;                      // T_0
        if (n > 1) tm[1] = 1.0L;            // T_1
        for (int d = 0; d < n; ++d) mono[d] += a[0] * tm1[d];
        if (n > 1)
            for (int d = 0; d < n; ++d) mono[d] += a[1] * tm[d];
        for (int m = 2; m < n; ++m) {
            std::vector<long double> tn(n, 0.0L);
            for (int d = 0; d < n; ++d) {
                long double v = -tm1[d];
                if (d > 0) v += 2.0L * tm[d - 1];
                tn[d] = v;
            }
            for (int d = 0; d < n; ++d) mono[d] += a[m] * tn[d];
            tm1 = tm;
            tm = tn;
        }
        for (int d = 0; d < n; ++d) coeffs[(size_t)i * n + d] = (double)mono[d];
    }
}

double kernel_poly_max_error(int alpha, double beta, double mu, int degree,
                             const std::vector<double> &coeffs) {
    const int n = degree + 1;
    double err = 0.0;
    for (int i = 0; i < alpha; ++i) {
        for (int s = 0; s <= 200; ++s) {
            double z = -1.0 + 2.0 * s / 200.0;
            double p = 0.0;
            for (int d = degree; d >= 0; --d) p = p * z + coeffs[(size_t)i * n + d];
            double t = -0.5 * alpha + i + 0.5 * (z + 1.0);
            err = std::max(err, std::fabs(p - es_kernel(t, alpha, beta, mu)));
        }
    }
    return err;
}

int choose_degree(int alpha, double beta, double mu, double eps_k, int precision) {
    // Degree alpha+3 is what Sect. 4.2 uses; take the lowest degree (at most
    // that) whose interpolation error stays an order below eps_k.
    // The edge cells carry the kernel's (alpha/2 - |t|)^mu behaviour, which
    // no polynomial follows closely; higher degrees do not help there, so the
    // search stops at the paper's alpha + 3 and keeps the most accurate degree.
    int top = alpha + 3;
    double target = eps_k / 20.0;
    if (precision == 0) target = std::max(target, 1e-7);
    int best = top;
    double best_err = 1e300;
    for (int d = std::max(3, alpha - 2); d <= top; ++d) {
        std::vector<double> c;
        kernel_poly(alpha, beta, mu, d, c);
        double e = kernel_poly_max_error(alpha, beta, mu, d, c);
        if (e <= target) return d;
        if (e < best_err) {
            best_err = e;
            best = d;
        }
    }
    return best;
}

double max_abs_nm1(int npix_x, int npix_y, double pixsize_x, double pixsize_y) {
    // largest |n - 1| over the pixel grid: the corner pixel (0, 0)
    double l = (double)(0 - npix_x / 2) * pixsize_x;
    double m = (double)(0 - npix_y / 2) * pixsize_y;
    double rho = l * l + m * m;
    double n = std::sqrt(1.0 - rho);
    return rho / (1.0 + n);
}

// Cost model (GPU form of Sect. 4.1).  Per apply: every w-plane moves its
// grid through HBM (gridder/degridder tile traffic plus the pruned two-pass
// FFT), and every visibility costs alpha^2 LDS updates per plane it touches.
// Rates are nominal MI355X figures (effective HBM and LDS-update throughput).
double predict_seconds(int alpha, double sigma, int precision, int do_w, int npix_x, int npix_y,
                       double max_nm1, int64_t n_vis, double wmin, double wmax) {
    // Mean time of one application (degridding and gridding averaged),
    // calibrated on this library's kernels with the wide-field workload
    // (2048^2, 92.9 million visibilities) over the kernels the planner
    // chose between 1e-4 and 1e-12:
    // * per w-plane: the plane traffic of the two FFT passes and of the
    //   visibility kernels, at an effective 4.0 TB/s (FP32) / 1.6 TB/s
    //   (FP64), plus launch tails;
    // * per visibility, with w-gridding: FP32 0.27 ns + 0.205 ps alpha^3,
    //   FP64 1.14 ps alpha^3 (the gather/accumulate over alpha^3 cells);
    //   without w: 1.4 ps (FP32) / 2.8 ps (FP64) alpha^2.
    const double sc = precision == 0 ? 8.0 : 16.0;
    const double sr = sc * 0.5;
    const double bw = precision == 0 ? 4.0e12 : 1.6e12;
    const double per_plane_overhead = 2e-6;
    int nu = grid_size(sigma, npix_x), nv = grid_size(sigma, npix_y);
    double nw = 1.0;
    if (do_w) {
        double dw = 1.0 / (2.0 * sigma * max_nm1);
        nw = std::ceil((wmax - wmin) / dw) + alpha;
    }
    double plane_bytes = (double)nu * nv * sc * 2.0 + (double)nu * npix_y * sc * 2.0 +
                         2.0 * (double)npix_x * npix_y * sr;
    double t_planes = nw * (plane_bytes / bw + per_plane_overhead);
    const double a2 = (double)alpha * alpha, a3 = a2 * alpha;
    double per_vis;
    if (do_w) per_vis = precision == 0 ? 2.7e-10 + 2.05e-13 * a3 : 1.14e-12 * a3;
    else per_vis = (precision == 0 ? 1.4e-12 : 2.8e-12) * a2;
    return t_planes + (double)n_vis * per_vis;
}

// Root-mean-square over the image of Psi(0)/Psi(l, m): the factor by which
// the correction 1/(n Psi) magnifies the rounding noise of the gridded planes
// and of the FFTs (largest towards the image corners, where all three kernel
// transforms approach the edge of the retained band).  Sampled at the
// centres of a 32 x 32 partition of the image.
double rounding_amplification(int alpha, double sigma, int do_w, int npix_x, int npix_y, double px,
                              double py) {
    const KernelRow *r = find_row(alpha, sigma);
    if (!r) return std::numeric_limits<double>::infinity();
    std::vector<double> t, w;
    psi_nodes(alpha, r->beta, r->mu, t, w);
    const double p0 = psi_eval(0.0, t, w);
    const int nu = grid_size(sigma, npix_x), nv = grid_size(sigma, npix_y);
    const double dw = do_w ? 1.0 / (2.0 * sigma * max_abs_nm1(npix_x, npix_y, px, py)) : 0.0;
    const int S = 32;
    std::vector<double> ix(S), iy(S), psx(S), psy(S);
    for (int i = 0; i < S; ++i) {
        ix[i] = std::floor((i + 0.5) * npix_x / S) - npix_x / 2;
        iy[i] = std::floor((i + 0.5) * npix_y / S) - npix_y / 2;
        psx[i] = psi_eval(ix[i] / nu, t, w) / p0;
        psy[i] = psi_eval(iy[i] / nv, t, w) / p0;
    }
    double acc = 0.0;
    for (int i = 0; i < S; ++i) {
        for (int j = 0; j < S; ++j) {
            double ps = psx[i] * psy[j];
            if (do_w) {
                double l = ix[i] * px, m = iy[j] * py;
                double rho = l * l + m * m;
                double nm1 = -rho / (1.0 + std::sqrt(1.0 - rho));
                ps *= psi_eval(nm1 * dw, t, w) / p0;
            }
            acc += 1.0 / (ps * ps);
        }
    }
    return std::sqrt(acc / (S * S));
}

// Rounding error of one apply relative to the result's norm: measured on
// MI355X at 0.2-1.1 unit roundoffs times the amplification above, over all
// printed supports in both precisions; 1.2 is taken as the bound.
double rounding_error(int alpha, double sigma, int precision, int do_w, int npix_x, int npix_y, double px,
                      double py) {
    const double ulp = precision == 0 ? 5.96e-8 : 1.11e-16;
    return 1.2 * ulp * rounding_amplification(alpha, sigma, do_w, npix_x, npix_y, px, py);
}

// ---- kernel-parameter search (Sect. 3.2) --------------------------------
// Map error function of eq. (maperror): for a frequency x in grid units
// (|x| <= 1/(2 sigma) is the retained band),
//   l(x)^2 = int_0^1 | 1 - sum_{a in U(nu)} phi(a - nu) e^{2 pi i (a - nu) x} / psi(x) |^2 dnu,
// where U(nu) are the alpha cells the kernel of a point at fractional
// position nu touches (a = ceil(nu - alpha/2) + i).  The set U changes at
// nu = frac(alpha/2), so the nu integral is split there; each piece uses
// tanh-sinh nodes, which follow the (alpha/2 - |t|)^mu edge behaviour of
// the kernel.  psi by the planner's own tanh-sinh quadrature (psi_nodes).
namespace {
struct NuRule {
    std::vector<double> nu, w;
};
NuRule nu_rule(int alpha) {
    NuRule r;
    const double brk = std::fmod(0.5 * alpha, 1.0);
    std::vector<std::pair<double, double>> segs;
    if (brk == 0.0) segs.push_back({0.0, 1.0});
    else {
        segs.push_back({0.0, brk});
        segs.push_back({brk, 1.0});
    }
    const double h = 1.0 / 12.0;
    for (auto sg : segs) {
        const double a = sg.first, b = sg.second, c = 0.5 * (a + b), hw = 0.5 * (b - a);
        for (int k = -48; k <= 48; ++k) {
            const double x = k * h;
            const double u = 0.5 * M_PI * std::sinh(x);
            const double t = std::tanh(u);
            const double wt = h * 0.5 * M_PI * std::cosh(x) / (std::cosh(u) * std::cosh(u));
            if (wt < 1e-18 || std::fabs(t) >= 1.0) continue;
            r.nu.push_back(c + hw * t);
            r.w.push_back(hw * wt);
        }
    }
    return r;
}
}  // namespace

double map_error(double x, int alpha, double beta, double mu, const std::vector<double> &qt,
                 const std::vector<double> &qw) {
    static thread_local int cached_alpha = -1;
    static thread_local NuRule rule;
    if (cached_alpha != alpha) {
        rule = nu_rule(alpha);
        cached_alpha = alpha;
    }
    const double ps = psi_eval(x, qt, qw);
    double acc = 0.0;
    for (size_t k = 0; k < rule.nu.size(); ++k) {
        const double nu = rule.nu[k];
        const double a0 = std::ceil(nu - 0.5 * alpha);
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < alpha; ++i) {
            const double off = a0 + i - nu;                      // a - nu in [-alpha/2, alpha/2)
            const double ph = es_kernel(off, alpha, beta, mu);
            const double ang = 2.0 * M_PI * off * x;
            sr += ph * std::cos(ang);
            si += ph * std::sin(ang);
        }
        const double dr = 1.0 - sr / ps, di = -si / ps;
        acc += rule.w[k] * (dr * dr + di * di);
    }
    return std::sqrt(acc);
}

double map_error_sup(int alpha, double sigma, double beta, double mu, bool refine) {
    std::vector<double> qt, qw;
    psi_nodes(alpha, beta, mu, qt, qw);
    const double xmax = 0.5 / sigma;
    // l(x) oscillates faster for wider kernels: the reported value samples
    // the band more densely than the search's cheaper objective
    const int nx = refine ? std::max(160, 48 * alpha) : 160;
    std::vector<double> xs(nx + 1), ls(nx + 1);
    for (int i = 0; i <= nx; ++i) {
        xs[i] = xmax * i / nx;
        ls[i] = map_error(xs[i], alpha, beta, mu, qt, qw);
    }
    // The minimax optimum equioscillates, so every local maximum of the
    // samples is refined, not only the largest one: by golden section on its
    // bracket (refine), else by the vertex of the parabola through the peak
    // sample and its neighbours (the search's cheaper objective).
    double top = 0.0;
    for (int i = 0; i <= nx; ++i) {
        top = std::max(top, ls[i]);
        const bool peak = (i == 0 || ls[i] >= ls[i - 1]) && (i == nx || ls[i] >= ls[i + 1]);
        if (!peak) continue;
        if (!refine) {
            if (i > 0 && i < nx) {
                const double c = 2.0 * ls[i] - ls[i - 1] - ls[i + 1];
                const double d = ls[i + 1] - ls[i - 1];
                if (c > 0.0) top = std::max(top, ls[i] + d * d / (8.0 * c));
            }
            continue;
        }
        double lo = xs[std::max(0, i - 1)], hi = xs[std::min(nx, i + 1)];
        const double g = 0.5 * (std::sqrt(5.0) - 1.0);
        double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
        double f1 = map_error(x1, alpha, beta, mu, qt, qw), f2 = map_error(x2, alpha, beta, mu, qt, qw);
        for (int it = 0; it < 24; ++it) {
            if (f1 > f2) {
                hi = x2; x2 = x1; f2 = f1; x1 = hi - g * (hi - lo); f1 = map_error(x1, alpha, beta, mu, qt, qw);
            } else {
                lo = x1; x1 = x2; f1 = f2; x2 = lo + g * (hi - lo); f2 = map_error(x2, alpha, beta, mu, qt, qw);
            }
        }
        top = std::max(top, std::max(f1, f2));
    }
    return top;
}

// Two-parameter search of Sect. 3.2: (beta, mu) minimising the supremum of
// l(x) over the retained band, for a given support and oversampling.  A
// coarse grid over the range the printed tables occupy (plus an optional
// caller start, e.g. the optimum of the neighbouring sigma), then
// Nelder-Mead on log sup l, restarted from its own result with a fresh
// simplex until a restart no longer improves (the objective is a maximum of
// equioscillating peaks, not smooth, and a single simplex can stall).
namespace {
double nelder_mead(const std::function<double(double, double)> &f, double &b, double &m, double fb, double db,
                   double dm) {
    double P[3][2] = {{b, m}, {b + db, m}, {b, m + dm}};
    double F[3] = {fb, f(P[1][0], P[1][1]), f(P[2][0], P[2][1])};
    for (int it = 0; it < 200; ++it) {
        int o[3] = {0, 1, 2};
        std::sort(o, o + 3, [&](int x, int y) { return F[x] < F[y]; });
        const int lo = o[0], mid = o[1], hi = o[2];
        if (std::fabs(F[hi] - F[lo]) < 1e-7 && std::fabs(P[hi][0] - P[lo][0]) + std::fabs(P[hi][1] - P[lo][1]) < 1e-6)
            break;
        const double c0 = 0.5 * (P[lo][0] + P[mid][0]), c1 = 0.5 * (P[lo][1] + P[mid][1]);
        const double r0 = 2.0 * c0 - P[hi][0], r1 = 2.0 * c1 - P[hi][1];
        const double fr = f(r0, r1);
        if (fr < F[lo]) {
            const double e0 = 3.0 * c0 - 2.0 * P[hi][0], e1 = 3.0 * c1 - 2.0 * P[hi][1];
            const double fe = f(e0, e1);
            if (fe < fr) { P[hi][0] = e0; P[hi][1] = e1; F[hi] = fe; }
            else { P[hi][0] = r0; P[hi][1] = r1; F[hi] = fr; }
        } else if (fr < F[mid]) {
            P[hi][0] = r0; P[hi][1] = r1; F[hi] = fr;
        } else {
            const double k0 = 0.5 * (c0 + P[hi][0]), k1 = 0.5 * (c1 + P[hi][1]);
            const double fk = f(k0, k1);
            if (fk < F[hi]) { P[hi][0] = k0; P[hi][1] = k1; F[hi] = fk; }
            else {
                for (int j : {mid, hi}) {
                    P[j][0] = 0.5 * (P[j][0] + P[lo][0]);
                    P[j][1] = 0.5 * (P[j][1] + P[lo][1]);
                    F[j] = f(P[j][0], P[j][1]);
                }
            }
        }
    }
    int best = 0;
    for (int j = 1; j < 3; ++j) if (F[j] < F[best]) best = j;
    b = P[best][0];
    m = P[best][1];
    return F[best];
}
}  // namespace

double kernel_search(int alpha, double sigma, double *beta, double *mu) {
    auto f = [&](double b, double m) {
        if (!(b > 0.3 && b < 4.0 && m > 0.2 && m < 1.0)) return 1e300;
        return std::log(map_error_sup(alpha, sigma, b, m, false));
    };
    struct Start { double f, b, m; };
    std::vector<Start> starts;
    for (double b = 1.1; b <= 2.6 + 1e-9; b += 0.1)
        for (double m = 0.47; m <= 0.62 + 1e-9; m += 0.025) starts.push_back({f(b, m), b, m});
    std::sort(starts.begin(), starts.end(), [](const Start &x, const Start &y) { return x.f < y.f; });
    starts.resize(std::min<size_t>(starts.size(), 2));
    if (*beta > 0.0 && *mu > 0.0) starts.push_back({f(*beta, *mu), *beta, *mu});
    double bf = 1e300, bb = 0.0, bm = 0.0;
    for (const Start &st : starts) {
        double b = st.b, m = st.m, fb = st.f;
        for (int restart = 0; restart < 6; ++restart) {
            const double fn = nelder_mead(f, b, m, fb, 0.03 / (1 + restart), 0.006 / (1 + restart));
            const bool better = fn < fb - 1e-6;
            fb = std::min(fb, fn);
            if (!better) break;
        }
        if (fb < bf) { bf = fb; bb = b; bm = m; }
    }
    *beta = bb;
    *mu = bm;
    return map_error_sup(alpha, sigma, bb, bm, true);
}

int select_kernel(double eps, int precision, int do_w, int npix_x, int npix_y, double px,
                  double py, int64_t n_vis, double wmin, double wmax, int *alpha,
                  double *sigma, double *seconds) {
    const double factor = do_w ? 3.0 : 2.0;
    double mn = max_abs_nm1(npix_x, npix_y, px, py);
    double best = std::numeric_limits<double>::infinity();
    int ba = 0;
    double bs = 0.0;
    const int npmax = npix_x > npix_y ? npix_x : npix_y;
    for (int a : kSupports) {
        // smallest printed sigma whose kernel error plus the estimated
        // rounding error of this precision stays within eps
        const KernelRow *r = nullptr;
        const KernelRow *end = planner_table().data() + planner_table().size();
        for (const KernelRow *c = smallest_feasible(a, eps, factor); c && c < end && c->alpha == a; ++c) {
            if (factor * c->eps + rounding_error(a, c->sigma, precision, do_w, npix_x, npix_y, px, py) <= eps) {
                r = c;
                break;
            }
        }
        if (!r) continue;
        if (grid_size(r->sigma, npmax) > max_grid(precision)) continue;
        double t = predict_seconds(a, r->sigma, precision, do_w, npix_x, npix_y, mn, n_vis, wmin, wmax);
        if (t < best) {
            best = t;
            ba = a;
            bs = r->sigma;
        }
    }
    if (!ba) return -1;
    *alpha = ba;
    *sigma = bs;
    if (seconds) *seconds = best;
    return 0;
}

}  // namespace wg
