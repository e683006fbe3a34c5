// Host-side planner mathematics; see host_math.cpp.
#pragma once
#include <cstdint>
#include <vector>

namespace wg {

constexpr int kTile = 16;          // uv tile edge of the visibility index (Sect. 4.3)
constexpr int kNumSupports = 13;   // supports 4..16 (printed rows of Appendix A, searched rows otherwise)
// Largest grid edge per precision: one strided transform line of K >= 1
// columns must fit the column-pass workgroup (FP32 12288, FP64 6144 values).
constexpr int kMaxGridF32 = 12288;
constexpr int kMaxGridF64 = 6144;
inline int max_grid(int precision) { return precision == 0 ? kMaxGridF32 : kMaxGridF64; }
extern const int kSupports[kNumSupports];

struct KernelRow {
    int alpha;
    double sigma, eps, beta, mu;
};

const std::vector<KernelRow> &planner_table();
bool is_printed(int alpha, double sigma);
const KernelRow *find_row(int alpha, double sigma);
const KernelRow *smallest_feasible(int alpha, double eps, double factor);
int good_size(long long nmin);
int grid_size(double sigma, int npix);
double es_kernel(double t, int alpha, double beta, double mu);
void psi_nodes(int alpha, double beta, double mu, std::vector<double> &t, std::vector<double> &wphi);
double psi_eval(double k, const std::vector<double> &t, const std::vector<double> &wphi);
void kernel_poly(int alpha, double beta, double mu, int degree, std::vector<double> &coeffs);
double kernel_poly_max_error(int alpha, double beta, double mu, int degree,
                             const std::vector<double> &coeffs);
int choose_degree(int alpha, double beta, double mu, double eps_k, int precision);
double max_abs_nm1(int npix_x, int npix_y, double pixsize_x, double pixsize_y);
double predict_seconds(int alpha, double sigma, int precision, int do_w, int npix_x, int npix_y,
                       double max_nm1, int64_t n_vis, double wmin, double wmax);
double rounding_amplification(int alpha, double sigma, int do_w, int npix_x, int npix_y, double px,
                              double py);
double rounding_error(int alpha, double sigma, int precision, int do_w, int npix_x, int npix_y, double px,
                      double py);
double map_error(double x, int alpha, double beta, double mu, const std::vector<double> &qt,
                 const std::vector<double> &qw);
double map_error_sup(int alpha, double sigma, double beta, double mu, bool refine = true);
double kernel_search(int alpha, double sigma, double *beta, double *mu);
int select_kernel(double eps, int precision, int do_w, int npix_x, int npix_y, double px,
                  double py, int64_t n_vis, double wmin, double wmax, int *alpha, double *sigma,
                  double *seconds);

}  // namespace wg
