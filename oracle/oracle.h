/* FP64 reference of the reverse ray tracer: test infrastructure only.
 * Declarations of the functions defined in oracle.c (see that file for the
 * sections of the paper each one follows). */
#ifndef RRT_ORACLE_H
#define RRT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
void orc_kernel_constants(double* out4);
double orc_Gt(double r, double h);
double orc_M4(double r, double h);
double orc_chord_closed(double h, double b, double z1, double z2);
double orc_chord_quad(double h, double b2, double z1, double z2, double rtol);
void orc_gk15_poly(double p, double a, double b, double* k15, double* err);
double orc_kernel_norm(double h, int32_t which);
int orc_columns(int64_t n, const float* pos, const float* h, const float* mu, const double* x,
                int32_t n_ray, const double* dirs, double L, double box,
                int64_t n_src, const int64_t* src, double rtol, int32_t mode,
                double* N_out, int64_t* row_hits, const int64_t* row_off,
                int32_t* hit_j, int32_t* hit_img, double* hit_fac, int32_t n_threads);
int orc_columns_near_far(int64_t n, const float* pos, const float* h, const float* mu,
                         const double* x, int32_t n_ray, const double* dirs, double L, double box,
                         int64_t n_src, const int64_t* src, double rtol, double* N_far,
                         double* N_near, int64_t* near_hits, int32_t n_threads);
double orc_x_evolve(double x0, double Gamma, double nH, double alpha, double gcoll, double t);
double orc_slab_lnG(double lnG0, double nH, double alpha, double gcoll, double sigma, double N);
double orc_slab_lnG_poly(int32_t n_bins, const double* sigma, const double* w, double N_far,
                         double nH, double alpha, double gcoll, double N_near);
void orc_gamma_near_far_poly(int64_t n_src, int32_t n_ray, const double* N_far,
                             const double* N_near, int32_t n_bins, const double* sigma,
                             const double* w, const double* nH, const double* alpha,
                             const double* gcoll, double* lnG, int32_t n_threads, int32_t share);
void orc_gamma_near_far(int64_t n_src, int32_t n_ray, const double* N_far, const double* N_near,
                        double w, double sigma, const double* nH, const double* alpha,
                        const double* gcoll, double* lnG, int32_t share);
void orc_gamma(int64_t n_src, int32_t n_ray, const double* N, int32_t n_bins,
               const double* sigma, const double* w, double* lnG, double* G, double* tau);
double orc_alpha_A(double T);
double orc_alpha_B(double T);
double orc_gamma_coll(double T);
double orc_xeq(double Gamma, double nH, double alpha, double gcoll, double y);
int orc_solve(int64_t n, const float* pos, const float* h, const float* mu, const float* nH,
              const float* T, int32_t n_ray, const double* dirs, int32_t n_bins,
              const double* sigma, const double* w, double L, double box, double tol,
              int32_t max_iter, const double* x_init, double rtol, int32_t n_threads,
              double* x_hist, double* lnG_hist, double* N_last, int32_t* iters_done,
              double* maxdx_hist);
int orc_solve_rule(int64_t n, const float* pos, const float* h, const float* mu, const float* nH,
                   const float* T, int32_t n_ray, const double* dirs, int32_t n_bins,
                   const double* sigma, const double* w, double L, double box, double tol,
                   int32_t max_iter, double tau_skip, double tau_case_b, int32_t relative,
                   int32_t n_blocks, double rtol, int32_t n_threads, double* x_hist,
                   double* lnG_hist, int32_t* skipped, int32_t* iters_done, double* maxdx_hist);
void orc_morton(int64_t n, const float* pos, uint64_t* codes);
void orc_morton_seg(int64_t n, const float* pos, int32_t n_halo, const int64_t* halo_off,
                    uint64_t* codes);
int64_t orc_lbvh_seg(int64_t n, const float* pos, const float* h, int32_t leaf_max,
                     int32_t n_halo, const int64_t* halo_off, int32_t* perm,
                     uint64_t* codes_sorted, float* node_lo, float* node_hi, int32_t* node_skip,
                     int32_t* node_first, int32_t* node_count, int32_t* seg_root,
                     int32_t* seg_end);
int64_t orc_lbvh(int64_t n, const float* pos, const float* h, int32_t leaf_max,
                 int32_t* perm, uint64_t* codes_sorted, float* node_lo, float* node_hi,
                 int32_t* node_skip, int32_t* node_first, int32_t* node_count);
#ifdef __cplusplus
}
#endif
#endif
