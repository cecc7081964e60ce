/*
 * oracle.h -- FP64 CPU oracle for per-pixel principal curvatures by robust iterative
 * parabolic-quadric patch fitting (Spek, Li, Drummond, "A Fast Method For Computing
 * Principal Curvatures From Range Images", Section 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library against a
 * plain, slow, obviously correct restatement of the method.  Only the test-suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * All arithmetic is IEEE double.  Units: metres in, inverse metres out.
 */
#ifndef QCURV_ORACLE_H
#define QCURV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t radius;         /* r: the fit window is (2r+1)^2 pixels */
    int32_t normal_radius;  /* r_n: the initial-normal window is (2r_n+1)^2 (7x7 in the paper) */
    int32_t iterations;     /* T: fixed number of re-weighted Gauss-Newton steps */
    int32_t reject;         /* 0: weights k/(k+e^2); 1: also zero points with e^2 >= 2*MSE */
    double k;               /* robust constant of Eq. (11), m^2, > 0 */
    int32_t stride;         /* s >= 1: the fit window samples the pixels at offsets that are
                               multiples of s from the centre, within +-r (the paper's
                               sparsely sampled large patch, Section 4); 1 = every pixel */
} oracle_params;

/* Per-pixel result flags. */
#define ORACLE_VALID 1u

/* Fits every pixel of a depth image (Z along the optical axis, metres, 0 or
 * non-finite = no depth).  depth is row-major with `width` doubles per row.
 * Outputs are arrays of width*height (normal: width*height*3, xyz per pixel);
 * any output pointer may be NULL.  Invalid pixels get NaN and flag 0.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on a bad argument. */
int oracle_fit_image(const double* depth, int32_t width, int32_t height,
                     double fx, double fy, double cx, double cy,
                     const oracle_params* params,
                     double* k1, double* k2, double* normal, double* residual,
                     uint8_t* flags, int32_t nthreads);

/* Same as oracle_fit_image, but only for the n pixels listed in `pixels`
 * (linear indices v*width+u).  Output element i belongs to pixels[i]. */
int oracle_fit_pixels(const double* depth, int32_t width, int32_t height,
                      double fx, double fy, double cx, double cy,
                      const oracle_params* params,
                      const int64_t* pixels, int64_t n,
                      double* k1, double* k2, double* normal, double* residual,
                      uint8_t* flags, int32_t nthreads);

/* Fits one patch given as an explicit point set (camera coordinates, metres).
 * pts: n x 3; the patch is centred on pts[centre]; n0 is the initial unit normal.
 * state_out (13 doubles, may be NULL): final R row-major (9), t_z, A, B, C.
 * Returns 1 if the fit is valid, 0 if not, -1 on a bad argument. */
int oracle_fit_patch(const double* pts, int32_t n, int32_t centre, const double n0[3],
                     const oracle_params* params,
                     double* k1, double* k2, double normal[3], double* residual,
                     double state_out[13]);

/* The residual of Eq. (6)/(8) for one centred point p' and its derivatives w.r.t.
 * (theta_x, theta_y, t_z, A, B, C); R is row-major.  Exposed for derivative checks. */
void oracle_residual_jacobian(const double R[9], double tz, double A, double B, double C,
                              const double p[3], double* eps, double J[6]);

/* Principal curvatures from (A, B, C) (Section 3.1.2). */
void oracle_principal_curvatures(double A, double B, double C, double* k1, double* k2);

#ifdef __cplusplus
}
#endif

#endif
