/*
 * oracle.c -- FP64 CPU oracle for per-pixel principal curvatures by robust iterative
 * parabolic-quadric patch fitting (Spek, Li, Drummond, "A Fast Method For Computing
 * Principal Curvatures From Range Images", Section 3).
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow, literal restatement of the method used to
 * check the GPU library.  Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the GPU library.
 *
 * Every step follows the paper's order and notation.  Where the paper is silent the
 * following readings are taken (each is marked "Reading" below):
 *   - pinhole back-projection with Z along the optical axis, pixel centres at integer
 *     (u, v); the initial-normal regression is done in metric camera coordinates;
 *   - the frame R is initialised as the smallest rotation taking the initial normal to
 *     the z axis; theta_x, theta_y are small rotations about the current local x and y
 *     axes applied on the left; the Gauss-Newton update is subtracted;
 *   - a fixed number of iterations, no convergence test; the first iteration's weights
 *     come from the residuals of the initial planar patch;
 *   - neighbours outside the image or without depth are skipped; a fit needs 3 points
 *     for the normal and 6 for the quadric;
 *   - T2 is evaluated as sqrt(((A-C)/2)^2 + B^2), algebraically equal to the printed
 *     sqrt(T1^2 - AC + B^2) but free of cancellation;
 *   - with rejection on, R = 2 * (unweighted mean of e^2 over the patch); nothing is
 *     rejected when that mean is zero;
 *   - the reported residual is sqrt(sum w e^2 / sum w) at the final parameters;
 *   - the large patch "sparsely sampled" for the timings of Section 4 takes the pixels
 *     at offsets that are multiples of a stride s from the centre, within +-r (the
 *     stride is not given; s = 1 samples every pixel); the normal window stays dense.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXPTS 1369   /* (2r+1)^2 for r <= 18 (the 37x37 patch of Section 3.2) */

/* ---------------------------------------------------------------------------------
 * Reading: pinhole back-projection.  The paper builds an organised point cloud from
 * the range image (Section 3.2, first step) without giving the camera model.
 * ------------------------------------------------------------------------------- */
static int depth_valid(double z) { return z > 0.0 && isfinite(z); }

static void back_project(double Z, int u, int v, double fx, double fy, double cx, double cy,
                         double P[3]) {
    P[0] = Z * ((double)u - cx) / fx;
    P[1] = Z * ((double)v - cy) / fy;
    P[2] = Z;
}

/* ---------------------------------------------------------------------------------
 * Initial normal, Section 3.2.1, Eq. (7): regress z = a x + b y (+ const) over the
 * points of a small window using the mean-centred sums M and v, then
 * n = (-a, -b, 1) / sqrt(1 + a^2 + b^2).  Returns 0 when the regression is singular.
 * ------------------------------------------------------------------------------- */
static int initial_normal(const double (*pts)[3], int n, double nrm[3]) {
    if (n < 3) return 0;
    double xb = 0, yb = 0, zb = 0;
    for (int i = 0; i < n; ++i) { xb += pts[i][0]; yb += pts[i][1]; zb += pts[i][2]; }
    xb /= n; yb /= n; zb /= n;
    double M00 = 0, M01 = 0, M11 = 0, v0 = 0, v1 = 0;
    for (int i = 0; i < n; ++i) {
        double dx = pts[i][0] - xb, dy = pts[i][1] - yb, dz = pts[i][2] - zb;
        M00 += dx * dx; M01 += dx * dy; M11 += dy * dy;
        v0 += dx * dz;  v1 += dy * dz;
    }
    double det = M00 * M11 - M01 * M01;
    double tr = M00 + M11;
    if (!(det > 1e-12 * tr * tr)) return 0;
    /* (a b)^T = M^{-1} v */
    double a = (M11 * v0 - M01 * v1) / det;
    double b = (M00 * v1 - M01 * v0) / det;
    double s = 1.0 / sqrt(1.0 + a * a + b * b);
    nrm[0] = -a * s; nrm[1] = -b * s; nrm[2] = s;
    return 1;
}

/* 3x3 helpers (row-major) */
static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void skew(const double w[3], double K[9]) {
    K[0] = 0;     K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0;     K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0;
}

/* Reading: R starts as the smallest rotation taking n0 onto the z axis (Section 3.2.2
 * only asks that the z axis align with the normal).  With v = n0 x e_z, c = n0 . e_z:
 * R = I + [v]x + [v]x^2 / (1 + c).  c > 0 because n0 points away from the camera. */
static void frame_from_normal(const double n0[3], double R[9]) {
    double v[3] = { n0[1], -n0[0], 0.0 };
    double c = n0[2];
    double K[9], K2[9];
    skew(v, K);
    mat3_mul(K, K, K2);
    for (int i = 0; i < 9; ++i) R[i] = ((i % 4) == 0 ? 1.0 : 0.0) + K[i] + K2[i] / (1.0 + c);
}

/* Exact rotation Exp([w]x) (Rodrigues). */
static void rotation_exp(const double w[3], double E[9]) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int i = 0; i < 9; ++i) E[i] = (i % 4) == 0 ? 1.0 : 0.0;
    if (th == 0.0) return;
    double u[3] = { w[0] / th, w[1] / th, w[2] / th };
    double K[9], K2[9];
    skew(u, K);
    mat3_mul(K, K, K2);
    double s = sin(th), c1 = 1.0 - cos(th);
    for (int i = 0; i < 9; ++i) E[i] += s * K[i] + c1 * K2[i];
}

/* ---------------------------------------------------------------------------------
 * Residual of one centred point, Eqs. (4), (6), (8): e = pbar^T E^T Q E pbar with
 * pbar = (p', 1), E = [R | (0, 0, t_z)] and the quadric Q of the parabolic patch
 * z = A/2 x^2 + B x y + C/2 y^2 (Eq. (2)).  Its derivatives w.r.t. the six parameters
 * (theta_x, theta_y, t_z, A, B, C) form one row of J (Section 3.2.3).  The rotation
 * parameters are small rotations about the current local x and y axes, so with
 * s = R p' and q = E pbar: dq/dtheta_x = e_x x s, dq/dtheta_y = e_y x s, dq/dt_z = e_z;
 * and de/dq = 2 (Q qbar)_{xyz}.
 * ------------------------------------------------------------------------------- */
void oracle_residual_jacobian(const double R[9], double tz, double A, double B, double C,
                              const double p[3], double* eps, double J[6]) {
    double E[16] = { R[0], R[1], R[2], 0.0,
                     R[3], R[4], R[5], 0.0,
                     R[6], R[7], R[8], tz,
                     0.0,  0.0,  0.0,  1.0 };
    double Q[16] = { A / 2, B / 2, 0.0,  0.0,
                     B / 2, C / 2, 0.0,  0.0,
                     0.0,   0.0,   0.0, -0.5,
                     0.0,   0.0,  -0.5,  0.0 };
    double pb[4] = { p[0], p[1], p[2], 1.0 };
    double q[4], Qq[4], s[3];
    for (int i = 0; i < 4; ++i) {
        q[i] = 0;
        for (int k = 0; k < 4; ++k) q[i] += E[4 * i + k] * pb[k];
    }
    for (int i = 0; i < 4; ++i) {
        Qq[i] = 0;
        for (int k = 0; k < 4; ++k) Qq[i] += Q[4 * i + k] * q[k];
    }
    double e = 0;
    for (int i = 0; i < 4; ++i) e += q[i] * Qq[i];
    *eps = e;
    for (int i = 0; i < 3; ++i) s[i] = R[3 * i] * p[0] + R[3 * i + 1] * p[1] + R[3 * i + 2] * p[2];
    double g[3] = { 2 * Qq[0], 2 * Qq[1], 2 * Qq[2] };
    double ex_s[3] = { 0.0, -s[2], s[1] };   /* e_x x s */
    double ey_s[3] = { s[2], 0.0, -s[0] };   /* e_y x s */
    J[0] = g[0] * ex_s[0] + g[1] * ex_s[1] + g[2] * ex_s[2];
    J[1] = g[0] * ey_s[0] + g[1] * ey_s[1] + g[2] * ey_s[2];
    J[2] = g[2];
    J[3] = q[0] * q[0] / 2;
    J[4] = q[0] * q[1];
    J[5] = q[1] * q[1] / 2;
}

/* Principal curvatures from the second fundamental form [[A, B], [B, C]]
 * (Section 3.1.2): T1 = (A+C)/2, T2 = sqrt(T1^2 - AC + B^2), k1 = T1+T2, k2 = T1-T2.
 * Reading: T2 is evaluated in the equivalent form sqrt(((A-C)/2)^2 + B^2). */
void oracle_principal_curvatures(double A, double B, double C, double* k1, double* k2) {
    double T1 = (A + C) / 2;
    double T2 = hypot((A - C) / 2, B);
    *k1 = T1 + T2;
    *k2 = T1 - T2;
}

/* Solves the 6x6 symmetric system H b = g by Cholesky factorisation.  Returns 0 when
 * H is not numerically positive definite (a pivot <= 1e-12 times its diagonal). */
static int solve_spd6(const double H[36], const double g[6], double b[6]) {
    double L[36];
    memset(L, 0, sizeof L);
    for (int j = 0; j < 6; ++j) {
        double d = H[6 * j + j];
        for (int k = 0; k < j; ++k) d -= L[6 * j + k] * L[6 * j + k];
        if (!(H[6 * j + j] > 0.0) || !(d > 1e-12 * H[6 * j + j])) return 0;
        double ljj = sqrt(d);
        L[6 * j + j] = ljj;
        for (int i = j + 1; i < 6; ++i) {
            double s = H[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = s / ljj;
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * b[k];
        b[i] = s / L[6 * i + i];
    }
    return 1;
}

/* Weights of Eq. (11): W(e) = k / (k + e^2) if e^2 < R, else 0.  With rejection off
 * R is infinite; with it on R = 2 * MSE of the patch (Section 3.2.3). */
static void robust_weights(const double* e, int n, const oracle_params* prm, double* w) {
    double R = INFINITY;
    if (prm->reject) {
        double mse = 0;
        for (int i = 0; i < n; ++i) mse += e[i] * e[i];
        mse /= n;
        if (mse > 0) R = 2 * mse;
    }
    for (int i = 0; i < n; ++i) {
        double e2 = e[i] * e[i];
        w[i] = e2 < R ? prm->k / (prm->k + e2) : 0.0;
    }
}

/* ---------------------------------------------------------------------------------
 * The iterative re-weighted fit of Section 3.2.2-3.2.3 on centred points p_i' (Eq. 5).
 * Start: R aligned to n0, A = B = C = 0, t_z = 0.  Each iteration recomputes the
 * residuals and their weights, forms b = (J^T W J)^{-1} J^T W e (Eq. (10)) and applies
 * it: rotation R <- Exp([(-b0, -b1, 0)]x) R, t_z -= b2, A -= b3, B -= b4, C -= b5.
 * ------------------------------------------------------------------------------- */
typedef struct { double R[9], tz, A, B, C; } fit_state;

static int fit_points(const double (*pp)[3], int n, const double n0[3],
                      const oracle_params* prm, fit_state* st, double* residual) {
    double e[MAXPTS], w[MAXPTS], J[MAXPTS][6];
    frame_from_normal(n0, st->R);
    st->tz = st->A = st->B = st->C = 0.0;
    for (int it = 0; it < prm->iterations; ++it) {
        for (int i = 0; i < n; ++i)
            oracle_residual_jacobian(st->R, st->tz, st->A, st->B, st->C, pp[i], &e[i], J[i]);
        robust_weights(e, n, prm, w);
        double H[36] = { 0 }, g[6] = { 0 }, b[6];
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < 6; ++r) {
                g[r] += w[i] * J[i][r] * e[i];
                for (int c = 0; c < 6; ++c) H[6 * r + c] += w[i] * J[i][r] * J[i][c];
            }
        if (!solve_spd6(H, g, b)) return 0;
        double om[3] = { -b[0], -b[1], 0.0 }, Ex[9];
        rotation_exp(om, Ex);
        mat3_mul(Ex, st->R, st->R);
        st->tz -= b[2];
        st->A -= b[3];
        st->B -= b[4];
        st->C -= b[5];
    }
    if (residual) {
        double Jd[6], sw = 0, swe = 0;
        for (int i = 0; i < n; ++i)
            oracle_residual_jacobian(st->R, st->tz, st->A, st->B, st->C, pp[i], &e[i], Jd);
        robust_weights(e, n, prm, w);
        for (int i = 0; i < n; ++i) { sw += w[i]; swe += w[i] * e[i] * e[i]; }
        *residual = sw > 0 ? sqrt(swe / sw) : NAN;
    }
    return 1;
}

static int check_params(const oracle_params* p) {
    if (!p) return 0;
    if (p->radius < 1 || (2 * p->radius + 1) * (2 * p->radius + 1) > MAXPTS) return 0;
    if (p->normal_radius < 1 || (2 * p->normal_radius + 1) * (2 * p->normal_radius + 1) > MAXPTS) return 0;
    if (p->iterations < 0) return 0;
    if (!(p->k > 0.0)) return 0;
    if (p->stride < 1 || p->stride > p->radius) return 0;
    return 1;
}

/* One pixel of the range image (Section 3.2): back-project, initial normal from the
 * small window, fit the quadric to the large window, then curvatures (Section 3.1.2)
 * and the refined normal, the local z axis of the final frame (Section 3.2.4). */
static void fit_pixel(const double* depth, int W, int Hh, double fx, double fy, double cx,
                      double cy, const oracle_params* prm, int u, int v,
                      double* k1, double* k2, double nrm[3], double* res, uint8_t* flag) {
    double pts[MAXPTS][3];
    *k1 = *k2 = *res = NAN;
    nrm[0] = nrm[1] = nrm[2] = NAN;
    *flag = 0;
    double Zc = depth[(size_t)v * W + u];
    if (!depth_valid(Zc)) return;
    double Pc[3];
    back_project(Zc, u, v, fx, fy, cx, cy, Pc);

    int rn = prm->normal_radius, n = 0;
    for (int dv = -rn; dv <= rn; ++dv)
        for (int du = -rn; du <= rn; ++du) {
            int uu = u + du, vv = v + dv;
            if (uu < 0 || vv < 0 || uu >= W || vv >= Hh) continue;
            double Z = depth[(size_t)vv * W + uu];
            if (!depth_valid(Z)) continue;
            back_project(Z, uu, vv, fx, fy, cx, cy, pts[n++]);
        }
    double n0[3];
    if (!initial_normal((const double (*)[3])pts, n, n0)) return;

    int r = prm->radius, s = prm->stride, m = r / s;
    n = 0;
    for (int j = -m; j <= m; ++j)
        for (int i = -m; i <= m; ++i) {
            int du = i * s, dv = j * s;
            int uu = u + du, vv = v + dv;
            if (uu < 0 || vv < 0 || uu >= W || vv >= Hh) continue;
            double Z = depth[(size_t)vv * W + uu];
            if (!depth_valid(Z)) continue;
            double P[3];
            back_project(Z, uu, vv, fx, fy, cx, cy, P);
            /* Eq. (5): points relative to the centre point */
            pts[n][0] = P[0] - Pc[0];
            pts[n][1] = P[1] - Pc[1];
            pts[n][2] = P[2] - Pc[2];
            ++n;
        }
    if (n < 6) return;
    fit_state st;
    double residual = NAN;
    if (!fit_points((const double (*)[3])pts, n, n0, prm, &st, &residual)) return;
    oracle_principal_curvatures(st.A, st.B, st.C, k1, k2);
    nrm[0] = st.R[6]; nrm[1] = st.R[7]; nrm[2] = st.R[8];
    *res = residual;
    *flag = ORACLE_VALID;
}

int oracle_fit_pixels(const double* depth, int32_t width, int32_t height,
                      double fx, double fy, double cx, double cy,
                      const oracle_params* params, const int64_t* pixels, int64_t npx,
                      double* k1, double* k2, double* normal, double* residual,
                      uint8_t* flags, int32_t nthreads) {
    if (!depth || width <= 0 || height <= 0 || !check_params(params) || npx < 0) return -1;
    if (npx > 0 && !pixels) return -1;
    for (int64_t i = 0; i < npx; ++i)
        if (pixels[i] < 0 || pixels[i] >= (int64_t)width * height) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npx; ++i) {
        int u = (int)(pixels[i] % width), v = (int)(pixels[i] / width);
        double a, b, rs, nn[3];
        uint8_t f;
        fit_pixel(depth, width, height, fx, fy, cx, cy, params, u, v, &a, &b, nn, &rs, &f);
        if (k1) k1[i] = a;
        if (k2) k2[i] = b;
        if (normal) { normal[3 * i] = nn[0]; normal[3 * i + 1] = nn[1]; normal[3 * i + 2] = nn[2]; }
        if (residual) residual[i] = rs;
        if (flags) flags[i] = f;
    }
    return 0;
}

int oracle_fit_image(const double* depth, int32_t width, int32_t height,
                     double fx, double fy, double cx, double cy,
                     const oracle_params* params,
                     double* k1, double* k2, double* normal, double* residual,
                     uint8_t* flags, int32_t nthreads) {
    if (!depth || width <= 0 || height <= 0 || !check_params(params)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int v = 0; v < height; ++v)
        for (int u = 0; u < width; ++u) {
            size_t i = (size_t)v * width + u;
            double a, b, rs, nn[3];
            uint8_t f;
            fit_pixel(depth, width, height, fx, fy, cx, cy, params, u, v, &a, &b, nn, &rs, &f);
            if (k1) k1[i] = a;
            if (k2) k2[i] = b;
            if (normal) { normal[3 * i] = nn[0]; normal[3 * i + 1] = nn[1]; normal[3 * i + 2] = nn[2]; }
            if (residual) residual[i] = rs;
            if (flags) flags[i] = f;
        }
    return 0;
}

int oracle_fit_patch(const double* pts, int32_t n, int32_t centre, const double n0[3],
                     const oracle_params* params,
                     double* k1, double* k2, double normal[3], double* residual,
                     double state_out[13]) {
    if (!pts || !n0 || n <= 0 || n > MAXPTS || centre < 0 || centre >= n) return -1;
    if (!check_params(params)) return -1;
    double (*pp)[3] = malloc(sizeof(double[3]) * MAXPTS);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) pp[i][c] = pts[3 * i + c] - pts[3 * centre + c];
    double nn = sqrt(n0[0] * n0[0] + n0[1] * n0[1] + n0[2] * n0[2]);
    double nu[3] = { n0[0] / nn, n0[1] / nn, n0[2] / nn };
    fit_state st;
    double res = NAN;
    int ok = n >= 6 && nu[2] > -1.0 && fit_points((const double (*)[3])pp, n, nu, params, &st, &res);
    free(pp);
    if (!ok) {
        if (k1) *k1 = NAN;
        if (k2) *k2 = NAN;
        if (residual) *residual = NAN;
        if (normal) normal[0] = normal[1] = normal[2] = NAN;
        return 0;
    }
    double a, b;
    oracle_principal_curvatures(st.A, st.B, st.C, &a, &b);
    if (k1) *k1 = a;
    if (k2) *k2 = b;
    if (residual) *residual = res;
    if (normal) { normal[0] = st.R[6]; normal[1] = st.R[7]; normal[2] = st.R[8]; }
    if (state_out) {
        memcpy(state_out, st.R, sizeof st.R);
        state_out[9] = st.tz; state_out[10] = st.A; state_out[11] = st.B; state_out[12] = st.C;
    }
    return 1;
}
