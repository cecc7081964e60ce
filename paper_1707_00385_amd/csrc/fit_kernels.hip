// fit_kernels.hip -- gfx950 kernels for per-pixel robust quadric-patch curvature fitting
// (Spek, Li, Drummond, "A Fast Method For Computing Principal Curvatures From Range
// Images", Section 3).
//
// One lane fits one pixel.  The fast pass stages a depth tile plus its halo in LDS and
// runs the whole fit in FP32; the FP64 pass re-runs the identical sequence of steps in
// double precision for a compacted list of pixels (or for every pixel).
//
// Arithmetic layout (exact in real arithmetic to the method's steps; chosen for FP32):
//  * Centring (Eq. (5)) is done on the integer/native depth samples: with D the depth in
//    native units and s metres per unit, p' = P_i - P_c = s * G0 * m with
//    m = ((u_i-u_c) D_i, (v_i-v_c) D_i, D_i - D_c), which is exact for U16 and F16 input,
//    and G0 = [[1/fx, 0, (u_c-cx)/fx], [0, 1/fy, (v_c-cy)/fy], [0, 0, 1]].
//  * Lengths are measured in units of h = r Z_c / fx (the window half-extent), so the
//    patch coefficients become A h, B h, C h, t_z / h and k / h^2; Gauss-Newton is
//    invariant under this rescaling, so the iterates are the same.
//  * Each neighbour contributes sqrt(w) J to the normal equations (H = sum (sqrt w J)
//    (sqrt w J)^T, g = sum (sqrt w J)(sqrt w e)), with w = 1/(k + e^2): the factor k of
//    Eq. (11) cancels in (J^T W J)^{-1} J^T W e.
//  * The 6x6 solve is Jacobi-equilibrated LDL^T; the pivot ratio estimates the
//    condition number that decides the FP64 recomputation.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <utility>

#include "fit_internal.h"

namespace qc {
namespace {

constexpr int kMaxRadius = 18;
constexpr uint8_t kFlagValid = 1, kFlagFp64 = 2, kFlagIll = 4;
constexpr int kTileW = 16;

// ---------------------------------------------------------------------------- scalars
template <typename T> __device__ __forceinline__ T fmaT(T a, T b, T c);
template <> __device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/sqrt(x) with 1/sqrt(+inf) = 0 (the weight of a missing neighbour).
template <typename T> __device__ __forceinline__ T rsqrtT(T x);
template <> __device__ __forceinline__ float rsqrtT(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsqrtT(double x) { return isinf(x) ? 0.0 : rsqrt(x); }

template <typename T> __device__ __forceinline__ T sqrtT(T x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T sinT(T x) { return sin(x); }

// ---------------------------------------------------------------------------- depth
__device__ __forceinline__ float load_sample(const FitDesc& d, int x, int y) {
    const char* row = static_cast<const char*>(d.depth) + static_cast<int64_t>(y) * d.pitch;
    if (d.format == 0) return static_cast<float>(reinterpret_cast<const uint16_t*>(row)[x]);
    if (d.format == 1) return __half2float(reinterpret_cast<const __half*>(row)[x]);
    return reinterpret_cast<const float*>(row)[x];
}

// (D, pen): D = depth in native units, pen = 0 for a valid sample and +inf for a
// missing one (outside the image, zero or non-finite).  pen is added to the weight's
// denominator so a missing neighbour gets weight exactly 0 without a branch.
__device__ __forceinline__ float2 sample_or_missing(const FitDesc& d, int x, int y) {
    if (x < 0 || y < 0 || x >= d.width || y >= d.height) return make_float2(0.f, INFINITY);
    float z = load_sample(d, x, y);
    bool ok = z > 0.f && z <= 3.0e38f;   // excludes 0, negatives, inf and NaN
    return make_float2(ok ? z : 0.f, ok ? 0.f : INFINITY);
}

// Neighbourhood accessors.  row(dv)[du] is the (D, pen) pair of pixel (u+du, v+dv).
struct LdsRow {
    const float2* p;
    __device__ __forceinline__ float2 operator[](int du) const { return p[du]; }
};
struct LdsSource {
    const float2* centre;   // entry of the pixel itself
    int pitch;              // entries per LDS row
    __device__ __forceinline__ LdsRow row(int dv) const { return LdsRow{centre + dv * pitch}; }
};
struct GlobalRow {
    const FitDesc* d;
    int u, y;
    __device__ __forceinline__ float2 operator[](int du) const { return sample_or_missing(*d, u + du, y); }
};
struct GlobalSource {
    const FitDesc* d;
    int u, v;
    __device__ __forceinline__ GlobalRow row(int dv) const { return GlobalRow{d, u, v + dv}; }
};

// ---------------------------------------------------------------------------- one pixel
template <typename Real>
struct PixelFit {
    Real k1, k2, n[3], residual;
    uint8_t flags;
};

// Per-pixel geometry: p'/h = G m (see the header comment).
template <typename Real>
struct Geometry {
    Real Dc, g00, g02, g11, g12, g22, h, ih, kt;
};

// Loops over the window rows -R..R; RC > 0 fixes R at compile time.  A row is fully
// unrolled for FP32 (U = 0); FP64 keeps it rolled (U = 1) to stay within the register file.
template <int RC, int U = 0, typename Src, typename F>
__device__ __forceinline__ void for_window(const Src& src, int radius, F&& f) {
    if constexpr (RC > 0 && U == 0) {
        for (int dv = -RC; dv <= RC; ++dv) {
            auto row = src.row(dv);
#pragma unroll
            for (int du = -RC; du <= RC; ++du) f(row[du], du, dv);
        }
    } else {
        const int r = RC > 0 ? RC : radius;
        for (int dv = -r; dv <= r; ++dv) {
            auto row = src.row(dv);
#pragma unroll 1
            for (int du = -r; du <= r; ++du) f(row[du], du, dv);
        }
    }
}

// The pixel's fit, Section 3.2: initial normal (Eq. (7)), frame set-up, fixed number of
// re-weighted Gauss-Newton steps (Eqs. (8)-(11)), curvatures, refined normal.
template <typename Real, int RC, typename Src>
__device__ PixelFit<Real> fit_pixel(const FitDesc& d, const Src& src, int u, int v, float Dc_f,
                                    bool want_residual) {
    PixelFit<Real> out;
    const Real nan = Real(NAN);
    out.k1 = out.k2 = out.residual = nan;
    out.n[0] = out.n[1] = out.n[2] = nan;
    out.flags = 0;
    using Acc = double;   // normal-equation sums and the 6x6 solve
    const int radius = RC > 0 ? RC : d.radius;
    const bool fp32 = sizeof(Real) == 4;

    // ---- geometry (Eq. (5) centring on native samples, lengths in units of h)
    Geometry<Real> g;
    g.Dc = Real(Dc_f);
    const Real s = Real(d.scale);
    const Real fx = Real(d.fx), fy = Real(d.fy);
    const Real Zc = g.Dc * s;
    g.h = Real(radius) * Zc / fx;
    g.ih = Real(1) / g.h;
    const Real ihs = g.ih * s;
    g.g00 = ihs / fx;
    g.g02 = ihs * ((Real(u) - Real(d.cx)) / fx);
    g.g11 = ihs / fy;
    g.g12 = ihs * ((Real(v) - Real(d.cy)) / fy);
    g.g22 = ihs;
    g.kt = Real(d.k) * g.ih * g.ih;

    // ---- initial normal, Section 3.2.1: regression z = a x + b y over the small window
    //      with mean-centred sums M, v; n0 = (-a, -b, 1) / sqrt(1 + a^2 + b^2)
    const int rn = d.normal_radius;
    Real cnt = 0, mx_ = 0, my_ = 0, mz_ = 0;
    for_window<0>(src, rn, [&](float2 t, int du, int dv) {
        const Real ok = t.y == 0.f ? Real(1) : Real(0);
        const Real D = Real(t.x), dD = D - g.Dc;
        const Real px = fmaT(g.g00, Real(du) * D, g.g02 * dD);
        const Real py = fmaT(g.g11, Real(dv) * D, g.g12 * dD);
        const Real pz = g.g22 * dD;
        cnt += ok;
        mx_ = fmaT(ok, px, mx_);
        my_ = fmaT(ok, py, my_);
        mz_ = fmaT(ok, pz, mz_);
    });
    if (cnt < Real(3)) return out;
    mx_ /= cnt; my_ /= cnt; mz_ /= cnt;
    Real M00 = 0, M01 = 0, M11 = 0, v0 = 0, v1 = 0;
    for_window<0>(src, rn, [&](float2 t, int du, int dv) {
        const Real ok = t.y == 0.f ? Real(1) : Real(0);
        const Real D = Real(t.x), dD = D - g.Dc;
        const Real px = fmaT(g.g00, Real(du) * D, g.g02 * dD) - mx_;
        const Real py = fmaT(g.g11, Real(dv) * D, g.g12 * dD) - my_;
        const Real pz = g.g22 * dD - mz_;
        const Real opx = ok * px, opy = ok * py;
        M00 = fmaT(opx, px, M00);
        M01 = fmaT(opx, py, M01);
        M11 = fmaT(opy, py, M11);
        v0 = fmaT(opx, pz, v0);
        v1 = fmaT(opy, pz, v1);
    });
    const Real det = M00 * M11 - M01 * M01;
    const Real tr = M00 + M11;
    bool ill = false;
    if (!(det > Real(1e-12) * tr * tr)) {
        if (fp32) out.flags = kFlagIll;   // let FP64 decide
        return out;
    }
    if (fp32 && !(det > Real(1e-4) * tr * tr)) ill = true;
    const Real ia = (M11 * v0 - M01 * v1) / det;
    const Real ib = (M00 * v1 - M01 * v0) / det;
    const Real nsc = Real(1) / sqrtT(Real(1) + ia * ia + ib * ib);
    const Real n0x = -ia * nsc, n0y = -ib * nsc, n0z = nsc;

    // ---- enough neighbours for six parameters
    Real nfit = 0;
    for_window<RC, sizeof(Real) == 8>(src, radius, [&](float2 t, int, int) { nfit += t.y == 0.f ? Real(1) : Real(0); });
    if (nfit < Real(6)) return out;

    // ---- frame: smallest rotation taking n0 to e_z; R = I + [w]x + [w]x^2/(1+c),
    //      w = n0 x e_z = (n0y, -n0x, 0), c = n0z > 0 (Section 3.2.2 initialisation)
    Real R[3][3];
    {
        const Real wx = n0y, wy = -n0x, ic = Real(1) / (Real(1) + n0z);
        R[0][0] = Real(1) - wy * wy * ic; R[0][1] = wx * wy * ic;           R[0][2] = wy;
        R[1][0] = wx * wy * ic;           R[1][1] = Real(1) - wx * wx * ic; R[1][2] = -wx;
        R[2][0] = -wy;                    R[2][1] = wx;                     R[2][2] = n0z;
    }
    Real tz = 0, A = 0, B = 0, C = 0;     // patch coefficients in units of h
    Acc kappa_max = 0, last_step = 0;

    for (int it = 0; it < d.iterations; ++it) {
        // R' = R G: maps m straight to the rotated, scaled, centred point s = R p'/h.
        // The third row is doubled: it yields 2 s_z, which the Jacobian needs.
        Real Rp[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const Real f = i == 2 ? Real(2) : Real(1);
            Rp[i][0] = f * R[i][0] * g.g00;
            Rp[i][1] = f * R[i][1] * g.g11;
            Rp[i][2] = f * fmaT(R[i][0], g.g02, fmaT(R[i][1], g.g12, R[i][2] * g.g22));
        }
        const Real Ah = Real(0.5) * A, Bh = Real(0.5) * B, Ch = Real(0.5) * C;
        // accumulators: Hij = sum ji jj with j = sqrt(w) * (J0, J1, -1, sx^2, sx sy, sy^2);
        // S_i = sum ji sqrt(w) (column 2 up to sign); Gi = sum ji sqrt(w) e.
        // The sums are accumulated in FP64 whatever the per-neighbour precision: FP32
        // accumulation of 225 terms is the dominant rounding error of the FP32 fit.
        Acc H00 = 0, H01 = 0, H03 = 0, H04 = 0, H05 = 0, H11 = 0, H13 = 0, H14 = 0, H15 = 0;
        Acc H33 = 0, H34 = 0, H35 = 0, H45 = 0, H55 = 0;
        Acc S0 = 0, S1 = 0, S2 = 0, S3 = 0, S4 = 0, S5 = 0;
        Acc G0 = 0, G1 = 0, G2 = 0, G3 = 0, G4 = 0, G5 = 0;
        for_window<RC, sizeof(Real) == 8>(src, radius, [&](float2 t, int du, int dv) {
            const Real D = Real(t.x);
            const Real dD = D - g.Dc;
            const Real mx = Real(du) * D, my = Real(dv) * D;
            const Real sx = fmaT(Rp[0][0], mx, fmaT(Rp[0][1], my, Rp[0][2] * dD));
            const Real sy = fmaT(Rp[1][0], mx, fmaT(Rp[1][1], my, Rp[1][2] * dD));
            const Real sz2 = fmaT(Rp[2][0], mx, fmaT(Rp[2][1], my, Rp[2][2] * dD));
            const Real qz = fmaT(Real(0.5), sz2, tz);
            const Real ap = fmaT(Ah, sx, Bh * sy);          // (A qx + B qy) / 2
            const Real cp = fmaT(Bh, sx, Ch * sy);          // (B qx + C qy) / 2
            const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz)); // Eq. (6): A/2 qx^2 + B qx qy + C/2 qy^2 - qz
            const Real den = fmaT(e, e, g.kt) + Real(t.y);
            const Real rw = rsqrtT(den);                    // sqrt of the weight, Eq. (11)
            const Real J0 = -fmaT(cp, sz2, sy);             // de/dtheta_x
            const Real J1 = fmaT(ap, sz2, sx);              // de/dtheta_y
            const Real j0r = rw * J0, j1r = rw * J1;
            const Real xr = rw * sx, yr = rw * sy;
            const Real j3r = xr * sx, j4r = xr * sy, j5r = yr * sy, jer = rw * e;
            const Acc j0 = Acc(j0r), j1 = Acc(j1r), wr = Acc(rw);
            const Acc j3 = Acc(j3r), j4 = Acc(j4r), j5 = Acc(j5r), je = Acc(jer);
            H00 = fmaT(j0, j0, H00); H01 = fmaT(j0, j1, H01); H03 = fmaT(j0, j3, H03);
            H04 = fmaT(j0, j4, H04); H05 = fmaT(j0, j5, H05);
            H11 = fmaT(j1, j1, H11); H13 = fmaT(j1, j3, H13); H14 = fmaT(j1, j4, H14);
            H15 = fmaT(j1, j5, H15);
            H33 = fmaT(j3, j3, H33); H34 = fmaT(j3, j4, H34); H35 = fmaT(j3, j5, H35);
            H45 = fmaT(j4, j5, H45); H55 = fmaT(j5, j5, H55);
            S0 = fmaT(j0, wr, S0); S1 = fmaT(j1, wr, S1); S2 = fmaT(wr, wr, S2);
            S3 = fmaT(j3, wr, S3); S4 = fmaT(j4, wr, S4); S5 = fmaT(j5, wr, S5);
            G0 = fmaT(j0, je, G0); G1 = fmaT(j1, je, G1); G2 = fmaT(wr, je, G2);
            G3 = fmaT(j3, je, G3); G4 = fmaT(j4, je, G4); G5 = fmaT(j5, je, G5);
        });
        // Normal equations of Eq. (10) for the parameters (theta_x, theta_y, t_z, A, B, C):
        // J2 = -1, and J3, J5 carry a factor 1/2 (de/dA = qx^2/2, de/dC = qy^2/2).
        // H44 = sum w qx^2 qy^2 = 4 * (H35 scaled) -- same sum as sx^2 * sy^2.
        Acc Hm[6][6], gv[6];
        Hm[0][0] = H00; Hm[0][1] = H01; Hm[0][2] = -S0; Hm[0][3] = Acc(0.5) * H03; Hm[0][4] = H04; Hm[0][5] = Acc(0.5) * H05;
        Hm[1][1] = H11; Hm[1][2] = -S1; Hm[1][3] = Acc(0.5) * H13; Hm[1][4] = H14; Hm[1][5] = Acc(0.5) * H15;
        Hm[2][2] = S2; Hm[2][3] = Acc(-0.5) * S3; Hm[2][4] = -S4; Hm[2][5] = Acc(-0.5) * S5;
        Hm[3][3] = Acc(0.25) * H33; Hm[3][4] = Acc(0.5) * H34; Hm[3][5] = Acc(0.25) * H35;
        Hm[4][4] = H35; Hm[4][5] = Acc(0.5) * H45;
        Hm[5][5] = Acc(0.25) * H55;
        gv[0] = G0; gv[1] = G1; gv[2] = -G2; gv[3] = Acc(0.5) * G3; gv[4] = G4; gv[5] = Acc(0.5) * G5;

        // Jacobi equilibration, then LDL^T with pivots dp[j] of the unit-diagonal matrix.
        Acc dsc[6];
        bool singular = false;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            singular |= !(Hm[i][i] > Acc(0));
            dsc[i] = Hm[i][i] > Acc(0) ? rsqrtT(Hm[i][i]) : Acc(0);
        }
        Acc L[6][6], dp[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            Acc dj = Acc(1);   // equilibrated diagonal
#pragma unroll
            for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k] * dp[k];
            dp[j] = dj;
            const Acc idj = dj > Acc(0) ? Acc(1) / dj : Acc(0);
#pragma unroll
            for (int i = j + 1; i < 6; ++i) {
                Acc sij = dsc[i] * dsc[j] * Hm[j][i];
#pragma unroll
                for (int k = 0; k < j; ++k) sij -= L[i][k] * L[j][k] * dp[k];
                L[i][j] = sij * idj;
            }
        }
        Acc pmin = dp[0], pmax = dp[0];
#pragma unroll
        for (int j = 1; j < 6; ++j) { pmin = fmin(pmin, dp[j]); pmax = fmax(pmax, dp[j]); }
        // FP64 reads its pivots literally, like the oracle's Cholesky test (1e-12 of the
        // diagonal); FP32 treats anything beyond its accuracy as a reason to recompute.
        if (singular || !(pmin > Acc(1e-12))) {
            if (fp32) out.flags = kFlagIll;
            return out;
        }
        kappa_max = fmax(kappa_max, pmax / pmin);
        Acc y[6], b[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            Acc sy = dsc[i] * gv[i];
#pragma unroll
            for (int k = 0; k < i; ++k) sy -= L[i][k] * y[k];
            y[i] = sy;
        }
#pragma unroll
        for (int i = 5; i >= 0; --i) {
            Acc sb = y[i] / dp[i];
#pragma unroll
            for (int k = i + 1; k < 6; ++k) sb -= L[k][i] * b[k];
            b[i] = sb;
        }
        Acc step = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i) { b[i] *= dsc[i]; step = fmax(step, fabs(b[i])); }
        last_step = step;

        // Update (Section 3.2.3): R <- Exp([(-b0, -b1, 0)]x) R (exact Rodrigues),
        // t_z -= b2, A -= b3, B -= b4, C -= b5.
        {
            const Real w0 = Real(-b[0]), w1 = Real(-b[1]);
            const Real th2 = w0 * w0 + w1 * w1;
            Real st = Real(1), c1 = Real(0.5);
            if (th2 > Real(0)) {
                const Real th = sqrtT(th2);
                st = sinT(th) / th;                         // sin(th)/th
                const Real sh = sinT(Real(0.5) * th) / th;  // sin(th/2)/th
                c1 = Real(2) * sh * sh;                     // (1-cos th)/th^2
            }
            const Real E00 = Real(1) - c1 * w1 * w1, E01 = c1 * w0 * w1, E02 = st * w1;
            const Real E11 = Real(1) - c1 * w0 * w0, E12 = -st * w0;
            const Real E20 = -st * w1, E21 = st * w0, E22 = Real(1) - c1 * th2;
            Real Rn[3][3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Rn[0][j] = fmaT(E00, R[0][j], fmaT(E01, R[1][j], E02 * R[2][j]));
                Rn[1][j] = fmaT(E01, R[0][j], fmaT(E11, R[1][j], E12 * R[2][j]));
                Rn[2][j] = fmaT(E20, R[0][j], fmaT(E21, R[1][j], E22 * R[2][j]));
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) R[i][j] = Rn[i][j];
        }
        tz -= Real(b[2]);
        A -= Real(b[3]);
        B -= Real(b[4]);
        C -= Real(b[5]);
    }

    if (want_residual) {
        // residual at the final parameters: sqrt(sum w e^2 / sum w), in metres
        Real Rp[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Rp[i][0] = R[i][0] * g.g00;
            Rp[i][1] = R[i][1] * g.g11;
            Rp[i][2] = fmaT(R[i][0], g.g02, fmaT(R[i][1], g.g12, R[i][2] * g.g22));
        }
        const Real Ah = Real(0.5) * A, Bh = Real(0.5) * B, Ch = Real(0.5) * C;
        Real sw = 0, swe = 0;
        for_window<RC, sizeof(Real) == 8>(src, radius, [&](float2 t, int du, int dv) {
            const Real D = Real(t.x), dD = D - g.Dc;
            const Real mx = Real(du) * D, my = Real(dv) * D;
            const Real sx = fmaT(Rp[0][0], mx, fmaT(Rp[0][1], my, Rp[0][2] * dD));
            const Real sy = fmaT(Rp[1][0], mx, fmaT(Rp[1][1], my, Rp[1][2] * dD));
            const Real sz = fmaT(Rp[2][0], mx, fmaT(Rp[2][1], my, Rp[2][2] * dD));
            const Real qz = sz + tz;
            const Real ap = fmaT(Ah, sx, Bh * sy), cp = fmaT(Bh, sx, Ch * sy);
            const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz));
            const Real rw = rsqrtT(fmaT(e, e, g.kt) + Real(t.y));
            const Real w = rw * rw;
            sw += w;
            swe = fmaT(w * e, e, swe);
        });
        out.residual = g.h * sqrtT(swe / sw);
    }

    // Curvatures (Section 3.1.2) with T2 = hypot((A-C)/2, B); back to inverse metres.
    const Real Am = A * g.ih, Bm = B * g.ih, Cm = C * g.ih;
    const Real T1 = Real(0.5) * (Am + Cm);
    const Real T2 = hypot(Real(0.5) * (Am - Cm), Bm);
    out.k1 = T1 + T2;
    out.k2 = T1 - T2;
    // Refined normal (Section 3.2.4): the local z axis of the final frame.
    out.n[0] = R[2][0];
    out.n[1] = R[2][1];
    out.n[2] = R[2][2];
    out.flags = kFlagValid | (fp32 ? 0 : kFlagFp64);
    if (fp32 && (ill || !(kappa_max <= Acc(d.cond_max)) || !(last_step <= Acc(d.step_max))))
        out.flags |= kFlagIll;
    return out;
}

template <typename Real>
__device__ __forceinline__ void store_pixel(const FitDesc& d, int64_t idx, const PixelFit<Real>& r) {
    d.k1[idx] = static_cast<float>(r.k1);
    d.k2[idx] = static_cast<float>(r.k2);
    if (d.normal) {
        d.normal[3 * idx + 0] = static_cast<float>(r.n[0]);
        d.normal[3 * idx + 1] = static_cast<float>(r.n[1]);
        d.normal[3 * idx + 2] = static_cast<float>(r.n[2]);
    }
    if (d.residual) d.residual[idx] = static_cast<float>(r.residual);
    if (d.flags) d.flags[idx] = r.flags;
}

// ---------------------------------------------------------------------------- kernels
// counts[0]: entries in the recomputation list, counts[1]: pixels they cover.
__global__ void zero_counts(uint32_t* counts) {
    counts[0] = 0u;
    counts[1] = 0u;
}

// Stages the depth samples of a (w + 2 halo) x (h + 2 halo) region whose top-left pixel
// is (x0, y0) into LDS as (D, pen) pairs.
__device__ __forceinline__ void stage_region(const FitDesc& d, float2* lds, int x0, int y0,
                                             int pitch, int rows) {
    for (int i = threadIdx.x; i < pitch * rows; i += blockDim.x) {
        const int ly = i / pitch, lx = i - ly * pitch;
        lds[i] = sample_or_missing(d, x0 + lx, y0 + ly);
    }
    __syncthreads();
}

template <typename Real>
__device__ __forceinline__ PixelFit<Real> missing_pixel() {
    PixelFit<Real> r;
    r.k1 = r.k2 = r.residual = Real(NAN);
    r.n[0] = r.n[1] = r.n[2] = Real(NAN);
    r.flags = 0;
    return r;
}

// Tiled pass: a kTileW x TH tile per workgroup, halo staged in LDS, one lane per pixel.
// In FP32 (MIXED) every wave lists the lanes whose fit is judged unreliable: one entry
// per 16x4 block of pixels with a 64-bit lane mask.
template <typename Real, int R, int TH>
__global__ __launch_bounds__(kTileW* TH) void fit_tile(FitDesc d, uint32_t* entries,
                                                       uint64_t* masks, uint32_t* counts) {
    extern __shared__ float2 tile[];
    const int halo = max(R, d.normal_radius);
    const int pitch = kTileW + 2 * halo;
    stage_region(d, tile, blockIdx.x * kTileW - halo, blockIdx.y * TH - halo, pitch, TH + 2 * halo);
    const int lx = threadIdx.x % kTileW, ly = threadIdx.x / kTileW;
    const int u = blockIdx.x * kTileW + lx, v = blockIdx.y * TH + ly;
    const bool inside = u < d.width && v < d.height;
    bool recompute = false;
    if (inside) {
        const float2* centre = tile + (ly + halo) * pitch + (lx + halo);
        const PixelFit<Real> r = centre->y != 0.f
            ? missing_pixel<Real>()
            : fit_pixel<Real, R>(d, LdsSource{centre, pitch}, u, v, centre->x, d.residual != nullptr);
        store_pixel(d, static_cast<int64_t>(v) * d.width + u, r);
        recompute = (r.flags & kFlagIll) != 0;
    }
    if (sizeof(Real) == 4 && d.precision != 2) {
        const uint64_t mask = __ballot(recompute);
        if (mask != 0 && (threadIdx.x % 64) == 0) {
            // 16x4 block index: (row of 4-pixel bands) * tiles_x + tile column
            const uint32_t tiles_x = (d.width + kTileW - 1) / kTileW;
            const uint32_t band = (blockIdx.y * TH + (threadIdx.x / 64) * 4) / 4;
            const uint32_t slot = atomicAdd(&counts[0], 1u);
            entries[slot] = band * tiles_x + blockIdx.x;
            masks[slot] = mask;
            atomicAdd(&counts[1], static_cast<uint32_t>(__popcll(mask)));
        }
    }
}

// FP64 recomputation of listed pixels: one 64-lane workgroup per 16x4 block entry,
// halo staged in LDS, lanes whose mask bit is set run the fit.
template <int R>
__global__ __launch_bounds__(64) void refit_blocks_f64(FitDesc d, const uint32_t* entries,
                                                       const uint64_t* masks,
                                                       const uint32_t* counts) {
    extern __shared__ float2 tile[];
    const uint32_t n = counts[0];
    const uint32_t tiles_x = (d.width + kTileW - 1) / kTileW;
    const int halo = max(R, d.normal_radius);
    const int pitch = kTileW + 2 * halo;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t e = entries[i];
        const uint64_t mask = masks[i];
        const int bx = static_cast<int>(e % tiles_x) * kTileW;
        const int by = static_cast<int>(e / tiles_x) * 4;
        stage_region(d, tile, bx - halo, by - halo, pitch, 4 + 2 * halo);
        const int lx = threadIdx.x % kTileW, ly = threadIdx.x / kTileW;
        if ((mask >> threadIdx.x) & 1u) {
            const int u = bx + lx, v = by + ly;
            const float2* centre = tile + (ly + halo) * pitch + (lx + halo);
            const PixelFit<double> r =
                fit_pixel<double, R>(d, LdsSource{centre, pitch}, u, v, centre->x, d.residual != nullptr);
            store_pixel(d, static_cast<int64_t>(v) * d.width + u, r);
        }
        __syncthreads();   // the next entry re-stages the LDS region
    }
}

template <int R>
hipError_t launch_radius(const FitDesc& d, uint32_t* entries, uint64_t* masks, uint32_t* counts,
                         hipStream_t st, hipEvent_t* ev) {
    const int halo = R > d.normal_radius ? R : d.normal_radius;
    const uint32_t tiles_x = (d.width + kTileW - 1) / kTileW;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    if (d.precision == 2) {
        constexpr int TH = 4;
        const size_t lds = sizeof(float2) * (kTileW + 2 * halo) * (TH + 2 * halo);
        dim3 grid(tiles_x, (d.height + TH - 1) / TH);
        hipLaunchKernelGGL((fit_tile<double, R, TH>), grid, dim3(kTileW * TH), lds, st, d, entries,
                           masks, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
        return hipSuccess;
    }
    constexpr int TH = 16;
    const size_t lds = sizeof(float2) * (kTileW + 2 * halo) * (TH + 2 * halo);
    dim3 grid(tiles_x, (d.height + TH - 1) / TH);
    hipLaunchKernelGGL((fit_tile<float, R, TH>), grid, dim3(kTileW * TH), lds, st, d, entries, masks,
                       counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if (d.precision == 0) {
        // One workgroup per listed block in the worst case, capped; each loops over entries.
        const uint32_t blocks = tiles_x * grid.y * (TH / 4);
        const uint32_t nwg = blocks < 8192u ? blocks : 8192u;
        const size_t lds64 = sizeof(float2) * (kTileW + 2 * halo) * (4 + 2 * halo);
        hipLaunchKernelGGL(refit_blocks_f64<R>, dim3(nwg), dim3(64), lds64, st, d, entries, masks,
                           counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    return hipSuccess;
}

template <int... Rs>
hipError_t dispatch_radius(int r, const FitDesc& d, uint32_t* entries, uint64_t* masks,
                           uint32_t* counts, hipStream_t st, hipEvent_t* ev,
                           std::integer_sequence<int, Rs...>) {
    hipError_t e = hipErrorInvalidValue;
    (void)((r == Rs + 1 ? (e = launch_radius<Rs + 1>(d, entries, masks, counts, st, ev), true) : false) || ...);
    return e;
}

}  // namespace

int64_t refit_capacity(int width, int height) {
    const int64_t tiles_x = (width + kTileW - 1) / kTileW;
    const int64_t tiles_y = (height + 15) / 16;
    return tiles_x * tiles_y * 4;
}

hipError_t launch_fit(const FitDesc& d, uint32_t* entries, uint64_t* masks, uint32_t* counts,
                      hipStream_t stream, hipEvent_t* events) {
    if (d.precision != 2) {
        hipLaunchKernelGGL(zero_counts, dim3(1), dim3(1), 0, stream, counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return dispatch_radius(d.radius, d, entries, masks, counts, stream, events,
                           std::make_integer_sequence<int, kMaxRadius>{});
}

}  // namespace qc
