// fit_device.h -- device code shared by the gfx950 kernels for per-pixel robust
// quadric-patch curvature fitting (Spek, Li, Drummond, "A Fast Method For Computing
// Principal Curvatures From Range Images", Section 3).
//
// The FP32 pass stages a depth tile plus its halo in LDS and one lane runs a pixel's
// whole fit; pixels whose FP32 fit is judged unreliable are listed, and the FP64 pass
// re-runs the identical sequence of steps in double precision for them, four lanes per
// pixel (FP64 mode: one lane per pixel, every pixel).
//
// Arithmetic layout (exact in real arithmetic to the method's steps; chosen for FP32):
//  * Centring (Eq. (5)) is done on the integer/native depth samples: with D the depth in
//    native units and s metres per unit, p' = P_i - P_c = s * G0 * m with
//    m = ((u_i-u_c) D_i, (v_i-v_c) D_i, D_i - D_c), which is exact for U16 and F16 input,
//    and G0 = [[1/fx, 0, (u_c-cx)/fx], [0, 1/fy, (v_c-cy)/fy], [0, 0, 1]].
//  * Lengths are measured in units of h = sqrt(k), so the patch coefficients become A h,
//    B h, C h, t_z / h and the weight of Eq. (11) becomes 1/(1 + e^2); Gauss-Newton is
//    invariant under this rescaling, so the iterates are the same.
//  * Each neighbour contributes sqrt(w) J to the normal equations (H = sum (sqrt w J)
//    (sqrt w J)^T, g = sum (sqrt w J)(sqrt w e)), with w = 1/(1 + e^2): the factor k of
//    Eq. (11) cancels in (J^T W J)^{-1} J^T W e.
//  * The 6x6 solve is Jacobi-equilibrated LDL^T; the pivot ratio estimates the
//    condition number that decides the FP64 recomputation.
#pragma once

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
// Relative distance from the rejection bound R within which an FP32 decision e^2 < R is
// not trusted (measured: decisions 1.6e-5 from R have gone the other way in FP64).
constexpr float kRejectMargin = 1e-4f;
// ... and within kRejectAbs * sqrt(R) * m of it, m the window's largest |terms| of the local
// depth coordinate (in units of h, doubled as in the fit's loop): FP32 rounds e to about
// 2^-24 m, which sets the error of e^2 near the bound and of the mean that sets R; it
// exceeds the relative margin where the residuals are at the rounding level of the input
// (noiseless float depth) or the surface is seen edge-on (large, cancelling terms).
constexpr float kRejectAbs = 1e-6f;
// Further reasons to recompute an FP32 fit in FP64 (measured against the oracle): a normal
// regression with det M <= kNormalDetMin (tr M)^2 starts the fit from an initial normal that
// FP32 and FP64 place differently enough to end apart, and an update before the last one
// larger than kPrevStepFactor times the last-update bound means the fit was still moving
// far one step before the end, where an FP32 step lands differently from the FP64 one.
constexpr float kNormalDetMin = 1e-2f;
constexpr float kPrevStepFactor = 1.5f;
// With rejection the point set changes between iterations, and a fit that still moves far
// after its first iteration (any later update beyond kRejectSettleFactor times the
// last-update bound) can follow a different path in FP32 than in FP64 and end far apart.
constexpr float kRejectSettleFactor = 5.0f;

// Compile-time tuning (measured defaults): waves per SIMD of the FP32 pass and of the
// FP64 recomputation, neighbours per unrolled step of the FP64 window loops.
#ifndef QC_F32_WAVES_PER_EU
#define QC_F32_WAVES_PER_EU 3
#endif
#ifndef QC_F64_WAVES_PER_EU
#define QC_F64_WAVES_PER_EU 2
#endif
#ifndef QC_F64_UNROLL
#define QC_F64_UNROLL 3
#endif

// ---------------------------------------------------------------------------- scalars
template <typename T> __host__ __device__ __forceinline__ T fmaT(T a, T b, T c);
template <> __host__ __device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __host__ __device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/sqrt(x) with 1/sqrt(+inf) = 0 (the weight of a missing neighbour).
template <typename T> __device__ __forceinline__ T rsqrtT(T x);
template <> __device__ __forceinline__ float rsqrtT(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate y refined by the second-order expansion of (1 - e)^(-1/2),
// e = 1 - x y^2, i.e. y (1 + e/2 + 3 e^2 / 8); written without branches so that it stays
// in the straight-line code of the window loop.
template <> __device__ __forceinline__ double rsqrtT(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    const double r = __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
    return x < INFINITY ? r : 0.0;
}

// 1/x for finite x > 0: hardware estimate y refined by y (1 + e + e^2), e = 1 - x y
// (third-order convergence, so the estimate's error is cubed).
__device__ __forceinline__ double rcp_pos(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, __builtin_fma(e, e, e), y);
}

template <typename T> __device__ __forceinline__ T sqrtT(T x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T sinT(T x) { return sin(x); }

// Coefficients 1/n! (n! is exact in double up to 20!, so each is correctly rounded).
__host__ __device__ constexpr double inv_factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

// The two factors of the exact rotation Exp([w]x) with th^2 = |w|^2 < 1:
// st = sin(th)/th = sum_n (-th^2)^n / (2n+1)!, c1 = (1 - cos th)/th^2 = sum_n (-th^2)^n / (2n+2)!,
// summed by Horner's rule up to the first omitted term below the type's rounding (for
// th^2 <= 1 that term is at most 1/(2N+1)! resp. 1/(2N+2)!: N = 5 in FP32, 9 in FP64).
template <typename T>
__host__ __device__ __forceinline__ void rotation_series(T th2, T& st, T& c1) {
    constexpr int N = sizeof(T) == 4 ? 5 : 9;
    const T nx = -th2;
    T s = T(inv_factorial(2 * N - 1)), c = T(inv_factorial(2 * N));
#pragma unroll
    for (int n = N - 2; n >= 0; --n) {
        s = fmaT(s, nx, T(inv_factorial(2 * n + 1)));
        c = fmaT(c, nx, T(inv_factorial(2 * n + 2)));
    }
    st = s;
    c1 = c;
}

// ---------------------------------------------------------------------------- depth
__device__ __forceinline__ float load_sample(const FitDesc& d, int x, int y) {
    const char* row = static_cast<const char*>(d.depth) + static_cast<int64_t>(y) * d.pitch;
    if (d.format == 0) return static_cast<float>(reinterpret_cast<const uint16_t*>(row)[x]);
    if (d.format == 1) return __half2float(reinterpret_cast<const __half*>(row)[x]);
    return reinterpret_cast<const float*>(row)[x];
}

// (D, c): D = depth in native units; c = 1 for a valid sample and +inf for a missing one
// (outside the image, zero or non-finite).  With lengths in units of sqrt(k) the weight
// of Eq. (11) is 1/(c + e^2): a missing neighbour gets weight exactly 0 without a branch.
__device__ __forceinline__ float2 sample_or_missing(const FitDesc& d, int x, int y) {
    if (x < 0 || y < 0 || x >= d.width || y >= d.height) return make_float2(0.f, INFINITY);
    float z = load_sample(d, x, y);
    bool ok = z > 0.f && z <= 3.0e38f;   // excludes 0, negatives, inf and NaN
    return make_float2(ok ? z : 0.f, ok ? 1.f : INFINITY);
}

__device__ __forceinline__ bool present(float2 t) { return t.y == 1.f; }

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
// The window sampled at a stride: row(j)[i] is pixel (u + i step, v + j step).
struct LdsStridedRow {
    const float2* p;
    int step;
    __device__ __forceinline__ float2 operator[](int i) const { return p[i * step]; }
};
struct LdsStridedSource {
    const float2* centre;
    int pitch, step;
    __device__ __forceinline__ LdsStridedRow row(int j) const {
        return LdsStridedRow{centre + j * step * pitch, step};
    }
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
    Real Dc, g00, g02, g11, g12, g22, h, ih;
};

// A pixel's fit may be shared by NP consecutive lanes: lane `part` takes the window rows
// dv = -r + part, -r + part + NP, ..., and sum() adds a value over the group by a
// butterfly, which leaves every lane of the group with the same bits (the additions are
// the same pairs in the same order up to commutation).  NP = 1 is one lane per pixel.
//
// Step M of the butterfly adds the value of a partner lane in the other half of the
// aligned group of 2M lanes.  Every lane of an M-lane half already holds that half's sum,
// so any partner there will do: the xor partner within a quad for M = 1, 2 (DPP quad
// permutations), the mirror image within 8 or 16 lanes for M = 4, 8 (DPP row_half_mirror,
// row_mirror), a cross-row shuffle beyond.  Each source lane lies in the same row of 16,
// so every lane is written and the old value of the destination is never used.
template <int M>
__device__ __forceinline__ int dpp_partner(int v) {
    constexpr int ctrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : M == 4 ? 0x141 : 0x140;
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}
template <int M, typename T>
__device__ __forceinline__ T partner(T x) {
    if constexpr (M <= 8) {
        if constexpr (sizeof(T) == 8) {
            const uint64_t b = __builtin_bit_cast(uint64_t, x);
            const uint32_t lo = static_cast<uint32_t>(dpp_partner<M>(static_cast<int>(b)));
            const uint32_t hi = static_cast<uint32_t>(dpp_partner<M>(static_cast<int>(b >> 32)));
            return __builtin_bit_cast(T, (static_cast<uint64_t>(hi) << 32) | lo);
        } else {
            return __builtin_bit_cast(T, dpp_partner<M>(__builtin_bit_cast(int, x)));
        }
    } else {
        return __shfl_xor(x, M);
    }
}

template <int NP>
struct LaneGroup {
    int part;
    template <typename T>
    __device__ __forceinline__ T sum(T x) const {
        if constexpr (NP > 1) x += partner<1>(x);
        if constexpr (NP > 2) x += partner<2>(x);
        if constexpr (NP > 4) x += partner<4>(x);
        if constexpr (NP > 8) x += partner<8>(x);
        if constexpr (NP > 16) x += partner<16>(x);
        if constexpr (NP > 32) x += partner<32>(x);
        return x;
    }
};

// Loops over this lane's window rows, calling row_end() after each row -- after each pair
// of rows for FP32; RC > 0 fixes R at compile time.  A row is fully unrolled for FP32
// (U = 0); FP64 unrolls it U neighbours at a time (U >= 2), so that the dependency chains
// of several neighbours interleave, or keeps it rolled (U = 1), to stay within the
// register file.
struct NoRowEnd {
    __device__ __forceinline__ void operator()() const {}
};

template <int RC, int U, int NP, typename Src, typename F, typename G = NoRowEnd>
__device__ __forceinline__ void for_window(const Src& src, int radius, const LaneGroup<NP>& grp,
                                           F&& f, G&& row_end = G{}) {
    const int r = RC > 0 ? RC : radius;
    const int first = NP > 1 ? -r + grp.part : -r;
    // The row loop stays rolled: unrolled, a short body (e.g. the mean of e^2 ahead of the
    // accumulation) would keep a whole window of samples live across the two passes.
    if constexpr (RC > 0 && U == 0) {
        // two rows per step, row_end() after each pair (and after a last, unpaired row)
#pragma unroll 1
        for (int dv = first; dv <= r; dv += 2 * NP) {
            {
                auto row = src.row(dv);
#pragma unroll
                for (int du = -RC; du <= RC; ++du) f(row[du], du, dv);
            }
            if (dv + NP <= r) {
                auto row = src.row(dv + NP);
#pragma unroll
                for (int du = -RC; du <= RC; ++du) f(row[du], du, dv + NP);
            }
            row_end();
        }
    } else if constexpr (U >= 2) {
        // U neighbours at a time; the samples of the next U are read before this group is
        // processed, so their latency overlaps its arithmetic (reads past the row's end
        // are clamped to its last sample and not used)
        const int n = 2 * r + 1, nfull = n / U * U;
#pragma unroll 1
        for (int dv = first; dv <= r; dv += NP) {
            auto row = src.row(dv);
            float2 cur[U];
#pragma unroll
            for (int k = 0; k < U; ++k) cur[k] = row[min(k, n - 1) - r];
#pragma unroll 1
            for (int i0 = 0; i0 < nfull; i0 += U) {
                float2 nxt[U];
#pragma unroll
                for (int k = 0; k < U; ++k) nxt[k] = row[min(i0 + U + k, n - 1) - r];
#pragma unroll
                for (int k = 0; k < U; ++k) f(cur[k], i0 + k - r, dv);
#pragma unroll
                for (int k = 0; k < U; ++k) cur[k] = nxt[k];
            }
#pragma unroll
            for (int k = 0; k < U - 1; ++k)
                if (nfull + k < n) f(cur[k], nfull + k - r, dv);
            row_end();
        }
    } else {
        // rolled row: the next sample's LDS read is issued before this one is used
        for (int dv = first; dv <= r; dv += NP) {
            auto row = src.row(dv);
            float2 cur = row[-r];
#pragma unroll 1
            for (int du = -r; du <= r; ++du) {
                const float2 nxt = row[du < r ? du + 1 : du];
                f(cur, du, dv);
                cur = nxt;
            }
            row_end();
        }
    }
}

// The 26 distinct sums of the normal equations as products of the seven scaled terms
// v = sqrt(w) (J0, J1, 1, sx^2, sx sy, sy^2, e): H00 H01 H03 H04 H05 H11 H13 H14 H15 H33
// H34 H35 H45 H55, S0..S5 (with v2 = sqrt(w)), G0..G5 (with v6 = sqrt(w) e).
constexpr int kSums = 26;
constexpr int kSumA[kSums] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 3, 3, 3, 4, 5, 0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 5};
constexpr int kSumB[kSums] = {0, 1, 3, 4, 5, 1, 3, 4, 5, 3, 4, 5, 5, 5, 2, 2, 2, 2, 2, 2, 6, 6, 6, 6, 6, 6};

// The pixel's fit, Section 3.2: initial normal (Eq. (7)), frame set-up, fixed number of
// re-weighted Gauss-Newton steps (Eqs. (8)-(11)), curvatures, refined normal.
// `nsrc` reads the (dense) initial-normal window, `src` the fit window; with STR the fit
// window is sampled at the stride d.stride (src indexes samples, not pixels), which is
// folded into the first two columns of the per-iteration map R'.
template <typename Real, int RC, int NP = 1, bool REJ = false, bool STR = false, typename NSrc,
          typename Src>
__device__ PixelFit<Real> fit_pixel(const FitDesc& d, const NSrc& nsrc, const Src& src, int u, int v,
                                    float Dc_f, bool want_residual,
                                    LaneGroup<NP> grp = LaneGroup<NP>{0}) {
    PixelFit<Real> out;
    const Real nan = Real(NAN);
    out.k1 = out.k2 = out.residual = nan;
    out.n[0] = out.n[1] = out.n[2] = nan;
    out.flags = 0;
    using Acc = double;   // normal-equation sums and the 6x6 solve
    const int radius = RC > 0 ? RC : d.radius;   // samples either side of the centre
    const int step = STR ? d.stride : 1;        // pixels between samples
    const bool fp32 = sizeof(Real) == 4;

    // ---- geometry (Eq. (5) centring on native samples, lengths in units of h)
    Geometry<Real> g;
    g.Dc = Real(Dc_f);
    const Real s = Real(d.scale);
    const Real fx = Real(d.fx), fy = Real(d.fy);
    g.h = sqrtT(Real(d.k));
    g.ih = Real(1) / g.h;
    const Real ihs = g.ih * s;
    g.g00 = ihs / fx;
    g.g02 = ihs * ((Real(u) - Real(d.cx)) / fx);
    g.g11 = ihs / fy;
    g.g12 = ihs * ((Real(v) - Real(d.cy)) / fy);
    g.g22 = ihs;

    // ---- initial normal, Section 3.2.1: regression z = a x + b y over the small window
    //      with mean-centred sums M, v; n0 = (-a, -b, 1) / sqrt(1 + a^2 + b^2)
    const int rn = d.normal_radius;
    Real cnt = 0, mx_ = 0, my_ = 0, mz_ = 0;
    for_window<0, 1>(nsrc, rn, grp, [&](float2 t, int du, int dv) {
        const Real ok = present(t) ? Real(1) : Real(0);
        const Real D = Real(t.x), dD = D - g.Dc;
        const Real px = fmaT(g.g00, Real(du) * D, g.g02 * dD);
        const Real py = fmaT(g.g11, Real(dv) * D, g.g12 * dD);
        const Real pz = g.g22 * dD;
        cnt += ok;
        mx_ = fmaT(ok, px, mx_);
        my_ = fmaT(ok, py, my_);
        mz_ = fmaT(ok, pz, mz_);
    });
    cnt = grp.sum(cnt);
    mx_ = grp.sum(mx_);
    my_ = grp.sum(my_);
    mz_ = grp.sum(mz_);
    if (cnt < Real(3)) return out;
    mx_ /= cnt; my_ /= cnt; mz_ /= cnt;
    Real M00 = 0, M01 = 0, M11 = 0, v0 = 0, v1 = 0;
    for_window<0, 1>(nsrc, rn, grp, [&](float2 t, int du, int dv) {
        const Real ok = present(t) ? Real(1) : Real(0);
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
    M00 = grp.sum(M00);
    M01 = grp.sum(M01);
    M11 = grp.sum(M11);
    v0 = grp.sum(v0);
    v1 = grp.sum(v1);
    const Real det = M00 * M11 - M01 * M01;
    const Real tr = M00 + M11;
    bool ill = false;
    if (!(det > Real(1e-12) * tr * tr)) {
        if (fp32) out.flags = kFlagIll;   // let FP64 decide
        return out;
    }
    if (fp32 && !(det > Real(kNormalDetMin) * tr * tr)) ill = true;
    const Real ia = (M11 * v0 - M01 * v1) / det;
    const Real ib = (M00 * v1 - M01 * v0) / det;
    const Real nsc = Real(1) / sqrtT(Real(1) + ia * ia + ib * ib);
    const Real n0x = -ia * nsc, n0y = -ib * nsc, n0z = nsc;

    // ---- enough neighbours for six parameters
    Real nfit = 0;
    for_window<RC, sizeof(Real) == 8 ? QC_F64_UNROLL : 0>(src, radius, grp,
                                      [&](float2 t, int, int) { nfit += present(t) ? Real(1) : Real(0); });
    nfit = grp.sum(nfit);
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
    Acc last_step = 0, prev_step = 0;     // sizes of the last two updates
    Acc later_step = 0;                   // largest update after the first (rejection)
    bool cond_ok = true;                  // pivot ratio within cond_max at every iteration
    bool near = false;                    // an FP32 rejection decision was too close to call
    // window half-extent r Z_c / fx in units of h
    const Acc hwin = Acc(radius * step) * Acc(g.Dc) * Acc(s) / Acc(fx) * Acc(g.ih);
    const Acc ihwin = Acc(1) / hwin;

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
            if constexpr (STR) {
                Rp[i][0] *= Real(step);
                Rp[i][1] *= Real(step);
            }
        }
        const Real Ah = Real(0.5) * A, Bh = Real(0.5) * B, Ch = Real(0.5) * C;
        // Rejection (Eq. (11) with R = 2 MSE, Section 3.2.3): R from the unweighted mean
        // of e^2 over the valid neighbours at the current parameters; none when it is 0.
        Real thresh = Real(INFINITY);
        Real zmag = 0;   // FP32: largest |terms| of the doubled local depth coordinate
        if constexpr (REJ) {
            Acc se = 0;
            Real rse = 0;
            for_window<RC, sizeof(Real) == 8 ? QC_F64_UNROLL : 0>(src, radius, grp, [&](float2 t, int du, int dv) {
                const Real D = Real(t.x), dD = D - g.Dc;
                const Real fdu = Real(du), fdv = Real(dv);
                const Real sx = fmaT(fmaT(Rp[0][0], fdu, Rp[0][1] * fdv), D, Rp[0][2] * dD);
                const Real sy = fmaT(fmaT(Rp[1][0], fdu, Rp[1][1] * fdv), D, Rp[1][2] * dD);
                const Real a2 = fmaT(Rp[2][0], fdu, Rp[2][1] * fdv), b2 = Rp[2][2] * dD;
                const Real sz2 = fmaT(a2, D, b2);
                const Real qz = fmaT(Real(0.5), sz2, tz);
                const Real ap = fmaT(Ah, sx, Bh * sy), cp = fmaT(Bh, sx, Ch * sy);
                const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz));
                if constexpr (sizeof(Real) == 4) {
                    rse = fmaT(e, present(t) ? e : Real(0), rse);
                    zmag = fmax(zmag, present(t) ? fabs(a2 * D) + fabs(b2) : Real(0));
                } else {
                    se += present(t) ? Acc(e * e) : Acc(0);
                }
            }, [&]() {
                // FP32: the sum of each pair of rows in FP32, the pairs in FP64 (as the
                // normal-equation sums below)
                if constexpr (sizeof(Real) == 4) {
                    se += Acc(rse);
                    rse = 0;
                }
            });
            se = grp.sum(se);
            const Acc mse = se / Acc(nfit);
            if (mse > Acc(0)) thresh = Real(Acc(2) * mse);
        }
        // FP32: the closest any decision e^2 < R came to the bound; a pixel with one too
        // close to be sure of is left to FP64
        Real gap = Real(INFINITY);
        // Normal-equation sums (kSumA / kSumB).  The FP32 path sums each pair of window
        // rows (2 (2r+1) terms) in FP32 and adds these partial sums in FP64: one sequence of
        // FP32 additions over the whole window (225 terms at r = 7) is the dominant rounding
        // error of an FP32 fit, while a row pair's error stays within a few times that of
        // the terms themselves; per neighbour this takes 26 FP32 FMAs instead of 7
        // conversions and 26 FP64 FMAs, and the 26 conversions and FP64 additions come
        // once per two rows.  The FP64 path accumulates in FP64 throughout.
        constexpr bool row_sums = sizeof(Real) == 4;
        Acc sum[kSums];
        Real rsum[kSums];
#pragma unroll
        for (int k = 0; k < kSums; ++k) {
            sum[k] = 0;
            rsum[k] = 0;
        }
        for_window<RC, sizeof(Real) == 8 ? QC_F64_UNROLL : 0>(src, radius, grp, [&](float2 t, int du, int dv) {
            // s = R' m with m = (du D, dv D, D - Dc), as (R'x0 du + R'x1 dv) D + R'x2 (D - Dc):
            // each term is rounded relative to itself, so a neighbour close to the centre
            // (small D - Dc) keeps its small coordinates accurate
            const Real D = Real(t.x);
            const Real dD = D - g.Dc;
            const Real fdu = Real(du), fdv = Real(dv);
            const Real sx = fmaT(fmaT(Rp[0][0], fdu, Rp[0][1] * fdv), D, Rp[0][2] * dD);
            const Real sy = fmaT(fmaT(Rp[1][0], fdu, Rp[1][1] * fdv), D, Rp[1][2] * dD);
            const Real sz2 = fmaT(fmaT(Rp[2][0], fdu, Rp[2][1] * fdv), D, Rp[2][2] * dD);
            const Real qz = fmaT(Real(0.5), sz2, tz);
            const Real ap = fmaT(Ah, sx, Bh * sy);          // (A qx + B qy) / 2
            const Real cp = fmaT(Bh, sx, Ch * sy);          // (B qx + C qy) / 2
            const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz)); // Eq. (6): A/2 qx^2 + B qx qy + C/2 qy^2 - qz
            Real c = Real(t.y);
            if constexpr (REJ) {
                const Real e2 = e * e;
                if constexpr (sizeof(Real) == 4) gap = fmin(gap, present(t) ? fabs(e2 - thresh) : Real(INFINITY));
                c = e2 < thresh ? c : Real(INFINITY);
            }
            const Real rw = rsqrtT(fmaT(e, e, c));          // sqrt of the weight, Eq. (11)
            const Real J0 = -fmaT(cp, sz2, sy);             // de/dtheta_x
            const Real J1 = fmaT(ap, sz2, sx);              // de/dtheta_y
            const Real xr = rw * sx, yr = rw * sy;
            const Real v[7] = {rw * J0, rw * J1, rw, xr * sx, xr * sy, yr * sy, rw * e};
            if constexpr (row_sums) {
#pragma unroll
                for (int k = 0; k < kSums; ++k) rsum[k] = fmaT(v[kSumA[k]], v[kSumB[k]], rsum[k]);
            } else {
                Acc va[7];
#pragma unroll
                for (int i = 0; i < 7; ++i) va[i] = Acc(v[i]);
#pragma unroll
                for (int k = 0; k < kSums; ++k) sum[k] = fmaT(va[kSumA[k]], va[kSumB[k]], sum[k]);
            }
        }, [&]() {
            // FP32: called after every pair of rows (the FP32 window loop takes two rows
            // per step); FP64: after every row, with nothing to flush
            if constexpr (row_sums) {
#pragma unroll
                for (int k = 0; k < kSums; ++k) {
                    sum[k] += Acc(rsum[k]);
                    rsum[k] = 0;
                }
            }
        });
        if constexpr (REJ && sizeof(Real) == 4)
            near |= thresh < Real(INFINITY) &&
                    gap <= fmax(Real(kRejectMargin) * thresh, Real(kRejectAbs) * sqrtT(thresh) * zmag);
        if constexpr (NP > 1) {
#pragma unroll
            for (int k = 0; k < kSums; ++k) sum[k] = grp.sum(sum[k]);
        }
        const Acc H00 = sum[0], H01 = sum[1], H03 = sum[2], H04 = sum[3], H05 = sum[4];
        const Acc H11 = sum[5], H13 = sum[6], H14 = sum[7], H15 = sum[8];
        const Acc H33 = sum[9], H34 = sum[10], H35 = sum[11], H45 = sum[12], H55 = sum[13];
        const Acc S0 = sum[14], S1 = sum[15], S2 = sum[16], S3 = sum[17], S4 = sum[18], S5 = sum[19];
        const Acc G0 = sum[20], G1 = sum[21], G2 = sum[22], G3 = sum[23], G4 = sum[24], G5 = sum[25];
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
        // Column j keeps U[i][j] = L[i][j] dp[j] (the sum before the division by the pivot)
        // beside L[i][j], so that every elimination step is one fused multiply-add.
        Acc dsc[6];
        bool singular = false;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const Acc hii = Hm[i][i];
            singular |= !(hii > Acc(0));
            const Acc r = rsqrtT(hii > Acc(0) ? hii : Acc(1));
            dsc[i] = hii > Acc(0) ? r : Acc(0);
        }
        Acc L[6][6], U[6][6], dp[6], idp[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            Acc dj = Acc(1);   // equilibrated diagonal
#pragma unroll
            for (int k = 0; k < j; ++k) dj = fmaT(-L[j][k], U[j][k], dj);
            dp[j] = dj;
            const Acc rj = rcp_pos(dj > Acc(0) ? dj : Acc(1));
            const Acc idj = dj > Acc(0) ? rj : Acc(0);
            idp[j] = idj;
#pragma unroll
            for (int i = j + 1; i < 6; ++i) {
                Acc sij = dsc[i] * dsc[j] * Hm[j][i];
#pragma unroll
                for (int k = 0; k < j; ++k) sij = fmaT(-L[i][k], U[j][k], sij);
                U[i][j] = sij;
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
        cond_ok = cond_ok && pmax <= Acc(d.cond_max) * pmin;
        Acc y[6], b[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            Acc sy = dsc[i] * gv[i];
#pragma unroll
            for (int k = 0; k < i; ++k) sy = fmaT(-L[i][k], y[k], sy);
            y[i] = sy;
        }
#pragma unroll
        for (int i = 5; i >= 0; --i) {
            Acc sb = y[i] * idp[i];
#pragma unroll
            for (int k = i + 1; k < 6; ++k) sb = fmaT(-L[k][i], b[k], sb);
            b[i] = sb;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) b[i] *= dsc[i];
        // Size of the update in window units (angles in radians, t_z in window
        // half-extents, curvatures times the half-extent): how far from converged.
        prev_step = last_step;
        last_step = fmax(fmax(fabs(b[0]), fabs(b[1])),
                         fmax(fabs(b[2]) * ihwin, hwin * fmax(fmax(fabs(b[3]), fabs(b[4])), fabs(b[5]))));
        if constexpr (REJ) later_step = it > 0 ? fmax(later_step, last_step) : later_step;

        // Update (Section 3.2.3): R <- Exp([(-b0, -b1, 0)]x) R (exact Rodrigues),
        // t_z -= b2, A -= b3, B -= b4, C -= b5.
        {
            const Real w0 = Real(-b[0]), w1 = Real(-b[1]);
            const Real th2 = w0 * w0 + w1 * w1;
            Real st, c1;
            if (th2 < Real(1)) {
                rotation_series(th2, st, c1);
            } else {
                const Real th = sqrtT(th2);
                const Real ith = Real(1) / th;
                st = sinT(th) * ith;                        // sin(th)/th
                const Real sh = sinT(Real(0.5) * th) * ith; // sin(th/2)/th
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
            if constexpr (STR) {
                Rp[i][0] *= Real(step);
                Rp[i][1] *= Real(step);
            }
        }
        const Real Ah = Real(0.5) * A, Bh = Real(0.5) * B, Ch = Real(0.5) * C;
        Real thresh = Real(INFINITY);
        Real zmag = 0;   // FP32: as in the fit's loop (the coordinate here is not doubled)
        if constexpr (REJ) {
            Acc se = 0;
            for_window<RC, sizeof(Real) == 8 ? QC_F64_UNROLL : 0>(src, radius, grp, [&](float2 t, int du, int dv) {
                const Real D = Real(t.x), dD = D - g.Dc;
                const Real mx = Real(du) * D, my = Real(dv) * D;
                const Real sx = fmaT(Rp[0][0], mx, fmaT(Rp[0][1], my, Rp[0][2] * dD));
                const Real sy = fmaT(Rp[1][0], mx, fmaT(Rp[1][1], my, Rp[1][2] * dD));
                const Real sz = fmaT(Rp[2][0], mx, fmaT(Rp[2][1], my, Rp[2][2] * dD));
                const Real qz = sz + tz;
                const Real ap = fmaT(Ah, sx, Bh * sy), cp = fmaT(Bh, sx, Ch * sy);
                const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz));
                se += present(t) ? Acc(e * e) : Acc(0);
                if constexpr (sizeof(Real) == 4)
                    zmag = fmax(zmag, present(t) ? Real(2) * (fabs(Rp[2][0] * mx) + fabs(Rp[2][1] * my) + fabs(Rp[2][2] * dD))
                                                 : Real(0));
            });
            se = grp.sum(se);
            const Acc mse = se / Acc(nfit);
            if (mse > Acc(0)) thresh = Real(Acc(2) * mse);
        }
        Real sw = 0, swe = 0, gap = Real(INFINITY);
        for_window<RC, sizeof(Real) == 8 ? QC_F64_UNROLL : 0>(src, radius, grp, [&](float2 t, int du, int dv) {
            const Real D = Real(t.x), dD = D - g.Dc;
            const Real mx = Real(du) * D, my = Real(dv) * D;
            const Real sx = fmaT(Rp[0][0], mx, fmaT(Rp[0][1], my, Rp[0][2] * dD));
            const Real sy = fmaT(Rp[1][0], mx, fmaT(Rp[1][1], my, Rp[1][2] * dD));
            const Real sz = fmaT(Rp[2][0], mx, fmaT(Rp[2][1], my, Rp[2][2] * dD));
            const Real qz = sz + tz;
            const Real ap = fmaT(Ah, sx, Bh * sy), cp = fmaT(Bh, sx, Ch * sy);
            const Real e = fmaT(ap, sx, fmaT(cp, sy, -qz));
            Real c = Real(t.y);
            if constexpr (REJ) {
                const Real e2 = e * e;
                if constexpr (sizeof(Real) == 4) gap = fmin(gap, present(t) ? fabs(e2 - thresh) : Real(INFINITY));
                c = e2 < thresh ? c : Real(INFINITY);
            }
            const Real rw = rsqrtT(fmaT(e, e, c));
            const Real w = rw * rw;
            sw += w;
            swe = fmaT(w * e, e, swe);
        });
        if constexpr (REJ && sizeof(Real) == 4)
            near |= thresh < Real(INFINITY) &&
                    gap <= fmax(Real(kRejectMargin) * thresh, Real(kRejectAbs) * sqrtT(thresh) * zmag);
        sw = grp.sum(sw);
        swe = grp.sum(swe);
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
    if (fp32 && (ill || near || !cond_ok || !(last_step <= Acc(d.step_max)) ||
                 !(prev_step <= Acc(kPrevStepFactor) * Acc(d.step_max)) ||
                 (REJ && !(later_step <= Acc(kRejectSettleFactor) * Acc(d.step_max)))))
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
__global__ void zero_counts(uint32_t* counts) {
    if (threadIdx.x < kCountWords) counts[threadIdx.x] = 0u;
}

// FP64 pass: each listed pixel is fitted by a group of kRefitLanes lanes that split its
// window rows, so a wave takes kChunk listed pixels at a time.
#ifndef QC_REFIT_LANES
#define QC_REFIT_LANES 4
#endif
constexpr int kRefitLanes = QC_REFIT_LANES;
constexpr uint32_t kChunk = 64 / kRefitLanes;

// Stages the depth samples of a (w + 2 halo) x (h + 2 halo) region whose top-left pixel
// is (x0, y0) into LDS as (D, c) pairs.
__device__ __forceinline__ void stage_region(const FitDesc& d, float2* lds, int x0, int y0,
                                             int pitch, int rows) {
    for (int i = threadIdx.x; i < pitch * rows; i += blockDim.x) {
        const int ly = i / pitch, lx = i - ly * pitch;
        lds[i] = sample_or_missing(d, x0 + lx, y0 + ly);
    }
    __syncthreads();
}

// The same for the FP64 kernels, whose workgroups are one wave: each lane reads B samples
// before it writes any, so that their loads are in flight together (one short loop per
// tile instead of one memory round trip per sample).  Coordinates outside the image are
// clamped for the read and marked missing.
template <typename T>
__device__ __forceinline__ float sample_value(T x) { return static_cast<float>(x); }
template <>
__device__ __forceinline__ float sample_value(__half x) { return __half2float(x); }

template <typename T, int B>
__device__ __forceinline__ void stage_batched(const FitDesc& d, float2* lds, int x0, int y0,
                                              int pitch, int total) {
    const float inv_pitch = 1.f / static_cast<float>(pitch);
    const int step = static_cast<int>(blockDim.x);
    for (int i0 = threadIdx.x; i0 < total; i0 += B * step) {
        float z[B];
        bool in[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int i = min(i0 + k * step, total - 1);
            // i / pitch for i < 2^16: (i + 1/2) / pitch lies at least 1/(2 pitch) away
            // from an integer, far more than the rounding of the float product
            const int ly = static_cast<int>((static_cast<float>(i) + 0.5f) * inv_pitch);
            const int x = x0 + i - ly * pitch, y = y0 + ly;
            in[k] = x >= 0 && y >= 0 && x < d.width && y < d.height;
            const int xc = min(max(x, 0), d.width - 1), yc = min(max(y, 0), d.height - 1);
            const T* row = reinterpret_cast<const T*>(static_cast<const char*>(d.depth) +
                                                      static_cast<int64_t>(yc) * d.pitch);
            z[k] = sample_value(row[xc]);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int i = i0 + k * step;
            const bool ok = in[k] && z[k] > 0.f && z[k] <= 3.0e38f;
            if (i < total) lds[i] = make_float2(ok ? z[k] : 0.f, ok ? 1.f : INFINITY);
        }
    }
}
__device__ __forceinline__ void stage_region_wave(const FitDesc& d, float2* lds, int x0, int y0,
                                                  int pitch, int rows) {
    constexpr int B = 8;
    if (d.format == 0) stage_batched<uint16_t, B>(d, lds, x0, y0, pitch, pitch * rows);
    else if (d.format == 1) stage_batched<__half, B>(d, lds, x0, y0, pitch, pitch * rows);
    else stage_batched<float, B>(d, lds, x0, y0, pitch, pitch * rows);
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

__device__ __forceinline__ int tiles_across(const FitDesc& d) {
    return (d.width + d.tile_w - 1) / d.tile_w;
}

// One tile of tw x (blockDim.x / tw) pixels, halo staged in LDS, one lane per pixel.  In
// MIXED precision the pixels whose FP32 fit is unreliable are not stored but listed: one
// list entry for the tile with a 256-bit mask of them (bit t = thread t = pixel
// (t % tw, t / tw)), and one record per 16 of its ranks naming the entry.
template <typename Real, int R, bool REJ = false, bool STR = false>
__device__ __forceinline__ void fit_tile_body(const FitDesc& d, int tx, int ty, uint32_t frame,
                                              const RefitList& list) {
    extern __shared__ float2 tile[];
    __shared__ uint64_t wave_masks[4];
    const int tw = d.tile_w, th = blockDim.x / tw;
    const int halo = max(R * (STR ? d.stride : 1), d.normal_radius);
    const int pitch = tw + 2 * halo;
    if constexpr (sizeof(Real) == 8)
        stage_region_wave(d, tile, tx * tw - halo, ty * th - halo, pitch, th + 2 * halo);
    else
        stage_region(d, tile, tx * tw - halo, ty * th - halo, pitch, th + 2 * halo);
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int u = tx * tw + lx, v = ty * th + ly;
    const bool mixed = sizeof(Real) == 4 && d.precision == 0;
    bool recompute = false;
    if (u < d.width && v < d.height) {
        const float2* centre = tile + (ly + halo) * pitch + (lx + halo);
        PixelFit<Real> r;
        if (!present(*centre)) {
            r = missing_pixel<Real>();
        } else if constexpr (STR) {
            r = fit_pixel<Real, R, 1, REJ, true>(d, LdsSource{centre, pitch},
                                                 LdsStridedSource{centre, pitch, d.stride}, u, v,
                                                 centre->x, d.residual != nullptr);
        } else {
            const LdsSource src{centre, pitch};
            r = fit_pixel<Real, R, 1, REJ>(d, src, src, u, v, centre->x, d.residual != nullptr);
        }
        recompute = mixed && (r.flags & kFlagIll) != 0;
        if (!recompute) store_pixel(d, static_cast<int64_t>(v) * d.width + u, r);
    }
    if constexpr (sizeof(Real) == 4) {
        if (mixed) {
            const uint64_t mask = __ballot(recompute);
            if ((threadIdx.x % 64) == 0) wave_masks[threadIdx.x / 64] = mask;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint64_t m[4];
                uint32_t n = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    m[w] = wave_masks[w];
                    n += static_cast<uint32_t>(__popcll(m[w]));
                }
                if (n != 0) {
                    // one 64-bit add takes the entry slot (high word) and the rank (low
                    // word); ranks advance by n rounded up to whole chunks
                    const uint32_t padded = (n + kChunk - 1) / kChunk * kChunk;
                    const unsigned long long old = atomicAdd(
                        reinterpret_cast<unsigned long long*>(list.counts), (1ull << 32) | padded);
                    atomicAdd(&list.counts[4], n);
                    const uint32_t slot = static_cast<uint32_t>(old >> 32);
                    const uint64_t entry = (frame << 24) | static_cast<uint32_t>(ty * tiles_across(d) + tx);
                    for (uint32_t c = 0; c < padded / kChunk; ++c)
                        list.chunks[static_cast<uint32_t>(old) / kChunk + c] = (entry << 32) | (slot << 8) | c;
#pragma unroll
                    for (int w = 0; w < 4; ++w) list.masks[4 * slot + w] = m[w];
                }
            }
            __syncthreads();   // wave_masks is reused by the next tile of a persistent loop
        }
    }
}

// Calls f(std::integral_constant<int, r>) for the window radius r in 1..kMaxRadius.
template <typename F, int... Rs>
__device__ __forceinline__ void with_radius(int r, F&& f, std::integer_sequence<int, Rs...>) {
    (void)((r == Rs + 1 ? (f(std::integral_constant<int, Rs + 1>{}), true) : false) || ...);
}
template <typename F>
__device__ __forceinline__ void with_radius(int r, F&& f) {
    with_radius(r, f, std::make_integer_sequence<int, kMaxRadius>{});
}

// ---------------------------------------------------------------------------- FP64 pass
// The FP64 pass takes kChunk consecutive ranks at a time per wave from counts[3]; as the
// ranks of an entry are padded to whole chunks, a chunk holds up to kChunk listed pixels
// of one tile, so the work is shared out chunk by chunk whatever the tiles' loads.

// Position (0..63) of the n-th set bit (n counted from 0) of m; m has more than n bits.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int n) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint64_t low = m & ((uint64_t{1} << width) - 1);
        const int c = __popcll(low);
        if (n >= c) {
            n -= c;
            m >>= width;
            pos += width;
        } else {
            m = low;
        }
    }
    return pos;
}

// The chunk of ranks that starts at `base` (a multiple of kChunk below counts[0]), the
// same in every lane: its entry ((frame << 24) | tile), the entry's slot in the masks, and
// the number of listed pixels of the entry before the chunk.
struct Chunk {
    uint32_t entry, slot, first;
};
__device__ __forceinline__ Chunk chunk_at(const RefitList& list, uint32_t base) {
    const uint64_t rec = list.chunks[base / kChunk];
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(rec));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(rec >> 32));
    return Chunk{hi, lo >> 8, (lo & 0xffu) * kChunk};
}

// Thread (pixel of the tile) of the n-th listed pixel of an entry's 256-bit mask
// (w0, w1, w2, w3), or -1 when the entry lists no more than n pixels.
__device__ __forceinline__ int listed_thread(uint64_t w0, uint64_t w1, uint64_t w2, uint64_t w3, int n) {
    const int c0 = __popcll(w0), c1 = c0 + __popcll(w1), c2 = c1 + __popcll(w2);
    const int c3 = c2 + __popcll(w3);
    if (n >= c3) return -1;
    if (n < c0) return nth_set_bit(w0, n);
    if (n < c1) return 64 + nth_set_bit(w1, n - c0);
    if (n < c2) return 128 + nth_set_bit(w2, n - c1);
    return 192 + nth_set_bit(w3, n - c2);
}

// Ranks of the FP64 passes, whose workgroups are one wave each: the first kChunk ranks
// of wave b are b kChunk (no atomic at the start, where the whole grid asking one counter
// at once would queue behind it); each later chunk is the next kChunk ranks after the
// first round, counted by `counter` (the same value in every lane).
__device__ __forceinline__ uint32_t first_ranks() { return blockIdx.x * kChunk; }
__device__ __forceinline__ uint32_t next_ranks(uint32_t* counter) {
    uint32_t base = 0;
    if ((threadIdx.x % 64) == 0) base = atomicAdd(counter, kChunk);
    return __builtin_amdgcn_readfirstlane(base) + gridDim.x * kChunk;
}

// FP64 recomputation of one chunk of a batch: the chunk lies in one entry, hence in one
// tile of one frame, so the frame's descriptor and window radius are uniform across the
// wave.  The wave stages that tile plus halo in its LDS `region` (sized by the host for
// the largest region of the batch) and fits its pixels from there: this lane's pixel is
// the n-th listed in the entry's mask w (none for the lanes of a part-filled chunk).
template <int R>
__device__ __forceinline__ void refit_chunk(const FitDesc& d, uint32_t tile, const uint64_t (&w)[4], int n,
                                            const LaneGroup<kRefitLanes>& grp, float2* region) {
    const int tw = d.tile_w, th = 256 / tw;
    const int across = tiles_across(d);
    const int bx = static_cast<int>(tile % across) * tw, by = static_cast<int>(tile / across) * th;
    const int halo = max(R, d.normal_radius);
    const int pitch = tw + 2 * halo;
    stage_region_wave(d, region, bx - halo, by - halo, pitch, th + 2 * halo);
    const int thread = listed_thread(w[0], w[1], w[2], w[3], n);
    if (thread >= 0) {
        const int lx = thread % tw, ly = thread / tw;
        const float2* centre = region + (ly + halo) * pitch + (lx + halo);
        const LdsSource src{centre, pitch};
        const PixelFit<double> r = fit_pixel<double, R, kRefitLanes>(d, src, src, bx + lx, by + ly, centre->x,
                                                                     d.residual != nullptr, grp);
        if (grp.part == 0) store_pixel(d, static_cast<int64_t>(by + ly) * d.width + bx + lx, r);
    }
    __syncthreads();   // the next chunk re-stages the region
}

inline size_t lds_bytes(int tile_w, int tile_h, int halo) {
    return sizeof(float2) * static_cast<size_t>(tile_w + 2 * halo) * static_cast<size_t>(tile_h + 2 * halo);
}

}  // namespace
}  // namespace qc
