// Tile engine: the direct sums behind the four interactions of paper §5
// (eq. PP, PC, CP, CC) and the direct method of §1.
//
// All four interactions are sums  out(t) = sum_s K(t, s) w_s  of one target
// set against a list of source sets (paper §5 notes they are all direct
// sums).  One workgroup owns one target cell:
//   near kernel: targets = the particles of a target leaf; sources = the
//                particles of its PP cells (one launch), or the proxies (with
//                proxy weights) of its PC cells (a later launch, together
//                with the far kernel's blocks);
//   far kernel:  targets = the (p+1)^2 proxies of a target cell; sources =
//                the particles of its CP cells, then the proxies of its CC
//                cells; the result is its accumulated proxy potential
//                (eq. CP_CC_accumulated).
// The source list is flattened and staged through LDS in chunks, recentred
// at the target cell's centre in FP64 (and, in the FP32 form, converted to
// FP32 after recentring).  Block path (tile_body): thread (t, g) of the 256
// owns target t and the sources g, g+G, ... of each chunk; the G partial sums
// of a target are combined in FP64 in a fixed order.  One-wave-per-leaf path
// (tile_leaf_wave, many target leaves of at most 64 points): lane t owns
// target t and every source, the wave stages its own sources.  Same-set FP32
// plans evaluate each pair of leaves whose PP entry holds both ways once
// (sym_pairs, k_sym_merge).  Every order is fixed, so results are
// deterministic.
//
// Kernels (x, y unit vectors, 1 - x.y = |x-y|^2/2):
//   Poisson   -(1/4pi) ln(1 - x.y): coordinates scaled by 1/sqrt2 so that the
//             squared distance is 1 - x.y; FP32 uses log2 and folds ln 2 in.
//   Biot-Savart -(1/4pi) (x cross y)/(1 - x.y) = -(1/2pi) x cross sum (y-x) w/|x-y|^2.
//   1/|x-y|   rsqrt of the squared distance.
//   biharmonic (1/4pi) dilog((1 + x.y)/2): coordinates scaled by 1/2 so that
//             the squared distance is v = 1 - (1 + x.y)/2; see dilog_1m below.
//   SAL       (3 rw/(4pi re)) ((1-b0)/g - (a1-b1) ln(g/2 + g^2/4)), g = |x-y|:
//             with the 1/2 scaling g/2 = sqrt(v), so the bracket is
//             ((1-b0)/2) (1/sqrt(v) + q ln(sqrt(v) + v)), q = -2(a1-b1)/(1-b0).
// The self term (squared distance exactly 0) contributes nothing.
#include <atomic>
#include <mutex>
#include <type_traits>

#include "common.h"
#include "dev_util.h"

namespace csfmm {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 512;
constexpr int kMaxEntries = 256;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kLn2 = 0.69314718055994530942;

template <bool F32>
using Real = typename std::conditional<F32, float, double>::type;

template <int KERN>
constexpr int vdim() {
    return KERN == CSFMM_K_BIOT_SAVART ? 3 : 1;
}

template <int KERN>
constexpr double coord_scale() {
    return KERN == CSFMM_K_POISSON_LOG ? kInvSqrt2
           : (KERN == CSFMM_K_BIHARMONIC || KERN == CSFMM_K_SAL) ? 0.5
                                                                  : 1.0;
}

__device__ __forceinline__ float dev_log2(float x) { return __builtin_amdgcn_logf(x); }

// FP64 1/sqrt(x) for finite x > 0: the hardware estimate (relative error about
// 5e-8, measured) and one third-order correction y (1 + e/2 + 3e^2/8),
// e = 1 - x y^2, which leaves about 1 ulp (measured 1.1e-16).  No special
// values: x = 0 gives a NaN, which the callers' zero test masks.
__device__ __forceinline__ double rsq64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
// FP64 1/x for finite x != 0: the hardware estimate and one third-order
// correction y (1 + e + e^2), e = 1 - x y.
__device__ __forceinline__ double rcp64(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}
// FP64 natural logarithm of a positive normal x (a zero squared distance is
// masked by the callers).  With x = m 2^e, m in [sqrt(1/2), sqrt(2)) (the
// hardware's mantissa and exponent split, m doubled below sqrt(1/2)),
// f = m - 1 (exact) and s = f / (m + 1), |s| <= 0.1716:
//   ln m = 2 atanh(s) = 2 s + R,  R = 2 s^3/3 + 2 s^5/5 + ...
// and, since 2 s = f - f s,  ln m = f - s (f - R/s)  with R/s = z q(z),
// z = s^2, q the Taylor coefficients 2/3, 2/5, ..., 2/21 (the first omitted
// term is below 3e-17 of the result).  The exact f carries the leading part,
// so the rounding of s enters only the correction s f ~ f^2/2; then
// ln x = e ln 2 + ln m.  Measured on 4M values from 1e-43 to 1e43 and near 1:
// at most 1.3 ulp, about 2.6 times the throughput of the library log.
__device__ __forceinline__ double log64(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool lo = m < kInvSqrt2;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;
    const double s = f * rcp64(m + 1.0);
    const double z = s * s;
    double q = 2.0 / 21.0;
#pragma unroll
    for (int k = 9; k >= 1; --k) q = fma(q, z, 2.0 / (2 * k + 1));
    return fma(double(e), kLn2, fma(-s, f - z * q, f));
}
// FP64 ln(1 + x) for x > -1 by Kahan's correction of a logarithm (Goldberg,
// "What every computer scientist should know about floating-point
// arithmetic", Theorem 4): with u = 1 + x rounded, ln(1 + x) = ln(u) x/(u - 1)
// (u - 1 is exact), and x itself when u rounds to 1; a few ulps with log64.
__device__ __forceinline__ double log1p64(double x) {
    const double u = 1.0 + x;
    const double d = u - 1.0;
    return d == 0.0 ? x : log64(u) * (x * rcp64(d));
}
__device__ __forceinline__ float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float dev_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// dilog(1 - v) for 0 < v (clamped to 1), dilog(u) = -int_0^u ln(1-t)/t dt.
// With the substitution w = -ln(1 - z) the dilogarithm is the series
// dilog(z) = sum_k B_k w^(k+1)/(k+1)!  (Bernoulli numbers B_k; only B_1 = -1/2
// and the even ones are nonzero), whose radius is 2 pi.  Both branches keep
// w <= ln 2:
//   v <= 1/2:  dilog(1-v) = pi^2/6 - ln(v) ln(1-v) - dilog(v), w = -ln(1-v)
//              (Euler's reflection formula);
//   v >  1/2:  dilog(1-v) directly, w = -ln(v).
// The odd part is w + w^2 (-1/4 + w sum_k c_k w^(2k-2)), c_k = B_2k/(2k+1)!;
// eight terms reach FP64 rounding on w <= ln 2, three reach FP32 rounding.
__device__ constexpr double kBern[8] = {
    1.0 / 36.0,          -1.0 / 3600.0,     1.0 / 211680.0,
    -1.0 / 10886400.0,   1.0 / 526901760.0, -691.0 / 16999766784000.0,
    1.0 / 1120863744000.0, -3617.0 / 181400588328960000.0};
constexpr double kPi2Over6 = 1.64493406684822643647;

__device__ __forceinline__ double dilog_1m(double v) {
    v = fmin(v, 1.0);
    const double l1 = log64(v), l2 = log1p64(-v);
    const bool refl = v <= 0.5;
    const double w = refl ? -l2 : -l1;
    const double w2 = w * w;
    double c = kBern[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) c = fma(c, w2, kBern[k]);
    const double sr = fma(w2, fma(w, c, -0.25), w);
    return refl ? (kPi2Over6 - l1 * l2) - sr : sr;
}

__device__ __forceinline__ float dilog_1m(float v) {
    constexpr float ln2 = 0.69314718055994530942f;
    v = fminf(v, 1.f);
    const float a = dev_log2(v), b = dev_log2(1.f - v);
    const bool refl = v <= 0.5f;
    const float w = (refl ? b : a) * -ln2;
    const float w2 = w * w;
    const float c = fmaf(fmaf(float(kBern[2]), w2, float(kBern[1])), w2, float(kBern[0]));
    const float sr = fmaf(w2, fmaf(w, c, -0.25f), w);
    return refl ? fmaf(-ln2 * ln2, a * b, float(kPi2Over6)) - sr : sr;
}

// SAL closed form, eq. (G_SAL_approx), with the Love number fit of §2.4.
constexpr double kSalA1 = -2.7, kSalB0 = -6.21196, kSalB1 = 6.1;
constexpr double kSalRho = 1025.0 / 5514.0;  // seawater / mean Earth density
constexpr double kSalQ = -2.0 * (kSalA1 - kSalB1) / (1.0 - kSalB0);
constexpr double kSalScale = 3.0 * kSalRho / (4.0 * kPi) * 0.5 * (1.0 - kSalB0);

// 1/sqrt(v) + q ln(sqrt(v) + v) for v = |x-y|^2/4 > 0
__device__ __forceinline__ double sal_bracket(double v) {
    const double rs = rsq64(v);
    return fma(kSalQ, log64(fma(v, rs, v)), rs);
}
__device__ __forceinline__ float sal_bracket(float v) {
    constexpr float q2 = float(kSalQ * kLn2);  // log2 in, natural log out
    const float rs = dev_rsq(v);
    return fmaf(q2, dev_log2(fmaf(v, rs, v)), rs);
}

// Evaluation forms of one (target, source) pair:
//  FORM_CHECK  direct differences, a zero squared distance (coincident point)
//              contributes nothing; for entries whose cells overlap the target
//  FORM_NEAR   cells that do not overlap the target (no check)
//  FORM_FAR    MAC-separated entries
//  FORM_EXACT  cells that do not overlap the target, exact differences and the
//              zero check (FP32 form: the PP entries the plan marks close,
//              whose points may come near each other across leaf edges)
// In the FP32 form every kernel takes |t-s|^2 = |t|^2 + |s|^2 - 2 t.s for
// FORM_NEAR and FORM_FAR (4 operations instead of 6; coordinates are recentred
// at the target cell, and the plan's close-pair rule, or the MAC, bounds
// (|t|^2 + |s|^2)/|t-s|^2, so the relative error of the squared distance stays
// within a few hundred FP32 ulps; Biot-Savart's difference vector is then
// assembled per group in run_group); FORM_CHECK keeps exact differences so
// that a coincident point gives exactly 0.
enum { FORM_CHECK = 0, FORM_NEAR = 1, FORM_FAR = 2, FORM_EXACT = 3 };

struct TargetRegs {
    double tx, ty, tz;          // FP64 form
    double d2, dmx, dmy, dmz;   // FP64 form: |t|^2 and -2 t (FORM_FAR)
    float fx, fy, fz, f2;       // FP32 form: recentred target and |t|^2
    float mx, my, mz;           // -2 t
};

// Target registers of a target at offset (dx, dy, dz) from its cell centre.
__device__ __forceinline__ TargetRegs target_regs(double dx, double dy, double dz, double scale) {
    TargetRegs TR;
    TR.tx = dx * scale;
    TR.ty = dy * scale;
    TR.tz = dz * scale;
    TR.d2 = TR.tx * TR.tx + TR.ty * TR.ty + TR.tz * TR.tz;
    TR.dmx = -2.0 * TR.tx;
    TR.dmy = -2.0 * TR.ty;
    TR.dmz = -2.0 * TR.tz;
    TR.fx = float(TR.tx);
    TR.fy = float(TR.ty);
    TR.fz = float(TR.tz);
    TR.f2 = float(double(TR.fx) * TR.fx + double(TR.fy) * TR.fy + double(TR.fz) * TR.fz);
    TR.mx = -2.f * TR.fx;
    TR.my = -2.f * TR.fy;
    TR.mz = -2.f * TR.fz;
    return TR;
}

// FP32 expanded squared distance |t|^2 + |s|^2 - 2 t.s (FORM_NEAR, FORM_FAR).
__device__ __forceinline__ float expanded_d2(const TargetRegs& T, float sx, float sy, float sz,
                                             float s2) {
    return fmaf(T.mx, sx, fmaf(T.my, sy, fmaf(T.mz, sz, s2 + T.f2)));
}
// FP64 expanded squared distance, MAC-separated pairs only (FORM_FAR): the MAC
// bounds (|t|^2 + |s|^2)/|t-s|^2 by (1 + (1 + 2 theta/(1 - theta))^2)/2 (8.5 at
// theta 0.6, 16.6 at 0.7), so it keeps FP64 accuracy within a few ulps.
__device__ __forceinline__ double expanded_d2(const TargetRegs& T, double sx, double sy,
                                              double sz, double s2) {
    return fma(T.dmx, sx, fma(T.dmy, sy, fma(T.dmz, sz, s2 + T.d2)));
}

// Unscaled value of a scalar kernel at scaled squared distance d (FP32 form):
// log2 d (Poisson), dilog(1 - d) (biharmonic), the SAL bracket, 1/sqrt(d).
template <int KERN>
__device__ __forceinline__ float kernel_value_f32(float d) {
    if constexpr (KERN == CSFMM_K_POISSON_LOG)
        return dev_log2(d);
    else if constexpr (KERN == CSFMM_K_BIHARMONIC)
        return dilog_1m(d);
    else if constexpr (KERN == CSFMM_K_SAL)
        return sal_bracket(d);
    else
        return dev_rsq(d);
}

template <int KERN, bool F32, int FORM>
__device__ __forceinline__ void eval_pair(const TargetRegs& T, Real<F32> sx, Real<F32> sy,
                                          Real<F32> sz, Real<F32> s2, Real<F32> w,
                                          Real<F32>* p) {
    using R = Real<F32>;
    R tx, ty, tz;
    if constexpr (F32) {
        tx = T.fx; ty = T.fy; tz = T.fz;
    } else {
        tx = T.tx; ty = T.ty; tz = T.tz;
    }
    constexpr bool expanded =
        F32 && (FORM == FORM_NEAR || FORM == FORM_FAR) && KERN != CSFMM_K_BIOT_SAVART;
    constexpr bool expanded64 = !F32 && FORM == FORM_FAR && KERN != CSFMM_K_BIOT_SAVART;
    if constexpr (expanded) {
        p[0] = fmaf(w, kernel_value_f32<KERN>(expanded_d2(T, sx, sy, sz, s2)), p[0]);
    } else if constexpr (expanded64) {
        const double d = expanded_d2(T, double(sx), double(sy), double(sz), double(s2));
        double g;
        if constexpr (KERN == CSFMM_K_POISSON_LOG)
            g = log64(d);
        else if constexpr (KERN == CSFMM_K_BIHARMONIC)
            g = dilog_1m(d);
        else if constexpr (KERN == CSFMM_K_SAL)
            g = sal_bracket(d);
        else
            g = rsq64(d);
        p[0] = fma(double(w), g, p[0]);
    } else {
        (void)s2;
        const R dx = sx - tx, dy = sy - ty, dz = sz - tz;
        const R r2 = dx * dx + dy * dy + dz * dz;
        if constexpr (KERN == CSFMM_K_POISSON_LOG) {
            R lg;
            if constexpr (F32)
                lg = dev_log2(r2);
            else
                lg = log64(r2);
            if constexpr (FORM == FORM_CHECK || FORM == FORM_EXACT) lg = r2 > R(0) ? lg : R(0);
            p[0] = fma(w, lg, p[0]);
        } else if constexpr (KERN == CSFMM_K_BIOT_SAVART) {
            R inv;
            if constexpr (F32)
                inv = dev_rcp(r2);
            else
                inv = rcp64(r2);
            R f = w * inv;
            if constexpr (FORM == FORM_CHECK || FORM == FORM_EXACT) f = r2 > R(0) ? f : R(0);
            p[0] = fma(dx, f, p[0]);
            p[1] = fma(dy, f, p[1]);
            p[2] = fma(dz, f, p[2]);
        } else if constexpr (KERN == CSFMM_K_BIHARMONIC) {
            R g = dilog_1m(r2);
            if constexpr (FORM == FORM_CHECK || FORM == FORM_EXACT) g = r2 > R(0) ? g : R(0);
            p[0] = fma(w, g, p[0]);
        } else if constexpr (KERN == CSFMM_K_SAL) {
            R g = sal_bracket(r2);
            if constexpr (FORM == FORM_CHECK || FORM == FORM_EXACT) g = r2 > R(0) ? g : R(0);
            p[0] = fma(w, g, p[0]);
        } else {
            R inv;
            if constexpr (F32)
                inv = dev_rsq(r2);
            else
                inv = rsq64(r2);
            if constexpr (FORM == FORM_CHECK || FORM == FORM_EXACT) inv = r2 > R(0) ? inv : R(0);
            p[0] = fma(w, inv, p[0]);
        }
    }
}

// Final scaling of an accumulated sum at a target point (x, y, z) (FP64).
template <int KERN, bool F32>
__device__ __forceinline__ void epilogue(const double* acc, double x, double y, double z,
                                         double* out) {
    if constexpr (KERN == CSFMM_K_POISSON_LOG) {
        out[0] = (F32 ? -kLn2 / (4.0 * kPi) : -1.0 / (4.0 * kPi)) * acc[0];
    } else if constexpr (KERN == CSFMM_K_BIOT_SAVART) {
        const double c = -1.0 / (2.0 * kPi);
        out[0] = c * (y * acc[2] - z * acc[1]);
        out[1] = c * (z * acc[0] - x * acc[2]);
        out[2] = c * (x * acc[1] - y * acc[0]);
    } else if constexpr (KERN == CSFMM_K_BIHARMONIC) {
        out[0] = acc[0] / (4.0 * kPi);
    } else if constexpr (KERN == CSFMM_K_SAL) {
        out[0] = kSalScale * acc[0];
    } else {
        out[0] = acc[0];
    }
}

struct TileArgs {
    const int32_t* tcells;
    const int32_t *tbegin, *tcount;
    const double* tcenter;
    const double *tx, *ty, *tz;  // target particles (near kernel)
    const double* tprox;         // target proxies [cell][3][KS] (far kernel)
    const int32_t *off_a, *src_a;  // list with particle sources (PP or CP)
    const int32_t *off_b, *src_b;  // list with proxy sources (PC or CC)
    const int32_t* novl;           // leading overlapping entries of list a (PP), or NULL
    const int32_t* ncl;            // close entries of list a after them (PP), or NULL
    const int32_t *sbegin, *scount;
    const double *sx, *sy, *sz, *sw;
    const double *sprox, *swbar;
    int K, KS;
    bool use_a, use_b;  // which of the two lists this launch takes
    double* out;
    int64_t comp_stride;
};

// The near kernel (TPROX = false) takes target particles of leaves with the PP
// list (mode kTileNearPP, into phinear) or the PC list (mode kTilePCFar, into
// phipc); the far kernel (TPROX = true) takes target proxies with CP and CC.
template <bool TPROX>
__device__ __forceinline__ TileArgs tile_args(const ReqView& V, int mode) {
    TileArgs a;
    a.tcells = TPROX ? V.far_targets : V.t_leaves;
    a.tbegin = V.t_begin;
    a.tcount = V.t_count;
    a.tcenter = V.t_center;
    a.tx = V.t_x;
    a.ty = V.t_y;
    a.tz = V.t_z;
    a.tprox = V.t_prox;
    a.off_a = V.off[TPROX ? kCP : kPP];
    a.src_a = V.src[TPROX ? kCP : kPP];
    a.off_b = V.off[TPROX ? kCC : kPC];
    a.src_b = V.src[TPROX ? kCC : kPC];
    a.novl = TPROX ? nullptr : V.novl;
    a.ncl = TPROX ? nullptr : V.ncl;
    a.sbegin = V.s_begin;
    a.scount = V.s_count;
    a.sx = V.s_x;
    a.sy = V.s_y;
    a.sz = V.s_z;
    a.sw = V.ws;
    a.sprox = V.s_prox;
    a.swbar = V.wbar;
    a.K = V.K;
    a.KS = V.KS;
    a.use_a = TPROX || mode == kTileNearPP;
    a.use_b = TPROX || mode == kTilePCFar;
    a.out = TPROX ? V.psi : (mode == kTileNearPP ? V.phinear : V.phipc);
    a.comp_stride = TPROX ? V.psi_stride : V.nt;
    return a;
}

constexpr int kMaxG = 32;   // source groups per target
constexpr int kUnroll = 4;  // one staged group of four sources per unrolled step
static_assert(kUnroll == 4, "Stage<true> packs sources in groups of four");
// Sources staged per step of the tile kernel.  The staging buffer (20 bytes a
// source in the FP32 form, 40 in FP64) and the block's other LDS arrays fit
// six blocks of four waves in a CU's 160 KB in the FP32 form and four in FP64,
// the occupancies the instances run at.
template <bool F32>
constexpr int tile_chunk() {
    return F32 ? 1024 : 768;
}
template <bool F32>
constexpr int lds_sources() {
    return tile_chunk<F32>() + kUnroll * kMaxG;
}

// Staged sources, recentred at the target cell, for CAP sources: groups of
// four sources, (x, y, z, |s|^2) each and then the four weights, so that one
// LDS address serves a whole unrolled step (FP32 or FP64 values).
template <bool F32, int CAP>
struct StageT;
template <int CAP>
struct StageT<true, CAP> {
    static_assert(CAP % 4 == 0, "groups of four");
    struct Quad {
        float4 p[4];
        float4 w;
    };
    Quad b[CAP / 4];
    __device__ __forceinline__ void put(int q, double x, double y, double z, double w) {
        const float fx = float(x), fy = float(y), fz = float(z);
        const float f2 = float(double(fx) * fx + double(fy) * fy + double(fz) * fz);
        b[q >> 2].p[q & 3] = make_float4(fx, fy, fz, f2);
        reinterpret_cast<float*>(&b[q >> 2].w)[q & 3] = float(w);
    }
};
template <int CAP>
struct StageT<false, CAP> {
    static_assert(CAP % 4 == 0, "groups of four");
    struct Quad {
        double4 p[4];
        double4 w;
    };
    Quad b[CAP / 4];
    __device__ __forceinline__ void put(int q, double x, double y, double z, double w) {
        b[q >> 2].p[q & 3] = make_double4(x, y, z, x * x + y * y + z * z);
        reinterpret_cast<double*>(&b[q >> 2].w)[q & 3] = w;
    }
};
template <bool F32>
using Stage = StageT<F32, lds_sources<F32>()>;

// One-wave-per-leaf path: each wave stages up to wave_items items of at most
// 64 sources at a time (padded to a multiple of four): four in the FP32
// form, three in FP64 (whose stage holds twice the bytes per source).
template <bool F32>
constexpr int wave_items() {
    return F32 ? 4 : 3;
}
template <bool F32>
using WaveStage = StageT<F32, 64 * wave_items<F32>() + kUnroll>;

// Sources per group when nq staged sources are split over G groups, a multiple
// of the unroll (the tail is padded with weightless sources).
__device__ __forceinline__ int group_len(int nq, int G) {
    return (((nq + G - 1) / G) + kUnroll - 1) / kUnroll * kUnroll;
}

// Sources base .. base + nj of a stage against TPT targets of one thread
// (each staged source read once serves all of them).
//
// Biot-Savart in the FP32 form, FORM_NEAR and FORM_FAR: with f = w / |t-s|^2
// from the expanded squared distance, the sum of f (s - t) is taken as
// A - t B, A = sum f s, B = sum f (nine operations a pair instead of eleven);
// coordinates are recentred at the target cell, so |s| and |t| stay within a
// few times |s - t| on the pairs these forms see (the close-pair rule and the
// MAC bound the ratio), and the cancellation in A - t B costs a few ulps.
template <int KERN, bool F32, int FORM, int CAP, int TPT>
__device__ __forceinline__ void run_group(const StageT<F32, CAP>& L, int base, int nj,
                                          const TargetRegs (&T)[TPT],
                                          Real<F32> (&p)[TPT][vdim<KERN>()]) {
    // nj is the same for every thread of the block: a scalar trip count keeps
    // the loop control off the vector unit
    nj = __builtin_amdgcn_readfirstlane(nj);
    const typename StageT<F32, CAP>::Quad* Qp = &L.b[base >> 2];  // base: a multiple of four
    if constexpr (F32 && KERN == CSFMM_K_BIOT_SAVART && (FORM == FORM_NEAR || FORM == FORM_FAR)) {
        float A[TPT][3], B[TPT];
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            A[q][0] = A[q][1] = A[q][2] = 0.f;
            B[q] = 0.f;
        }
        for (int j = 0; j < nj; j += kUnroll) {
            const auto& Q = *Qp++;
            const float4 w4 = Q.w;
            const float ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const float4 s = Q.p[u];
#pragma unroll
                for (int q = 0; q < TPT; ++q) {
                    const float f = ws[u] * dev_rcp(expanded_d2(T[q], s.x, s.y, s.z, s.w));
                    A[q][0] = fmaf(f, s.x, A[q][0]);
                    A[q][1] = fmaf(f, s.y, A[q][1]);
                    A[q][2] = fmaf(f, s.z, A[q][2]);
                    B[q] += f;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            p[q][0] += fmaf(-T[q].fx, B[q], A[q][0]);
            p[q][1] += fmaf(-T[q].fy, B[q], A[q][1]);
            p[q][2] += fmaf(-T[q].fz, B[q], A[q][2]);
        }
        return;
    }
    for (int j = 0; j < nj; j += kUnroll) {
        const auto& Q = *Qp++;
        const auto w4 = Q.w;
        const Real<F32> ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const auto s = Q.p[u];
#pragma unroll
            for (int q = 0; q < TPT; ++q)
                eval_pair<KERN, F32, FORM>(T[q], s.x, s.y, s.z, s.w, ws[u], p[q]);
        }
    }
}
template <int KERN, bool F32, int FORM, int CAP>
__device__ __forceinline__ void run_group(const StageT<F32, CAP>& L, int base, int nj,
                                          const TargetRegs& T, Real<F32>* p) {
    const TargetRegs T1[1] = {T};
    Real<F32> p1[1][vdim<KERN>()];
#pragma unroll
    for (int v = 0; v < vdim<KERN>(); ++v) p1[0][v] = p[v];
    run_group<KERN, F32, FORM, CAP, 1>(L, base, nj, T1, p1);
#pragma unroll
    for (int v = 0; v < vdim<KERN>(); ++v) p[v] = p1[0][v];
}

// Element i of a global array read through the global address space (a load
// with a wave-uniform address then gives a wave-uniform value).
template <class T>
__device__ __forceinline__ T gload(const T* base, int64_t i) {
    return ((const __attribute__((address_space(1))) T*)base)[i];
}
// A request view read word by word through the global address space, so that
// its fields are wave-uniform values.
__device__ __forceinline__ ReqView load_view(const ReqView* p) {
    static_assert(sizeof(ReqView) % 8 == 0, "whole words");
    ReqView v;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(p);
    uint64_t* dst = reinterpret_cast<uint64_t*>(&v);
#pragma unroll
    for (int i = 0; i < int(sizeof(ReqView) / 8); ++i) dst[i] = gload(src, i);
    return v;
}
// The same for a wave-uniform base and a per-lane index i with i * sizeof(T)
// below 2^32: a 32-bit byte offset on a scalar base address.
template <class T>
__device__ __forceinline__ T gload_near(const T* base, unsigned i) {
    const unsigned byte = i * unsigned(sizeof(T));
    return *(const __attribute__((address_space(1))) T*)(
        (const __attribute__((address_space(1))) char*)base + byte);
}

// Point o of a list entry (stage_source: recentred and scaled, into stage slot
// q).  code >= 0: the entry is the particles of a leaf starting at sorted
// position code; code < 0: the KS-strided proxies of cell -(code + 1) with
// their weights.  o is below the entry's size (a leaf's points or K proxies).
__device__ __forceinline__ void load_source(const TileArgs& a, int code, int o, double& yx,
                                            double& yy, double& yz, double& w) {
    if (code >= 0) {
        yx = gload_near(a.sx + code, o);
        yy = gload_near(a.sy + code, o);
        yz = gload_near(a.sz + code, o);
        w = gload_near(a.sw + code, o);
    } else {
        const int64_t sc = -(code + 1);
        const double* ps = a.sprox + sc * 3 * a.KS;
        yx = gload_near(ps, o);
        yy = gload_near(ps + a.KS, o);
        yz = gload_near(ps + 2 * a.KS, o);
        w = gload_near(a.swbar + sc * a.KS, o);
    }
}
template <class St>
__device__ __forceinline__ void stage_source(const TileArgs& a, int code, int o, double cx,
                                             double cy, double cz, double scale, St& L, int q) {
    double yx, yy, yz, w;
    load_source(a, code, o, yx, yy, yz, w);
    L.put(q, (yx - cx) * scale, (yy - cy) * scale, (yz - cz) * scale, w);
}

template <int KERN, bool F32>
struct TileSmem {
    Stage<F32> L[1];
    int e_code[kMaxEntries];
    int e_pref[kMaxEntries + 1];
    int lw[4];
    // the per-target reduction over source groups reuses the staging buffer
    static_assert(sizeof(Stage<F32>) >= sizeof(double) * 2 * vdim<KERN>() * kThreads, "red");
    __device__ __forceinline__ double (*red())[kThreads] {
        return reinterpret_cast<double (*)[kThreads]>(&L[0]);
    }
};

// One target cell of one request: near field (TPROX = false) or far field.
// The forms a launch can meet (kFormsAll, or kFormsPP: PP launches, no
// MAC-separated form; kFormsFar: PC + far launches, that form only), so that
// an instance holds no target registers for forms it never takes.
enum { kFormsAll = 0, kFormsPP = 1, kFormsFar = 2 };
template <int KERN, bool F32, bool TPROX, int FORMS = kFormsAll>
__device__ __forceinline__ void tile_body(const ReqView& V, int mode, int local,
                                          TileSmem<KERN, F32>& sm) {
    using R = Real<F32>;
    constexpr int VD = vdim<KERN>();
    constexpr double scale = coord_scale<KERN>();
    Stage<F32>* L = sm.L;
    int* e_code = sm.e_code;
    int* e_pref = sm.e_pref;
    int* lw = sm.lw;
    auto red = sm.red();
    const TileArgs a = tile_args<TPROX>(V, mode);
    const int T = a.tcells[local];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const double cx = a.tcenter[3 * T], cy = a.tcenter[3 * T + 1], cz = a.tcenter[3 * T + 2];
    const int KS = a.KS;
    const int nT = TPROX ? a.K : a.tcount[T];
    const int tb = TPROX ? 0 : a.tbegin[T];
    const int ea0 = a.off_a[T], nea = a.use_a ? a.off_a[T + 1] - ea0 : 0;
    const int eb0 = a.off_b[T], neb = a.use_b ? a.off_b[T + 1] - eb0 : 0;
    const int nov = (a.use_a && a.novl) ? a.novl[T] : 0;
    const int ncl = (a.use_a && a.ncl) ? a.ncl[T] : 0;
    // entry ranges of the four forms: [0,nov) check, [nov,nov+ncl) exact,
    // [nov+ncl,nea) near, [nea,nea+neb) far; sources of the far kernel are all
    // MAC separated
    const int ph_hi[4] = {TPROX ? 0 : nov, TPROX ? 0 : nov + ncl, TPROX ? 0 : nea, nea + neb};
    const int ne_all = nea + neb;

    // each thread takes two targets (t and t + TC), so that a block's threads
    // split a leaf of any size evenly over source groups and each staged
    // source read serves two evaluations (in the FP32 form too: the
    // 1/|x-y| workload's FP32 form 4.20 -> 3.89 ms, although the FP32
    // instances then spill more at 80 VGPRs)
    constexpr int TPT = 2;
    for (int t0 = 0; t0 < nT; t0 += TPT * kThreads) {
        const int TC = min((nT - t0 + TPT - 1) / TPT, kThreads);
        const int G = min(kThreads / TC, kMaxG);
        const int t = tid % TC, g = tid / TC;
        const bool active = g < G;
        constexpr int kTileChunk = tile_chunk<F32>();
        const int Tj_full = group_len(kTileChunk, G);
        double gx[TPT], gy[TPT], gz[TPT];
        TargetRegs TR[TPT];
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const int it = t0 + t + q * TC;  // this thread's q-th target
            gx[q] = cx;
            gy[q] = cy;
            gz[q] = cz;
            if (active && it < nT) {
                if constexpr (TPROX) {
                    const double* pc = a.tprox + int64_t(T) * 3 * KS;
                    gx[q] = pc[it];
                    gy[q] = pc[KS + it];
                    gz[q] = pc[2 * KS + it];
                } else {
                    gx[q] = a.tx[tb + it];
                    gy[q] = a.ty[tb + it];
                    gz[q] = a.tz[tb + it];
                }
            }
            TR[q] = target_regs(gx[q] - cx, gy[q] - cy, gz[q] - cz, scale);
        }
        double acc[TPT][VD];
#pragma unroll
        for (int q = 0; q < TPT; ++q)
#pragma unroll
            for (int v = 0; v < VD; ++v) acc[q][v] = 0.0;

        // Entries are processed in batches of up to kMaxEntries; inside a batch
        // the flattened sources split into the three forms (check, near, far)
        // and each form into chunks of at most kTileChunk staged through LDS.
        for (int ebase = 0; ebase < ne_all; ebase += kMaxEntries) {
            const int ne = min(kMaxEntries, ne_all - ebase);
            int sz = 0;
            if (tid < ne) {
                const int e = ebase + tid;
                if (e < nea) {
                    const int s = a.src_a[ea0 + e];
                    e_code[tid] = a.sbegin[s];
                    sz = a.scount[s];
                } else {
                    const int s = a.src_b[eb0 + e - nea];
                    e_code[tid] = -(s + 1);
                    sz = a.K;
                }
            }
            const int incl = block_scan_incl_256(sz, lw);
            e_pref[tid] = incl - sz;
            if (tid == kThreads - 1) e_pref[kMaxEntries] = incl;
            __syncthreads();
            // source offsets where the forms change inside this batch
            int bnd[5];
            bnd[0] = 0;
            bnd[4] = e_pref[kMaxEntries];
#pragma unroll
            for (int q = 1; q < 4; ++q) bnd[q] = e_pref[min(max(ph_hi[q - 1] - ebase, 0), kMaxEntries)];
            for (int ph = FORMS == kFormsFar ? 3 : 0; ph < (FORMS == kFormsPP ? 3 : 4); ++ph) {
                for (int q0 = bnd[ph]; q0 < bnd[ph + 1]; q0 += kTileChunk) {
                    const int nq = min(kTileChunk, bnd[ph + 1] - q0);
                    const int Tj = nq == kTileChunk ? Tj_full : group_len(nq, G);
                    const int npad = G * Tj;
                    Stage<F32>& Lb = L[0];
                    // padding after the chunk: far away and weightless
                    for (int q = nq + tid; q < npad; q += kThreads) Lb.put(q, 2.0, 2.0, 2.0, 0.0);
                    // each wave stages whole entries (a leaf's contiguous particles or
                    // a cell's proxies) that overlap [q0, q0 + nq), its lanes one point
                    // each: no per-point search for the owning entry
                    const int qe = q0 + nq;
                    int e = 0;
                    {
                        int hi = ne - 1;
                        while (e < hi) {
                            const int mid = (e + hi + 1) >> 1;
                            if (e_pref[mid] <= q0)
                                e = mid;
                            else
                                hi = mid - 1;
                        }
                    }
                    e = __builtin_amdgcn_readfirstlane(e) + wave;
                    for (; e < ne; e += kThreads / 64) {
                        const int pb = __builtin_amdgcn_readfirstlane(e_pref[e]);
                        if (pb >= qe) break;
                        const int pe = min(__builtin_amdgcn_readfirstlane(e_pref[e + 1]), qe);
                        const int code = __builtin_amdgcn_readfirstlane(e_code[e]);
                        for (int q = max(pb, q0) + lane; q < pe; q += 64)
                            stage_source(a, code, q - pb, cx, cy, cz, scale, Lb, q - q0);
                    }
                    __syncthreads();
                    if (active) {
                        R p[TPT][VD];
#pragma unroll
                        for (int q = 0; q < TPT; ++q)
#pragma unroll
                            for (int v = 0; v < VD; ++v) p[q][v] = R(0);
                        constexpr int CAP = lds_sources<F32>();
                        if constexpr (FORMS != kFormsFar) {
                            if (ph == 0)
                                run_group<KERN, F32, FORM_CHECK, CAP, TPT>(Lb, g * Tj, Tj, TR, p);
                            else if (ph == 1)
                                run_group<KERN, F32, FORM_EXACT, CAP, TPT>(Lb, g * Tj, Tj, TR, p);
                            else if (ph == 2)
                                run_group<KERN, F32, FORM_NEAR, CAP, TPT>(Lb, g * Tj, Tj, TR, p);
                        }
                        if constexpr (FORMS != kFormsPP)
                            if (ph == 3)
                                run_group<KERN, F32, FORM_FAR, CAP, TPT>(Lb, g * Tj, Tj, TR, p);
#pragma unroll
                        for (int q = 0; q < TPT; ++q)
#pragma unroll
                            for (int v = 0; v < VD; ++v) acc[q][v] += double(p[q][v]);
                    }
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int q = 0; q < TPT; ++q)
#pragma unroll
            for (int v = 0; v < VD; ++v) red[q * VD + v][tid] = active ? acc[q][v] : 0.0;
        __syncthreads();
        if (tid < TC) {
#pragma unroll
            for (int q = 0; q < TPT; ++q) {
                const int it = t0 + tid + q * TC;
                if (it >= nT) continue;
                double r[VD], o[VD];
#pragma unroll
                for (int v = 0; v < VD; ++v) {
                    r[v] = 0.0;
                    for (int gg = 0; gg < G; ++gg) r[v] += red[q * VD + v][gg * TC + tid];
                }
                epilogue<KERN, F32>(r, gx[q], gy[q], gz[q], o);
                const int64_t base = TPROX ? int64_t(T) * KS + it : int64_t(tb) + it;
#pragma unroll
                for (int v = 0; v < VD; ++v) a.out[v * a.comp_stride + base] = o[v];
            }
        }
        __syncthreads();
    }
}

// One wave's LDS on the symmetric PP path: one partner leaf staged (up to 64
// sources) and a tile of column terms, 64 rows (target lanes) by sym_cols
// columns (sources): 16 FP32 or 8 FP64 columns, 4 KB either way.  It overlays
// the wave's stage of the other phases.
template <bool F32>
constexpr int sym_cols() {
    return F32 ? 16 : 8;
}
// tile column stride in values: the rows plus a pad that keeps the 16-byte
// reads of one column's lanes on distinct banks
template <bool F32>
constexpr int sym_stride() {
    return kWaveLeaf + (F32 ? 4 : 2);
}
template <bool F32>
struct SymLds {
    StageT<F32, kWaveLeaf> st;
    Real<F32> m[sym_cols<F32>() * sym_stride<F32>()];  // column c, row i: m[stride c + i]
};
template <bool F32>
constexpr int wave_lds_bytes() {
    return sizeof(SymLds<F32>) > sizeof(WaveStage<F32>) ? int(sizeof(SymLds<F32>))
                                                         : int(sizeof(WaveStage<F32>));
}

// x of another lane of the same row of 16 lanes (DPP control CTRL: a
// quad_perm, or row_half_mirror 0x141, lane i <- lane 7 - i of its eight)
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                 CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_row(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xf, 0xf,
                                                             true));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xf,
                                                             0xf, true));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Kernel value of a symmetric PP pair (scalar kernels, cells that do not
// overlap): the FP32 form takes the expanded squared distance (the close
// entries stay one way), FP64 exact differences; unscaled as in eval_pair.
template <int KERN, bool F32>
__device__ __forceinline__ Real<F32> sym_value(const TargetRegs& T, Real<F32> sx, Real<F32> sy,
                                               Real<F32> sz, Real<F32> s2) {
    if constexpr (F32) {
        return kernel_value_f32<KERN>(expanded_d2(T, sx, sy, sz, s2));
    } else {
        (void)s2;
        const double dx = sx - T.tx, dy = sy - T.ty, dz = sz - T.tz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if constexpr (KERN == CSFMM_K_POISSON_LOG)
            return log64(r2);
        else if constexpr (KERN == CSFMM_K_BIHARMONIC)
            return dilog_1m(r2);
        else if constexpr (KERN == CSFMM_K_SAL)
            return sal_bracket(r2);
        else
            return rsq64(r2);
    }
}

__device__ __forceinline__ void wave_sync();

// One symmetric PP pair on the wave of its owner A: for every staged source j
// of the partner B (nj, a multiple of the tile's C columns, padded with
// weightless sources) the kernel value g_ij at every lane's target i of A
// serves both directions: the row sum p_i += w_j g_ij and the column sum
// col_j = sum_i wA_i g_ij.  The column terms of C sources go through the LDS
// tile (column-major): lane i writes its term of each column as it is
// computed, then the 64/C lanes of a column each sum C consecutive rows of
// it (lane l: column l / (64/C), rows C (l % (64/C)) ..) and a DPP tree joins
// their partial sums (quads; in FP64 then the two quads of eight lanes), in
// an order that does not depend on scheduling; col_j goes to colout[j] for
// j < nB.
template <int KERN, bool F32>
__device__ __forceinline__ void run_sym(SymLds<F32>& S, int base, int nj, int nB,
                                        const TargetRegs& T, Real<F32> wA, Real<F32>* p,
                                        Real<F32>* __restrict__ colout) {
    using R = Real<F32>;
    using R4 = typename std::conditional<F32, float4, double4>::type;
    constexpr int C = sym_cols<F32>(), LPC = 64 / C, SD = sym_stride<F32>();
    const int lane = threadIdx.x & 63;
    nj = __builtin_amdgcn_readfirstlane(nj);
    for (int j0 = 0; j0 < nj; j0 += C) {
        // the next group of four sources is read while the current one is
        // evaluated
        const auto* Qp = &S.st.b[(base + j0) >> 2];
        R4 cur[5], nxt[5];
#pragma unroll
        for (int k = 0; k < 4; ++k) cur[k] = Qp[0].p[k];
        cur[4] = Qp[0].w;
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            if (q + 1 < C / 4) {
#pragma unroll
                for (int k = 0; k < 4; ++k) nxt[k] = Qp[q + 1].p[k];
                nxt[4] = Qp[q + 1].w;
            }
            const R ws[4] = {cur[4].x, cur[4].y, cur[4].z, cur[4].w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const R4 sp = cur[u];
                const R g = sym_value<KERN, F32>(T, sp.x, sp.y, sp.z, sp.w);
                p[0] = fma(ws[u], g, p[0]);
                // column term, stored at once (no registers held for the tile)
                S.m[SD * (4 * q + u) + lane] = wA * g;
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) cur[k] = nxt[k];
        }
        wave_sync();
        const int col = lane / LPC, r0 = lane % LPC;
        R sum;
        if constexpr (F32) {
            const float4* cp = reinterpret_cast<const float4*>(&S.m[SD * col + C * r0]);
            float4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = cp[k];
            float part[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) part[k] = (v[k].x + v[k].y) + (v[k].z + v[k].w);
            sum = (part[0] + part[1]) + (part[2] + part[3]);
        } else {
            const double2* cp = reinterpret_cast<const double2*>(&S.m[SD * col + C * r0]);
            double2 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = cp[k];
            sum = ((v[0].x + v[0].y) + (v[1].x + v[1].y)) + ((v[2].x + v[2].y) + (v[3].x + v[3].y));
        }
        sum += dpp_row<0xB1>(sum);  // quad_perm [1,0,3,2]
        sum += dpp_row<0x4E>(sum);  // quad_perm [2,3,0,1]
        if constexpr (!F32) sum += dpp_row<0x141>(sum);  // row_half_mirror: the other quad
        if (r0 == 0 && j0 + col < nB) colout[j0 + col] = sum;
        wave_sync();
    }
}

// Orders a wave's LDS stores before its later loads (and the reverse) across
// lanes; the stage of the one-wave-per-leaf path belongs to one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The symmetric pairs owned by target leaf T (one wave, lane = target of T),
// one partner leaf (at most 64 points) at a time, padded to a multiple of the
// tile's columns; the loads of the next partner are in flight while the
// current one is evaluated.  Row sums into acc, column sums to the pair's
// slot of sym_col.
template <int KERN, bool F32>
__device__ __forceinline__ void sym_pairs(const TileArgs& a, const ReqView& V, int T, int tb,
                                          int nT, double cx, double cy, double cz,
                                          const TargetRegs& TR, double* acc, SymLds<F32>& S) {
    using R = Real<F32>;
    constexpr int C = sym_cols<F32>();
    constexpr double scale = coord_scale<KERN>();
    const int lane = threadIdx.x & 63;
    R* __restrict__ cols = static_cast<R*>(V.sym_col);
    // T's points as sources of the column direction (same set: same order)
    const R wA = lane < nT ? R(gload_near(a.sw + tb, lane)) : R(0);
    const int o0 = gload(V.own_off, T), o1 = gload(V.own_off, T + 1);
    int cnt = 0;
    double yx = 0.0, yy = 0.0, yz = 0.0, yw = 0.0;
    auto fetch = [&](int k) {
        const int c = gload(V.own_src, k);
        const int code = gload(a.sbegin, c);
        cnt = gload(a.scount, c);
        if (cnt > 0) load_source(a, code, min(lane, cnt - 1), yx, yy, yz, yw);
    };
    if (o0 < o1) fetch(o0);
    R p = R(0);
    for (int k = o0; k < o1; ++k) {
        const int n = cnt, npad = (n + C - 1) / C * C;
        if (lane < n)
            S.st.put(lane, (yx - cx) * scale, (yy - cy) * scale, (yz - cz) * scale, yw);
        else if (lane < npad)
            S.st.put(lane, 2.0, 2.0, 2.0, 0.0);  // far, weightless
        wave_sync();
        if (k + 1 < o1) fetch(k + 1);
        if (n > 0) run_sym<KERN, F32>(S, 0, npad, n, TR, wA, &p, cols + int64_t(k) * kWaveLeaf);
        wave_sync();
    }
    acc[0] += double(p);
}

// Near field of one target leaf of at most 64 particles on one wave: lane t
// holds target t and sums over every source, so no cross-wave reduction and no
// block barrier.  The entries are taken in list order, split into the same
// three forms as tile_body (overlapping PP entries, the other PP entries, PC
// entries), and staged up to wave_items x 64 sources at a time.
template <int KERN, bool F32, int FORMS = kFormsAll>
__device__ __forceinline__ void tile_leaf_wave(const ReqView& V, int mode, int leaf, bool sym,
                                               char* lds) {
    WaveStage<F32>& L = *reinterpret_cast<WaveStage<F32>*>(lds);
    using R = Real<F32>;
    constexpr int VD = vdim<KERN>();
    constexpr double scale = coord_scale<KERN>();
    const TileArgs a = tile_args<false>(V, mode);
    const int lane = threadIdx.x & 63;
    // global loads of wave-uniform indices: uniform values (scalar registers)
    const int T = gload(a.tcells, leaf);
    const int nT = gload(a.tcount, T), tb = gload(a.tbegin, T);
    const double cx = gload(a.tcenter, 3 * T), cy = gload(a.tcenter, 3 * T + 1),
                 cz = gload(a.tcenter, 3 * T + 2);
    const bool active = lane < nT;
    const double gx = active ? gload_near(a.tx + tb, lane) : cx;
    const double gy = active ? gload_near(a.ty + tb, lane) : cy;
    const double gz = active ? gload_near(a.tz + tb, lane) : cz;
    const TargetRegs TR = target_regs(gx - cx, gy - cy, gz - cz, scale);
    double acc[VD];
#pragma unroll
    for (int v = 0; v < VD; ++v) acc[v] = 0.0;
    const int ea0 = a.use_a ? gload(a.off_a, T) : 0;
    const int nea = a.use_a ? gload(a.off_a, T + 1) - ea0 : 0;
    const int eb0 = a.use_b ? gload(a.off_b, T) : 0;
    const int neb = a.use_b ? gload(a.off_b, T + 1) - eb0 : 0;
    const int nov = (a.use_a && a.novl) ? gload(a.novl, T) : 0;
    const int ncl = (a.use_a && a.ncl) ? gload(a.ncl, T) : 0;
    // symmetric PP path (scalar kernels, PP launch): the distinct leaves'
    // entries split into one-way entries (here, phases 1 and 2; in the FP32
    // form the close ones lead the one-way list) and owned pairs (sym_pairs
    // below); pairs owned by the partner come in through k_sym_merge
    constexpr bool kSymKernel = KERN != CSFMM_K_BIOT_SAVART;
    sym = kSymKernel && sym && a.use_a;
    const int32_t* list1 = sym ? V.one_src : a.src_a + ea0;
    const int base1 = sym ? gload(V.one_off, T) : nov;
    const int end1 = sym ? gload(V.one_off, T + 1) : nea;
    // phases: 0 overlapping entries (check), 1 close entries (exact
    // differences), 2 the other PP entries, 3 PC entries (far form)
    for (int ph = FORMS == kFormsFar ? 3 : 0; ph < (FORMS == kFormsPP ? 3 : 4); ++ph) {
        const int e_beg = ph == 1 ? base1 : ph == 2 ? base1 + ncl : 0;
        const int e_end = ph == 0 ? nov : ph == 1 ? base1 + ncl : ph == 2 ? end1 : neb;
        // entry cache: lane l holds the code and size of entry cb + l
        int cb = e_beg - 64, c_code = 0, c_size = 0;
        int e = e_beg, off = 0;  // next entry and its sources already staged
        while (e < e_end) {
            // Up to kItems items of at most 64 sources (the rest of an entry or
            // its next 64) per step: every lane issues the loads of its point of
            // all items before the first store, one memory latency per step.
            constexpr int kItems = wave_items<F32>();
            int it_code[kItems], it_off[kItems], it_cnt[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                it_code[k] = 0;
                it_off[k] = 0;
                it_cnt[k] = 0;
                if (e < e_end) {
                    if (e >= cb + 64) {
                        cb = e;
                        const int ee = cb + lane;
                        c_code = 0;
                        c_size = 0;
                        if (ee < e_end) {
                            if (ph < 3) {
                                const int sc = ph == 0 ? gload(a.src_a, ea0 + ee)
                                                       : gload(list1, ee);
                                c_code = gload(a.sbegin, sc);
                                c_size = gload(a.scount, sc);
                            } else {
                                c_code = -(gload(a.src_b, eb0 + ee) + 1);
                                c_size = a.K;
                            }
                        }
                    }
                    const int size = __builtin_amdgcn_readlane(c_size, e - cb);
                    it_code[k] = __builtin_amdgcn_readlane(c_code, e - cb);
                    it_off[k] = off;
                    it_cnt[k] = min(size - off, 64);
                    off += it_cnt[k];
                    if (off == size) {
                        ++e;
                        off = 0;
                    }
                }
            }
            // every lane loads (lanes past an item's end repeat its last point), so
            // the loads need no per-lane branches
            double yx[kItems], yy[kItems], yz[kItems], yw[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k)
                if (it_cnt[k] > 0)
                    load_source(a, it_code[k], it_off[k] + min(lane, it_cnt[k] - 1), yx[k],
                                yy[k], yz[k], yw[k]);
            int n = 0;
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                if (lane < it_cnt[k])
                    L.put(n + lane, (yx[k] - cx) * scale, (yy[k] - cy) * scale,
                          (yz[k] - cz) * scale, yw[k]);
                n += it_cnt[k];
            }
            const int npad = (n + kUnroll - 1) / kUnroll * kUnroll;
            if (lane < npad - n) L.put(n + lane, 2.0, 2.0, 2.0, 0.0);  // far, weightless
            wave_sync();
            R p[VD];
#pragma unroll
            for (int v = 0; v < VD; ++v) p[v] = R(0);
            if constexpr (FORMS != kFormsFar) {
                if (ph == 0)
                    run_group<KERN, F32, FORM_CHECK>(L, 0, npad, TR, p);
                else if (ph == 1)
                    run_group<KERN, F32, FORM_EXACT>(L, 0, npad, TR, p);
                else if (ph == 2)
                    run_group<KERN, F32, FORM_NEAR>(L, 0, npad, TR, p);
            }
            if constexpr (FORMS != kFormsPP)
                if (ph == 3) run_group<KERN, F32, FORM_FAR>(L, 0, npad, TR, p);
#pragma unroll
            for (int v = 0; v < VD; ++v) acc[v] += double(p[v]);
            wave_sync();
        }
    }
    if constexpr (kSymKernel && FORMS != kFormsFar) {
        if (sym)
            sym_pairs<KERN, F32>(a, V, T, tb, nT, cx, cy, cz, TR, acc,
                                 *reinterpret_cast<SymLds<F32>*>(lds));
    }
    if (active) {
        double o[VD];
        epilogue<KERN, F32>(acc, gx, gy, gz, o);
#pragma unroll
        for (int v = 0; v < VD; ++v) a.out[v * a.comp_stride + tb + lane] = o[v];
    }
}

// Far-field and near-field blocks in one grid: prefix2 locates far-field work
// (none in a kTileNearPP launch), prefix near-field work.  Every XCD runs its
// share of far-field blocks first and then its share of near-field blocks; in
// a kTilePCFar launch the far-field blocks are the long ones and the short PC
// blocks fill the tail.  Near-field blocks of a request marked in leaf_wave
// take four target leaves, one per wave (tile_leaf_wave); the others take one
// leaf over the whole block (tile_body).  The occupancy hint keeps the scalar
// FP32 instances at 80 VGPRs (6 waves per SIMD; measured faster than 5),
// Biot-Savart's FP32 instances (three components and the A - t B sums) at 96
// (5 waves, which removes their spills; measured 1% faster than 6 on N =
// 1,572,864); the FP64 instances, whose transcendentals are longer and which
// hold two targets a thread, get 3 waves per SIMD, but 1/|x-y| 4 (1.5% faster
// on 6,291,456 sources x 1,000,000 targets, p = 10: 8.74 -> 8.61 ms, then with
// 12 VGPRs spilled outside the inner loops).
// PPONLY: the instance for PP launches (no far-field blocks, no
// MAC-separated form); else the one for PC + far launches (that form only).
// Each then holds only its forms' target registers: the 1/|x-y| FP64
// instances fit 4 waves without spills (117 and 123 VGPRs; the PP launch of
// that workload 7.15 -> 6.24 ms, results bitwise unchanged), FP64 Poisson's
// PP instance 4 waves instead of 3.
template <int KERN, bool F32, bool PPONLY>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(F32 ? (KERN == CSFMM_K_BIOT_SAVART ? 5 : 6) : (KERN == CSFMM_K_INV_DIST ? 4 : 3)))) void k_tile(Batch b) {
    __shared__ TileSmem<KERN, F32> sm;
    bool far;
    const int blk = xcd_split_block(blockIdx.x, gridDim.x, b.prefix2[b.n], far);
    int req, local;
    if (PPONLY) far = false;  // a PP launch has no far-field blocks
    if (far) {
        batch_locate2(b, blk, req, local);
        tile_body<KERN, F32, true, kFormsFar>(*b.v[req], b.mode, local, sm);
    } else {
        batch_locate(b, blk, req, local);
        const ReqView V = load_view(b.v[req]);
        if (b.leaf_wave[req]) {
            // four leaves per block, one per wave, each wave with its own stage
            // (the same per-wave work as in k_tile_wave, so a request's result does
            // not depend on the other requests of its batch)
            constexpr int kWaveBytes = wave_lds_bytes<F32>();
            static_assert(4 * kWaveBytes <= int(sizeof(sm)), "wave stages");
            const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            const int leaf = 4 * local + wave;
            char* st = reinterpret_cast<char*>(&sm) + wave * kWaveBytes;
            if (leaf < V.nleaves_t)
                tile_leaf_wave<KERN, F32, PPONLY ? kFormsPP : kFormsFar>(V, b.mode, leaf,
                                                                         b.sym[req] != 0, st);
        } else {
            tile_body<KERN, F32, false, PPONLY ? kFormsPP : kFormsFar>(V, b.mode, local, sm);
        }
    }
}

// Near-field launch whose requests all take the one-wave-per-leaf path: four
// target leaves per block, one a wave, the waves independent of each other
// (measured faster than blocks of one wave).
template <int KERN, bool F32>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(F32 ? (KERN == CSFMM_K_BIOT_SAVART ? 5 : 6) : 4))) void k_tile_wave(Batch b) {
    constexpr int kWaveBytes = wave_lds_bytes<F32>();
    __shared__ __attribute__((aligned(16))) char lds[(kThreads / 64) * kWaveBytes];
    int req, local;
    batch_locate(b, xcd_logical_block(blockIdx.x, gridDim.x), req, local);
    const ReqView V = load_view(b.v[req]);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int leaf = 4 * local + wave;
    if (leaf < V.nleaves_t)
        tile_leaf_wave<KERN, F32, kFormsPP>(V, b.mode, leaf, b.sym[req] != 0,
                                            lds + wave * kWaveBytes);
}

// Adds the column sums of the symmetric PP pairs owned by other leaves to the
// near field of each target leaf (one wave per leaf, four per block, the
// block layout of the PP launch), in the order of the leaf's receive list, so
// the result does not depend on scheduling.
template <int KERN, bool F32>
__global__ __launch_bounds__(kThreads) void k_sym_merge(Batch b) {
    int req, local;
    batch_locate(b, xcd_logical_block(blockIdx.x, gridDim.x), req, local);
    if (!b.sym[req]) return;
    const ReqView V = load_view(b.v[req]);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int leaf = 4 * local + wave;
    if (leaf >= V.nleaves_t) return;
    const int T = gload(V.t_leaves, leaf);
    const int nT = gload(V.t_count, T), tb = gload(V.t_begin, T);
    const int r0 = gload(V.recv_off, T), r1 = gload(V.recv_off, T + 1);
    const Real<F32>* cols = static_cast<const Real<F32>*>(V.sym_col);
    double acc = 0.0;
    for (int k = r0; k < r1; ++k) {
        const int64_t slot = gload(V.recv_slot, k);
        if (lane < nT) acc += double(cols[slot * kWaveLeaf + lane]);
    }
    if (lane < nT && r1 > r0) {
        double o;
        epilogue<KERN, F32>(&acc, 0.0, 0.0, 0.0, &o);
        V.phinear[tb + lane] += o;
    }
}

// ----------------------------------------------------------------- direct
// Direct sum over all sources (paper §1).  Grid (target blocks of 64, source
// splits); FP32 form on hi/lo split coordinates.  Partial sums per split
// [split][VD][nt] are combined in order by k_direct_reduce.
template <bool F32>
struct DSrc;
template <>
struct alignas(16) DSrc<true> {
    float hx, hy, hz, w, lx, ly, lz, pad;
};
template <>
struct alignas(32) DSrc<false> {
    double x, y, z, w;
};

template <int KERN, bool F32>
__global__ __launch_bounds__(kThreads) void k_direct(const double* __restrict__ tgt, int64_t nt,
                                                     const double* __restrict__ srcp, int64_t ns,
                                                     const double* __restrict__ w, int64_t nsp,
                                                     double* __restrict__ part) {
    using R = Real<F32>;
    constexpr int VD = vdim<KERN>();
    __shared__ DSrc<F32> src[kChunk];
    __shared__ double red[VD][kThreads];
    const int tid = threadIdx.x;
    const int t = tid & 63, g = tid >> 6;  // 64 targets x 4 source groups
    const int64_t i = int64_t(blockIdx.x) * 64 + t;
    const bool valid = i < nt;
    const double gx = valid ? tgt[3 * i] : 0.0, gy = valid ? tgt[3 * i + 1] : 0.0,
                 gz = valid ? tgt[3 * i + 2] : 0.0;
    R hx, hy, hz, lx = R(0), ly = R(0), lz = R(0);
    hx = R(gx);
    hy = R(gy);
    hz = R(gz);
    if constexpr (F32) {
        lx = R(gx - double(hx));
        ly = R(gy - double(hy));
        lz = R(gz - double(hz));
    }
    const int64_t s0 = int64_t(blockIdx.y) * nsp;
    const int64_t s1 = (s0 + nsp < ns) ? s0 + nsp : ns;
    double acc[VD];
#pragma unroll
    for (int v = 0; v < VD; ++v) acc[v] = 0.0;
    for (int64_t q0 = s0; q0 < s1; q0 += kChunk) {
        const int nq = int((s1 - q0 < kChunk) ? s1 - q0 : int64_t(kChunk));
        for (int q = tid; q < nq; q += kThreads) {
            const int64_t j = q0 + q;
            const double yx = srcp[3 * j], yy = srcp[3 * j + 1], yz = srcp[3 * j + 2];
            DSrc<F32> e;
            if constexpr (F32) {
                e.hx = float(yx);
                e.hy = float(yy);
                e.hz = float(yz);
                e.lx = float(yx - double(e.hx));
                e.ly = float(yy - double(e.hy));
                e.lz = float(yz - double(e.hz));
                e.w = float(w[j]);
                e.pad = 0.f;
            } else {
                e.x = yx;
                e.y = yy;
                e.z = yz;
                e.w = w[j];
            }
            src[q] = e;
        }
        __syncthreads();
        R p[VD];
#pragma unroll
        for (int v = 0; v < VD; ++v) p[v] = R(0);
        for (int j = g; j < nq; j += 4) {
            const DSrc<F32>& e = src[j];
            R dx, dy, dz;
            if constexpr (F32) {
                dx = (e.hx - hx) + (e.lx - lx);
                dy = (e.hy - hy) + (e.ly - ly);
                dz = (e.hz - hz) + (e.lz - lz);
            } else {
                dx = e.x - hx;
                dy = e.y - hy;
                dz = e.z - hz;
            }
            const R r2 = dx * dx + dy * dy + dz * dz;
            if constexpr (KERN == CSFMM_K_POISSON_LOG) {
                R lg;
                if constexpr (F32)
                    lg = dev_log2(R(0.5) * r2);
                else
                    lg = log64(R(0.5) * r2);
                lg = r2 > R(0) ? lg : R(0);
                p[0] = fma(e.w, lg, p[0]);
            } else if constexpr (KERN == CSFMM_K_BIOT_SAVART) {
                R inv;
                if constexpr (F32)
                    inv = dev_rcp(r2);
                else
                    inv = rcp64(r2);
                const R f = r2 > R(0) ? e.w * inv : R(0);
                p[0] = fma(dx, f, p[0]);
                p[1] = fma(dy, f, p[1]);
                p[2] = fma(dz, f, p[2]);
            } else if constexpr (KERN == CSFMM_K_BIHARMONIC) {
                const R g = r2 > R(0) ? dilog_1m(R(0.25) * r2) : R(0);
                p[0] = fma(e.w, g, p[0]);
            } else if constexpr (KERN == CSFMM_K_SAL) {
                const R g = r2 > R(0) ? sal_bracket(R(0.25) * r2) : R(0);
                p[0] = fma(e.w, g, p[0]);
            } else {
                R inv;
                if constexpr (F32)
                    inv = dev_rsq(r2);
                else
                    inv = rsq64(r2);
                const R f = r2 > R(0) ? inv : R(0);
                p[0] = fma(e.w, f, p[0]);
            }
        }
#pragma unroll
        for (int v = 0; v < VD; ++v) acc[v] += double(p[v]);
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < VD; ++v) red[v][tid] = acc[v];
    __syncthreads();
    if (tid < 64 && valid) {
#pragma unroll
        for (int v = 0; v < VD; ++v) {
            const double r = red[v][tid] + red[v][64 + tid] + red[v][128 + tid] + red[v][192 + tid];
            part[(int64_t(blockIdx.y) * VD + v) * nt + i] = r;
        }
    }
}

template <int KERN, bool F32>
__global__ void k_direct_reduce(const double* __restrict__ tgt, int64_t nt,
                                const double* __restrict__ part, int nsplit,
                                double* __restrict__ out) {
    constexpr int VD = vdim<KERN>();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    double acc[VD], o[VD];
#pragma unroll
    for (int v = 0; v < VD; ++v) {
        acc[v] = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) acc[v] += part[(int64_t(sp) * VD + v) * nt + i];
    }
    epilogue<KERN, F32>(acc, tgt[3 * i], tgt[3 * i + 1], tgt[3 * i + 2], o);
    // Biot-Savart acc holds sum (y - x) w / |x-y|^2 like the tile kernels.
#pragma unroll
    for (int v = 0; v < VD; ++v) out[i * VD + v] = o[v];
}

// ---------------------------------------------------------------- treecode
// Cubed sphere treecode (paper §7, Algorithm 1), FP64.  A wave owns 64
// consecutive targets of the sorted target order (so its targets are close
// together) and walks the source tree depth first from the six roots with a
// stack of (cluster, lane mask) in LDS; the mask holds the lanes whose
// traversal reaches the cluster.  At a cluster every lane decides for its own
// target: separated (r^2 < MAC^2 R^2, R from the target to the centre) with
// more than N0 points -> PC over the cluster's proxies; separated with at
// most N0 points, or a leaf that is not separated -> PP over its points;
// otherwise the cluster is opened and its non-empty children are pushed with
// the mask of the lanes that opened it.  Each lane accumulates only its own
// interactions, so the result is the per-target traversal of Algorithm 1.
// Stack bound: at most 5 waiting roots and 3 waiting siblings per level below
// them, plus 4 pushed children: 5 + 3 * 19 + 4 = 66 entries for 20 levels.
// A push beyond the stack sets the status word instead (the host then fails
// the call), so a broken bound can never drop a cluster silently.
constexpr int kTcStack = 72;

__device__ __forceinline__ bool tc_separated(double x, double y, double z, const double* c,
                                             double r, double theta2) {
#pragma clang fp contract(off)
    const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
    const double R2 = dx * dx + dy * dy + dz * dz;
    return r * r < theta2 * R2;
}

template <int KERN>
__global__ __launch_bounds__(256) void k_treecode(TcArgs a) {
    // The coordinate scaling below must round before eval_pair subtracts: a
    // multiply fused into the subtraction would leave the rounding residue of
    // x * scale instead of an exact 0 for a coincident target and source.
#pragma clang fp contract(off)
    constexpr int VD = vdim<KERN>();
    constexpr double scale = coord_scale<KERN>();
    __shared__ int st_node[4][kTcStack];
    __shared__ uint32_t st_lo[4][kTcStack], st_hi[4][kTcStack];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t(blockIdx.x) * 4 + wv) * 64 + lane;
    const bool valid = i < a.nt;
    const double gx = valid ? a.tx[i] : 0.0, gy = valid ? a.ty[i] : 0.0,
                 gz = valid ? a.tz[i] : 0.0;
    TargetRegs T;
    T.tx = gx * scale;
    T.ty = gy * scale;
    T.tz = gz * scale;
    double acc[VD];
#pragma unroll
    for (int v = 0; v < VD; ++v) acc[v] = 0.0;
    const uint64_t vmask = __ballot(valid);
    int sp = 0;
    bool overflow = false;
    if (vmask) {
        for (int c = a.nroots - 1; c >= 0; --c)
            if (a.scount[c] > 0) {
                st_node[wv][sp] = c;
                st_lo[wv][sp] = uint32_t(vmask);
                st_hi[wv][sp] = uint32_t(vmask >> 32);
                ++sp;
            }
    }
    while (sp > 0) {
        --sp;
        const int c = __builtin_amdgcn_readfirstlane(st_node[wv][sp]);
        // (through uint32_t: readfirstlane returns a signed int)
        const uint64_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(st_hi[wv][sp])));
        const uint64_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(st_lo[wv][sp])));
        const uint64_t m = (hi << 32) | lo;
        const bool mine = (m >> lane) & 1;
        const int cnt = a.scount[c];
        const int c0 = a.schild0[c];
        const bool leaf = c0 < 0;
        const bool sep = mine && tc_separated(gx, gy, gz, a.scenter + 3 * int64_t(c),
                                              a.sradius[c], a.theta2);
        const bool pc = sep && cnt > a.N0;
        const bool pp = mine && !pc && (sep || leaf);
        const bool op = mine && !sep && !leaf;
        if (__ballot(pc)) {
            const double* px = a.sprox + int64_t(c) * 3 * a.KS;
            const double* pw = a.swbar + int64_t(c) * a.KS;
            for (int k = 0; k < a.K; ++k) {
                if (pc)
                    eval_pair<KERN, false, FORM_NEAR>(T, px[k] * scale, px[a.KS + k] * scale,
                                                      px[2 * a.KS + k] * scale, 0.0, pw[k], acc);
            }
        }
        if (__ballot(pp)) {
            const int b0 = a.sbegin[c];
            for (int j = b0; j < b0 + cnt; ++j) {
                if (pp)
                    eval_pair<KERN, false, FORM_CHECK>(T, a.sx[j] * scale, a.sy[j] * scale,
                                                       a.sz[j] * scale, 0.0, a.sw[j], acc);
            }
        }
        const uint64_t om = __ballot(op);
        if (om) {
            for (int q = 3; q >= 0; --q) {
                if (a.scount[c0 + q] <= 0) continue;
                if (sp >= kTcStack) {
                    overflow = true;
                    continue;
                }
                st_node[wv][sp] = c0 + q;
                st_lo[wv][sp] = uint32_t(om);
                st_hi[wv][sp] = uint32_t(om >> 32);
                ++sp;
            }
        }
    }
    if (overflow && lane == 0) *a.status = 1;
    if (valid) {
        double o[VD];
        epilogue<KERN, false>(acc, gx, gy, gz, o);
        const int64_t dst = a.tperm[i];
#pragma unroll
        for (int v = 0; v < VD; ++v) a.out[dst * VD + v] = o[v];
    }
}

}  // namespace

// Compute units of the current device (queried once per device).
int device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

namespace {

template <int KERN, bool F32>
int launch_tile_t(const Batch& b, hipStream_t s) {
    const int nblocks = b.prefix[b.n] + b.prefix2[b.n];
    if (nblocks <= 0) return CSFMM_OK;
    if (b.wave_kernel)
        k_tile_wave<KERN, F32><<<nblocks, kThreads, 0, s>>>(b);
    else if (b.mode == kTileNearPP)
        k_tile<KERN, F32, true><<<nblocks, kThreads, 0, s>>>(b);
    else
        k_tile<KERN, F32, false><<<nblocks, kThreads, 0, s>>>(b);
    CSFMM_LAUNCH_CHECK();
    return CSFMM_OK;
}

// Source splits of the direct sum: enough (target block, split) blocks to
// fill the device, at most one split per source chunk.
int64_t direct_splits(int64_t nt, int64_t ns) {
    const int64_t ntb = (nt + 63) / 64;
    const int64_t maxsplit = (ns + kChunk - 1) / kChunk;
    const int64_t nsplit = (4096 + ntb - 1) / ntb;
    return std::max<int64_t>(1, std::min<int64_t>(nsplit, std::min<int64_t>(maxsplit, 65535)));
}

// Partial sums [split][VD][nt] go to `part` when given (it holds at least
// direct_splits * VD * nt doubles), else to a stream-ordered allocation.
template <int KERN, bool F32>
int launch_direct_t(const double* tgt, int64_t nt, const double* src, int64_t ns, const double* w,
                    double* out, hipStream_t s, double* part) {
    constexpr int VD = vdim<KERN>();
    const int64_t ntb = (nt + 63) / 64;
    const int64_t nsplit = direct_splits(nt, ns);
    const int64_t nsp = (ns + nsplit - 1) / nsplit;
    const bool own = part == nullptr;
    if (own)
        CSFMM_HIP_TRY(hipMallocAsync((void**)&part, sizeof(double) * size_t(nsplit * VD * nt), s));
    k_direct<KERN, F32><<<dim3(unsigned(ntb), unsigned(nsplit)), kThreads, 0, s>>>(tgt, nt, src, ns,
                                                                                  w, nsp, part);
    hipError_t e1 = hipGetLastError();
    k_direct_reduce<KERN, F32><<<unsigned((nt + 255) / 256), 256, 0, s>>>(tgt, nt, part,
                                                                          int(nsplit), out);
    hipError_t e2 = hipGetLastError();
    if (own) (void)hipFreeAsync(part, s);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("direct launch failed: %s",
                  hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return CSFMM_E_HIP;
    }
    return CSFMM_OK;
}

// Scratch of the direct sum for callers that cannot allocate: one array per
// device, held until the process ends.  Host code uses only the device
// address that hipGetSymbolAddress returns for the current device (the
// array's name on the host is a stand-in, not a device address).
static __device__ __align__(256) double scratch[kDirectScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

int scratch_address(double** out) {
    int dev = 0;
    CSFMM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device %d out of range for the scratch table", dev);
        return CSFMM_E_HIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        CSFMM_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return CSFMM_OK;
}

}  // namespace

template <int KERN>
int launch_sym_merge_t(const Batch& b, bool fp32, hipStream_t s) {
    const int nblocks = b.prefix[b.n];
    if (nblocks <= 0) return CSFMM_OK;
    if (fp32)
        k_sym_merge<KERN, true><<<nblocks, kThreads, 0, s>>>(b);
    else
        k_sym_merge<KERN, false><<<nblocks, kThreads, 0, s>>>(b);
    CSFMM_LAUNCH_CHECK();
    return CSFMM_OK;
}

int launch_sym_merge(const Batch& b, int kernel, bool fp32, hipStream_t s) {
    switch (kernel) {
        case CSFMM_K_POISSON_LOG: return launch_sym_merge_t<1>(b, fp32, s);
        case CSFMM_K_INV_DIST: return launch_sym_merge_t<3>(b, fp32, s);
        case CSFMM_K_BIHARMONIC: return launch_sym_merge_t<4>(b, fp32, s);
        case CSFMM_K_SAL: return launch_sym_merge_t<5>(b, fp32, s);
        default:
            set_error("no symmetric PP path for kernel id %d", kernel);
            return CSFMM_E_INVALID;
    }
}

int launch_tile_batch(const Batch& b, int kernel, bool fp32, hipStream_t s) {
    switch (kernel) {
        case CSFMM_K_POISSON_LOG:
            return fp32 ? launch_tile_t<1, true>(b, s) : launch_tile_t<1, false>(b, s);
        case CSFMM_K_BIOT_SAVART:
            return fp32 ? launch_tile_t<2, true>(b, s) : launch_tile_t<2, false>(b, s);
        case CSFMM_K_INV_DIST:
            return fp32 ? launch_tile_t<3, true>(b, s) : launch_tile_t<3, false>(b, s);
        case CSFMM_K_BIHARMONIC:
            return fp32 ? launch_tile_t<4, true>(b, s) : launch_tile_t<4, false>(b, s);
        case CSFMM_K_SAL:
            return fp32 ? launch_tile_t<5, true>(b, s) : launch_tile_t<5, false>(b, s);
        default:
            set_error("unknown kernel id %d", kernel);
            return CSFMM_E_INVALID;
    }
}

int launch_treecode(const TcArgs& a, int kernel, hipStream_t s) {
    const unsigned grid = unsigned((a.nt + 255) / 256);
    if (grid == 0) return CSFMM_OK;
    switch (kernel) {
        case CSFMM_K_POISSON_LOG: k_treecode<1><<<grid, 256, 0, s>>>(a); break;
        case CSFMM_K_BIOT_SAVART: k_treecode<2><<<grid, 256, 0, s>>>(a); break;
        case CSFMM_K_INV_DIST: k_treecode<3><<<grid, 256, 0, s>>>(a); break;
        case CSFMM_K_BIHARMONIC: k_treecode<4><<<grid, 256, 0, s>>>(a); break;
        case CSFMM_K_SAL: k_treecode<5><<<grid, 256, 0, s>>>(a); break;
        default:
            set_error("unknown kernel id %d", kernel);
            return CSFMM_E_INVALID;
    }
    CSFMM_LAUNCH_CHECK();
    return CSFMM_OK;
}

int launch_direct(const double* tgt, int64_t nt, const double* src, int64_t ns, const double* w,
                  int kernel, bool fp32, double* out, hipStream_t s, bool no_alloc) {
    double* part = nullptr;
    if (no_alloc) {
        const int64_t need = direct_splits(nt, ns) * (kernel == CSFMM_K_BIOT_SAVART ? 3 : 1) * nt;
        if (need > kDirectScratchDoubles) {
            set_error("direct without allocation: %lld partial sums exceed the scratch of %lld "
                      "doubles (at most %lld targets, a third for Biot-Savart)",
                      (long long)need, (long long)kDirectScratchDoubles,
                      (long long)kDirectScratchDoubles);
            return CSFMM_E_INVALID;
        }
        int rc = scratch_address(&part);
        if (rc != CSFMM_OK) return rc;
    }
    switch (kernel) {
        case CSFMM_K_POISSON_LOG:
            return fp32 ? launch_direct_t<1, true>(tgt, nt, src, ns, w, out, s, part)
                        : launch_direct_t<1, false>(tgt, nt, src, ns, w, out, s, part);
        case CSFMM_K_BIOT_SAVART:
            return fp32 ? launch_direct_t<2, true>(tgt, nt, src, ns, w, out, s, part)
                        : launch_direct_t<2, false>(tgt, nt, src, ns, w, out, s, part);
        case CSFMM_K_INV_DIST:
            return fp32 ? launch_direct_t<3, true>(tgt, nt, src, ns, w, out, s, part)
                        : launch_direct_t<3, false>(tgt, nt, src, ns, w, out, s, part);
        case CSFMM_K_BIHARMONIC:
            return fp32 ? launch_direct_t<4, true>(tgt, nt, src, ns, w, out, s, part)
                        : launch_direct_t<4, false>(tgt, nt, src, ns, w, out, s, part);
        case CSFMM_K_SAL:
            return fp32 ? launch_direct_t<5, true>(tgt, nt, src, ns, w, out, s, part)
                        : launch_direct_t<5, false>(tgt, nt, src, ns, w, out, s, part);
        default:
            set_error("unknown kernel id %d", kernel);
            return CSFMM_E_INVALID;
    }
}

}  // namespace csfmm
