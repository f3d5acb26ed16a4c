// Device-side building blocks of the all-pairs kernels (gfx950, wave64).
//
// Layout of the packed j-records the kernels stream (written by the pack
// kernels from the caller's FP64 arrays, padded to a multiple of 64 records
// with zero-weight particles placed far away):
//   gravity  {x, y, z, m}                               4 x T
//   LJC      {x, y, z, qs, sh, se, 0, 0}                8 x T
//            qs = q sqrt(2k/D)  so that qs_i qs_j = 2 k q_i q_j / D,
//            sh = sigma / 2     so that sh_i + sh_j = (sigma_i + sigma_j) / 2,
//            se = sqrt(24 eps)  so that se_i se_j = 24 sqrt(eps_i eps_j), the
//                               Lennard-Jones force prefactor.
//   adjoint records append the cotangent g_j = dL/dF_j (see adjoint.hip).
//
// The j index of the inner loop is wave-uniform.  The j records reach the
// arithmetic either through scalar loads into SGPRs (j_stage 0) or through a
// wave-private double-buffered LDS slot read back as broadcasts (j_stage 1);
// see allpairs.h.  The i-particles live in VGPRs, I of them per lane (the
// i-unrolling of Section 3.3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbk {

constexpr int kWave = 64;
constexpr double kPadCoord = 1.0e18;   // position of padding records (weight 0)

enum Law { GRAVITY = 0, LJC = 1, LJC_CONST = 2, LJC_SIG = 3 };

// Law constants seen by every pair: the gravity softening squared and, for
// the sigmoidal dielectric, zeta(r) = exp(za r^3 + zb r^2 + zc r + zd) with
// zb2 = 2 zb and za3 = 3 za precomputed for zeta'/zeta = (za3 r + zb2) r + zc.
template <typename T> struct PairK {
    T eps2;
    T za, zb, zc, zd, za3, zb2;
};
enum Prec { P_FP64 = 0, P_KAHAN = 1, P_FP64ACC = 2, P_PLAIN = 3 };

template <int PREC> struct RealOf { using type = float; };
template <> struct RealOf<P_FP64> { using type = double; };

template <typename T> struct alignas(4 * sizeof(T)) GravRec { T x, y, z, m; };
// gravity adjoint records: position, mass and the cotangent g = dL/da of the particle
template <typename T> struct alignas(4 * sizeof(T)) GravAdjRec { T x, y, z, m, gx, gy, gz, p0; };
template <typename T> struct alignas(4 * sizeof(T)) LjcRec { T x, y, z, qs, sh, se, p0, p1; };

template <typename T, int LAW> struct RecOf { using type = LjcRec<T>; };   // every LJC variant
template <typename T> struct RecOf<T, GRAVITY> { using type = GravRec<T>; };

// ---------------------------------------------------------------- reciprocals
// FP32: the hardware v_rsq_f32 / v_rcp_f32 (about 1 ulp).
// FP64: the hardware estimate refined by two Newton steps (quadratic
// convergence: y <- y (3 - x y^2) / 2 for x^-1/2, y <- y (2 - x y) for x^-1).
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
// e^{-y}: the hardware 2^x (v_exp_f32, about 1 ulp) of -y log2(e) in FP32; libm exp in FP64
__device__ __forceinline__ float exp_neg_(float y) { return __builtin_amdgcn_exp2f(-1.44269504088896341f * y); }
__device__ __forceinline__ double exp_neg_(double y) { return ::exp(-y); }
__device__ __forceinline__ double rsqrt_(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = __builtin_fma(-h, y, 1.0);          // 1 - x y^2
    y = __builtin_fma(0.5 * y, e, y);
    h = x * y;
    e = __builtin_fma(-h, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}
__device__ __forceinline__ double rcp_(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
// v clamped to [lo, hi]: one v_med3_f32 in FP32
__device__ __forceinline__ float clamp_(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }
__device__ __forceinline__ double clamp_(double v, double lo, double hi)
{
    return __builtin_fmin(__builtin_fmax(v, lo), hi);
}

// Bounds on the sigmoidal-dielectric factors.  The exponent of zeta(r) and
// r zeta'/zeta are clamped so that both stay finite for every pair, including
// the zero-charge padding records at 1e18 (whose factors would otherwise be
// 0 * inf).  The exponent bound is reached only where zeta < e^-80 or
// zeta > e^80 (FP32; e^+-700 in FP64), i.e. for Coulomb terms below 1e-35 of
// their unscreened value, so no physical pair is affected.
template <typename T> struct ZetaBound;
template <> struct ZetaBound<float> {
    static constexpr float poly = 80.0f, rdl = 1.0e30f;
};
template <> struct ZetaBound<double> {
    static constexpr double poly = 700.0, rdl = 1.0e300;
};

// ----------------------------------------------------------------- pair laws
// Per-lane i state and the pair contribution to the four running sums
// p[0..2] (vector) and p[3] (potential).  MASK is set only on tiles that may
// contain j == i; there the self pair is neutralised without division by 0.

template <typename T> struct GravI { T x, y, z; };

// Gravity, Eq. 1: p += m_j d / s^3 (d = r_j - r_i), p3 += m_j / s.
// FP32 instruction count: 3 sub, 3 fma (r^2 + eps^2), 1 rsq, 3 mul,
// 3 fma (+1 add for the potential): 19 flops, 20 with the potential
// (multiply-add = 2, rsq = 1).
template <bool MASK, bool POT, typename T>
__device__ __forceinline__ void grav_pair(const GravI<T> &i, T xj, T yj, T zj, T mj,
                                          const PairK<T> &k, bool self, T (&p)[4])
{
    const T dx = xj - i.x, dy = yj - i.y, dz = zj - i.z;
    T r2 = fma_(dx, dx, k.eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    T m = mj;
    if (MASK) {
        r2 = self ? T(1) : r2;
        m = self ? T(0) : m;
    }
    const T ri = rsqrt_(r2);
    const T mr = m * ri;
    const T mr3 = mr * (ri * ri);
    p[0] = fma_(mr3, dx, p[0]);
    p[1] = fma_(mr3, dy, p[1]);
    p[2] = fma_(mr3, dz, p[2]);
    if (POT) p[3] += mr;
}

template <typename T> struct LjcI { T x, y, z, qs, sh, se; };

// LJ + Coulomb, F_i += W (r_i - r_j) = -W d with the Lennard-Jones part
// (24 e x)(2 s6^2 - s6), x = 1/r^2, s6 = (sigma_ij^2 x)^3, and a Coulomb part
// per dielectric (qs carries sqrt of the Coulomb prefactor):
//   LJC       eps(r) = D r : W_C = qq x^2,              p3 += 2u = qq x + 8 e (s6^2 - s6)
//   LJC_CONST eps = D      : W_C = qq / r^3,            p3 += u = qq / r + 4 e (s6^2 - s6)
//   LJC_SIG   eps = zeta(r): W_C = qq (1 + r zeta'/zeta) / (zeta r^3),
//                                                       p3 += u = qq / (zeta r) + 4 e (...)
// FP32 instruction count of LJC without the potential: 3 sub, 1 mul + 2 fma
// (r^2), 1 rcp, 3 mul (qq, e, s^2 x) + 1 add (sigma) + 1 mul (sigma^2), 2 mul
// (s^6), 1 fma (2 s6 - 1), 2 mul, 1 mul (C x), 1 fma + 1 mul (W), 3 fma: 30
// flops; the potential adds 2 fma + 1 add: 35.  LJC_CONST replaces the rcp by
// rsq + 1 mul (31 / 36 flops); LJC_SIG adds r, the two polynomials, exp and
// the (1 + r zeta'/zeta) factor (48 / 53 flops; the two clamps of the zeta
// factors are comparisons, not counted).
// The scalar part of an LJC pair, symmetric in its two atoms: from r^2 and the combined
// charge (qq), Lennard-Jones (e) and sigma (sg) factors, the force factor W (F_i = -W d,
// d = r_j - r_i) and, with POT, the pair's energy term du (2 u_ij for LJC, u_ij for the other
// dielectrics).  The one-sided pair adds W to one atom; the symmetric tiles to both.
template <bool POT, int LAW, typename T>
__device__ __forceinline__ void ljc_terms(T r2, T qq, T e, T sg, const PairK<T> &k, T &W, T &du)
{
    T x, cx, wc;
    if constexpr (LAW == LJC) {
        x = rcp_(r2);
        cx = qq * x;
        wc = cx;
    } else if constexpr (LAW == LJC_CONST) {
        const T ri = rsqrt_(r2);
        x = ri * ri;
        cx = qq * ri;
        wc = cx;
    } else {
        const T ri = rsqrt_(r2);
        x = ri * ri;
        const T r = r2 * ri;
        T poly = fma_(fma_(fma_(k.za, r, k.zb), r, k.zc), r, k.zd);
        poly = clamp_(poly, -ZetaBound<T>::poly, ZetaBound<T>::poly);
        const T dl = fma_(fma_(k.za3, r, k.zb2), r, k.zc);
        const T rdl = clamp_(r * dl, -ZetaBound<T>::rdl, ZetaBound<T>::rdl);
        cx = (qq * ri) * exp_neg_(poly);
        wc = fma_(cx, rdl, cx);
    }
    const T s2 = (sg * sg) * x;
    const T s6 = (s2 * s2) * s2;
    const T lj = e * s6;                     // 24 eps_ij (sigma_ij / r)^6
    const T t = fma_(s6, T(2), T(-1));
    W = fma_(lj, t, wc) * x;                 // (24 eps_ij (2 s^12 - s^6) + wc) / r^2
    if (POT) {
        const T v = fma_(lj, s6, -lj);       // 24 eps_ij (s^12 - s^6)
        if constexpr (LAW == LJC)
            du = fma_(v, T(1.0 / 3.0), cx);  // 2 u_ij
        else
            du = fma_(v, T(1.0 / 6.0), cx);  // u_ij
    }
}

template <bool MASK, bool POT, int LAW, typename T>
__device__ __forceinline__ void ljc_pair(const LjcI<T> &i, T xj, T yj, T zj, T qsj, T shj, T sej,
                                         const PairK<T> &k, bool self, T (&p)[4])
{
    const T dx = xj - i.x, dy = yj - i.y, dz = zj - i.z;
    T r2 = dx * dx;
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    T qq = i.qs * qsj;
    T e = i.se * sej;
    if (MASK) {
        r2 = self ? T(1) : r2;
        qq = self ? T(0) : qq;
        e = self ? T(0) : e;
    }
    T W, du = T(0);
    ljc_terms<POT, LAW>(r2, qq, e, i.sh + shj, k, W, du);
    p[0] = fma_(-W, dx, p[0]);
    p[1] = fma_(-W, dy, p[1]);
    p[2] = fma_(-W, dz, p[2]);
    if (POT) p[3] += du;
}

// ------------------------------------------------------------ running sums
// A tile partial p (FP32 or FP64, started at 0) is folded into the running
// sum at the end of each j-tile.
template <int PREC> struct RunSum;

template <> struct RunSum<P_FP64ACC> {     // FP32 partial -> FP64 sum
    double s = 0.0;
    __device__ void begin(float &p) const { p = 0.0f; }
    __device__ void fold(float p) { s += (double)p; }
    __device__ double value() const { return s; }
};

template <> struct RunSum<P_KAHAN> {       // FP32 partial -> Kahan FP32 sum
    float s = 0.0f, c = 0.0f;
    __device__ void begin(float &p) const { p = 0.0f; }
    __device__ void fold(float p)
    {
#pragma clang fp contract(off)
        const float y = p - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ double value() const { return (double)s - (double)c; }
};

template <> struct RunSum<P_PLAIN> {       // one plain FP32 sum over all j
    float s = 0.0f;
    __device__ void begin(float &p) const { p = s; }
    __device__ void fold(float p) { s = p; }
    __device__ double value() const { return (double)s; }
};

template <> struct RunSum<P_FP64> {        // FP64 partial -> Neumaier FP64 sum
    double s = 0.0, c = 0.0;
    __device__ void begin(double &p) const { p = 0.0; }
    __device__ void fold(double p)
    {
#pragma clang fp contract(off)
        const double t = s + p;
        c += (__builtin_fabs(s) >= __builtin_fabs(p)) ? ((s - t) + p) : ((p - t) + s);
        s = t;
    }
    __device__ double value() const { return s + c; }
};

// Neumaier-compensated FP64 accumulation used by the fixed-order reductions.
struct NSum {
    double s = 0.0, c = 0.0;
    __device__ void add(double x)
    {
#pragma clang fp contract(off)
        const double t = s + x;
        c += (__builtin_fabs(s) >= __builtin_fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ double value() const { return s + c; }
    // add another compensated sum; commutative bit for bit, so both lanes of a
    // butterfly pair end with the same (s, c)
    __device__ void merge(double s2, double c2)
    {
#pragma clang fp contract(off)
        const double t = s + s2;
        const double e = (__builtin_fabs(s) >= __builtin_fabs(s2)) ? ((s - t) + s2) : ((s2 - t) + s);
        c = (c + c2) + e;
        s = t;
    }
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The value of lane (l + 1) mod 64, for the symmetric tiles' j sums that travel with their
// particle: through the LDS crossbar (ds_bpermute, no LDS memory; byte_addr = 4 ((l + 1) mod 64)),
// or on the VALU by a DPP rotation of the whole wave by one lane (wave_rol:1).
__device__ __forceinline__ float from_next_lane(int byte_addr, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(byte_addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float from_next_lane_dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}

// Fixed-order sum of the nsplit partials of row r (part s at
// partial + s * part_stride + r * width, NC columns) by a group of G lanes (G
// a power of two <= 64, groups aligned in the wave): lane q of the group adds
// parts q, q + G, q + 2G, ... in that order, then the group merges its lanes
// over log2 G butterfly steps.  Every lane of the group ends with the same
// sums.  All lanes of the wave must take part (lanes without a row pass
// valid = false).
template <int NC>
__device__ __forceinline__ void split_group_sum(const double *__restrict__ partial, int64_t part_stride,
                                                int width, int64_t r, bool valid, int64_t nsplit, int q,
                                                int G, double (&out)[NC])
{
    NSum v[NC];
    if (valid) {
        // four parts' loads in flight before their adds (the adds keep the order)
        int64_t s = q;
        for (; s + 3 * G < nsplit; s += 4 * G) {
            double x[4][NC];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < NC; ++c) x[u][c] = partial[(s + u * G) * part_stride + r * width + c];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < NC; ++c) v[c].add(x[u][c]);
        }
        for (; s < nsplit; s += G) {
            const double *o = partial + s * part_stride + r * width;
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c].add(o[c]);
        }
    }
    for (int m = 1; m < G; m <<= 1)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double s2 = __shfl_xor(v[c].s, m);
            const double c2 = __shfl_xor(v[c].c, m);
            v[c].merge(s2, c2);
        }
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = v[c].value();
}

// wave-uniform "any lane" (result lives in an SGPR)
__device__ __forceinline__ bool wave_any(bool v) { return __any(v) != 0; }

}  // namespace nbk
