// Device-side building blocks of the all-pairs kernels (gfx950, wave64).
//
// Layout of the packed j-records the kernels stream (written by the pack
// kernels from the caller's FP64 arrays, padded to a multiple of 64 records
// with zero-weight particles placed far away):
//   gravity  {x, y, z, m}                               4 x T
//   LJC      {x, y, z, qs, sh, se, 0, 0}                8 x T
//            qs = q sqrt(2k/D)  so that qs_i qs_j = 2 k q_i q_j / D,
//            sh = sigma / 2     so that sh_i + sh_j = (sigma_i + sigma_j) / 2,
//            se = sqrt(eps)     so that se_i se_j = sqrt(eps_i eps_j).
//   adjoint records append the cotangent g_j = dL/dF_j (see adjoint.hip).
//
// The j index of the inner loop is wave-uniform, so record loads compile to
// scalar loads (s_load) into SGPRs and every VALU instruction of the pair
// arithmetic takes its j operand straight from an SGPR: the j stream costs no
// VGPRs, no LDS and no barriers.  The i-particles live in VGPRs, I of them per
// lane (the i-unrolling of Section 3.3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbk {

constexpr int kWave = 64;
constexpr double kPadCoord = 1.0e18;   // position of padding records (weight 0)

enum Law { GRAVITY = 0, LJC = 1 };
enum Prec { P_FP64 = 0, P_KAHAN = 1, P_FP64ACC = 2, P_PLAIN = 3 };

template <int PREC> struct RealOf { using type = float; };
template <> struct RealOf<P_FP64> { using type = double; };

template <typename T> struct alignas(4 * sizeof(T)) GravRec { T x, y, z, m; };
template <typename T> struct alignas(4 * sizeof(T)) LjcRec { T x, y, z, qs, sh, se, p0, p1; };

template <typename T, int LAW> struct RecOf;
template <typename T> struct RecOf<T, GRAVITY> { using type = GravRec<T>; };
template <typename T> struct RecOf<T, LJC> { using type = LjcRec<T>; };

// ---------------------------------------------------------------- reciprocals
// FP32: the hardware v_rsq_f32 / v_rcp_f32 (about 1 ulp).
// FP64: the hardware estimate refined by two Newton steps (quadratic
// convergence: y <- y (3 - x y^2) / 2 for x^-1/2, y <- y (2 - x y) for x^-1).
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
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
__device__ __forceinline__ void grav_pair(const GravI<T> &i, T xj, T yj, T zj, T mj, T eps2,
                                          bool self, T (&p)[4])
{
    const T dx = xj - i.x, dy = yj - i.y, dz = zj - i.z;
    T r2 = fma_(dx, dx, eps2);
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

// LJC(linear): p -= W d with W = 2kqq/(D r^4) + (24 e/r^2)(2 s^12/r^12 - s^6/r^6),
// p3 += 2 u_ij = kqq/(D r^2) * 2 + 8 e ((s/r)^12 - (s/r)^6).
// FP32 instruction count without the potential: 3 sub, 1 mul + 2 fma (r^2),
// 1 rcp, 3 mul (qq, e, s^2 x) + 1 add (sigma) + 1 mul (sigma^2), 2 mul (s^6),
// 1 fma (2 s6 - 1), 2 mul, 1 mul (C x), 1 fma + 1 mul (W), 3 fma: 30 flops;
// the potential adds 2 fma + 1 add: 35 flops.
template <bool MASK, bool POT, typename T>
__device__ __forceinline__ void ljc_pair(const LjcI<T> &i, T xj, T yj, T zj, T qsj, T shj, T sej,
                                         bool self, T (&p)[4])
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
    const T x = rcp_(r2);
    const T sg = i.sh + shj;
    const T s2 = (sg * sg) * x;
    const T s6 = (s2 * s2) * s2;
    const T lj = e * s6;
    const T t = fma_(s6, T(2), T(-1));
    const T wl = lj * t;
    const T cx = qq * x;
    const T W = fma_(wl, T(24), cx) * x;
    p[0] = fma_(-W, dx, p[0]);
    p[1] = fma_(-W, dy, p[1]);
    p[2] = fma_(-W, dz, p[2]);
    if (POT) {
        const T v = fma_(lj, s6, -lj);       // e (s6^2 - s6)
        p[3] += fma_(v, T(8), cx);           // 2 u_ij
    }
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
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// wave-uniform "any lane" (result lives in an SGPR)
__device__ __forceinline__ bool wave_any(bool v) { return __any(v) != 0; }

}  // namespace nbk
