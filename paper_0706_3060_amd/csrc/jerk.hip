// Gravitational acceleration and jerk (Table 1 "Gravity (accel & jerk)", the
// GAJ kernel of Section 2) and the fourth-order Hermite integrator that uses
// them, with a shared step or with block individual steps (the setting in
// which Section 3.4 evaluates forces on a subset of the particles).
//
//   pack / predict   FP64 state -> padded records {x, y, z, m, vx, vy, vz, 0},
//                    optionally after the Hermite predictor to a common time;
//   k_jerk           the shared tiled j loop (allpairs.h) with the GAJ pair
//                    operation, over all rows or a row list;
//   k_jerk_reduce    fixed-order sum of the j-split partials;
//   k_hermite_correct  FP64 corrector (and, for block steps, the next step);
//   k_sched_*        block-step scheduling on the device: the next block time
//                    and the ordered list of the particles due then.
#include <type_traits>

#include "allpairs.h"
#include "kernels.h"
#include "jerk.h"

namespace nbk {

template <typename T> struct alignas(4 * sizeof(T)) GajRec { T x, y, z, m, vx, vy, vz, p0; };
template <typename T> struct GajI { T x, y, z, vx, vy, vz; };

template <typename T>
__device__ __forceinline__ void load_i(const GajRec<T> *rec, int64_t p, GajI<T> &s)
{
    const GajRec<T> r = rec[p];
    s.x = r.x;
    s.y = r.y;
    s.z = r.z;
    s.vx = r.vx;
    s.vy = r.vy;
    s.vz = r.vz;
}

template <typename T> __device__ __forceinline__ void settle(const GajI<T> &s)
{
    asm volatile("" ::"v"(s.x), "v"(s.y), "v"(s.z), "v"(s.vx), "v"(s.vy), "v"(s.vz));
}

// One pair: with d = r_j - r_i, w = v_j - v_i, s^2 = |d|^2 + eps^2,
//   a    += m_j d / s^3
//   jerk += m_j [ w - 3 (d.w) d / s^2 ] / s^3
//   phi  += m_j / s                                (scaled by -G at the end)
// FP32 instruction count: 6 sub, 3 fma (s^2), 1 rsq, 3 mul (1/s^2, m/s,
// m/s^3), 1 mul + 2 fma (d.w), 2 mul (-3 (d.w)/s^2), 3 fma (a), 3 fma
// (w - 3 (d.w) d / s^2), 3 fma (jerk): 41 flops (multiply-add = 2, rsq = 1);
// the potential adds 1: 42, Table 1's count for this kernel.
template <bool MASK, bool POT, typename T>
__device__ __forceinline__ void gaj_pair(const GajI<T> &i, const GajRec<T> &j, T eps2, bool self,
                                         T (&p)[8])
{
    const T dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
    const T wx = j.vx - i.vx, wy = j.vy - i.vy, wz = j.vz - i.vz;
    T r2 = fma_(dx, dx, eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    T m = j.m;
    if (MASK) {
        r2 = self ? T(1) : r2;
        m = self ? T(0) : m;
    }
    const T ri = rsqrt_(r2);
    const T ri2 = ri * ri;
    const T mr = m * ri;
    const T mr3 = mr * ri2;
    T dw = dx * wx;
    dw = fma_(dy, wy, dw);
    dw = fma_(dz, wz, dw);
    const T q = (dw * ri2) * T(-3);
    p[0] = fma_(mr3, dx, p[0]);
    p[1] = fma_(mr3, dy, p[1]);
    p[2] = fma_(mr3, dz, p[2]);
    const T ux = fma_(q, dx, wx), uy = fma_(q, dy, wy), uz = fma_(q, dz, wz);
    p[3] = fma_(mr3, ux, p[3]);
    p[4] = fma_(mr3, uy, p[4]);
    p[5] = fma_(mr3, uz, p[5]);
    if (POT) p[6] += mr;
}

template <bool POT> struct JerkOp {
    static constexpr int NC = POT ? 7 : 6;
    static constexpr int NP = 8;
    template <bool MASK, typename T>
    static __device__ __forceinline__ void run(const GajI<T> &i, const GajRec<T> &j, const PairK<T> &k,
                                               bool self, T (&p)[NP])
    {
        gaj_pair<MASK, POT>(i, j, k.eps2, self, p);
    }
};

// ------------------------------------------------------- pack and predict ----
// Hermite predictor over a time tau (FP64):
//   xp = x + v tau + a tau^2/2 + jerk tau^3/6,  vp = v + a tau + jerk tau^2/2
__device__ __forceinline__ void predict(const double *x, const double *v, const double *a,
                                        const double *j, double tau, double *xp, double *vp)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xp[c] = x[c] + tau * (v[c] + tau * (0.5 * a[c] + tau * (j[c] / 6.0)));
        vp[c] = v[c] + tau * (a[c] + tau * (0.5 * j[c]));
    }
}

// record i of the (optionally predicted) state; padding records past n
template <typename T>
__device__ __forceinline__ void pack_record(const JerkPackLaunch &a, int64_t i)
{
    GajRec<T> r;
    if (i >= a.n) {
        r.x = r.y = r.z = (T)kPadCoord;
        r.m = r.vx = r.vy = r.vz = r.p0 = T(0);
        ((GajRec<T> *)a.rec)[i] = r;
        return;
    }
    double x[3], v[3];
    if (a.predict) {
        const double tp = a.t_pred_dev ? *a.t_pred_dev : a.t_pred;
        const double tau = a.t_i ? tp - a.t_i[i] : a.tau;
        predict(a.pos + 3 * i, a.vel + 3 * i, a.acc + 3 * i, a.jerk + 3 * i, tau, x, v);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = a.pos[3 * i + c];
            v[c] = a.vel[3 * i + c];
        }
    }
    r.x = (T)x[0];
    r.y = (T)x[1];
    r.z = (T)x[2];
    r.m = (T)a.mass[i];
    r.vx = (T)v[0];
    r.vy = (T)v[1];
    r.vz = (T)v[2];
    r.p0 = T(0);
    ((GajRec<T> *)a.rec)[i] = r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack_jerk(JerkPackLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.npad) return;
    if (a.live_dev && *a.live_dev <= 0) return;      // a block step with nothing due
    pack_record<T>(a, i);
}

hipError_t launch_pack_jerk(const JerkPackLaunch &p, hipStream_t s)
{
    if (p.npad <= 0) return hipSuccess;
    const dim3 grid((unsigned)((p.npad + 255) / 256)), block(256);
    if (p.prec != P_FP64) hipLaunchKernelGGL(k_pack_jerk<float>, grid, block, 0, s, p);
    else hipLaunchKernelGGL(k_pack_jerk<double>, grid, block, 0, s, p);
    return hipGetLastError();
}

// --------------------------------------------------------------- all pairs ----
// rows to evaluate and the split, fixed or read from device memory (clamped to
// the bounds the grid and the partial buffer were sized for)
__device__ __forceinline__ int64_t dev_rows(int64_t fixed, const int64_t *dev)
{
    if (!dev) return fixed;
    const int64_t d = *dev;
    return d < fixed ? (d > 0 ? d : 0) : fixed;
}

// (a device split is also held to what the partial buffer holds for nrows rows;
// the jerk kernel and the kernel summing its partials apply the same clamp)
__device__ __forceinline__ int64_t dev_split(int64_t bound, const int64_t *dev, int64_t cap_rows,
                                             int64_t nrows)
{
    if (!dev) return bound;
    if (cap_rows > 0 && nrows > 0 && cap_rows / nrows < bound) bound = cap_rows / nrows;
    const int64_t d = *dev;
    return d < 1 ? 1 : (d > bound ? bound : d);
}

__device__ __forceinline__ void jerk_finish(const JerkLaunch &a, int64_t r, const double *v, bool pot)
{
    a.out_acc[3 * r] = a.G * v[0];
    a.out_acc[3 * r + 1] = a.G * v[1];
    a.out_acc[3 * r + 2] = a.G * v[2];
    a.out_jerk[3 * r] = a.G * v[3];
    a.out_jerk[3 * r + 1] = a.G * v[4];
    a.out_jerk[3 * r + 2] = a.G * v[5];
    if (pot && a.out_pot) a.out_pot[r] = -a.G * v[6];
}

template <int PREC, int I, bool POT, int JS>
__global__ __launch_bounds__(256) void k_jerk(const GajRec<typename RealOf<PREC>::type> *__restrict__ rec,
                                              JerkLaunch a)
{
    using T = typename RealOf<PREC>::type;
    using R = GajRec<T>;
    using Op = JerkOp<POT>;
    constexpr int NC = Op::NC;
    const int lane = lane_id();
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nrows = dev_rows(a.nrows, a.nrows_dev);
    int64_t part = blockIdx.y, split_len = a.split_len, nsplit = a.j_split;
    if (a.split_dev) {
        // 1-D grid: wave w takes row wave w % rw of j part w / rw, for the split
        // the scheduler chose
        const int64_t rw = (nrows + kWave * I - 1) / (kWave * I);
        nsplit = dev_split(a.j_split, a.split_dev, a.partial_rows, nrows);
        if (rw == 0 || wave >= rw * nsplit) return;
        part = wave / rw;
        wave -= part * rw;
        split_len = ((a.npad + nsplit - 1) / nsplit + kWave - 1) / kWave * kWave;
    }
    const int64_t rbase = wave * (int64_t)(kWave * I);
    if (rbase >= nrows) return;
    const int64_t jb = part * split_len;
    const int64_t je = (jb + split_len < a.npad) ? jb + split_len : a.npad;

    GajI<T> is[I];
    int64_t pid[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
        int64_t r = rbase + lane + (int64_t)kWave * k;
        r = r < nrows ? r : nrows - 1;
        int64_t q = a.rows ? a.rows[r] : r;
        q = q < 0 ? 0 : (q < a.npad ? q : a.npad - 1);     // never read outside the records
        pid[k] = q;
        load_i(rec, q, is[k]);
    }
    RunSum<PREC> acc[I][NC];
    T p[I][Op::NP];
#pragma unroll
    for (int k = 0; k < I; ++k) p[k][6] = T(0);
    __shared__ R lds_j[JS ? 4 : 1][2][kWave];
    PairK<T> kc{};
    kc.eps2 = (T)a.eps2;
    j_range<JS, Op, PREC, I>(rec, jb, je, a.j_tile, is, pid, kc, acc, p,
                             lds_j[JS ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0]);
#pragma unroll
    for (int k = 0; k < I; ++k) {
        const int64_t r = rbase + lane + (int64_t)kWave * k;
        if (r >= nrows) continue;
        double v[8];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = acc[k][c].value();
        if (nsplit > 1) {
            double *o = a.partial + (part * nrows + r) * 8;
#pragma unroll
            for (int c = 0; c < NC; ++c) o[c] = v[c];
        } else {
            jerk_finish(a, r, v, POT);
        }
    }
}

template <int PREC, int I, bool POT>
static void launch_jerk_one(const JerkLaunch &a, dim3 grid, hipStream_t s)
{
    using T = typename RealOf<PREC>::type;
    if (a.j_stage == 1)
        hipLaunchKernelGGL((k_jerk<PREC, I, POT, 1>), grid, dim3(a.block), 0, s, (const GajRec<T> *)a.rec, a);
    else
        hipLaunchKernelGGL((k_jerk<PREC, I, POT, 0>), grid, dim3(a.block), 0, s, (const GajRec<T> *)a.rec, a);
}

template <int PREC, bool POT>
static bool jerk_ipl(const JerkLaunch &a, dim3 grid, hipStream_t s)
{
    switch (a.ipl) {
    case 1: launch_jerk_one<PREC, 1, POT>(a, grid, s); return true;
    case 2: launch_jerk_one<PREC, 2, POT>(a, grid, s); return true;
    default: return false;
    }
}

template <bool POT>
static bool jerk_prec(const JerkLaunch &a, dim3 grid, hipStream_t s)
{
    switch (a.prec) {
    case P_FP64: return jerk_ipl<P_FP64, POT>(a, grid, s);
    case P_KAHAN: return jerk_ipl<P_KAHAN, POT>(a, grid, s);
    case P_FP64ACC: return jerk_ipl<P_FP64ACC, POT>(a, grid, s);
    default: return false;
    }
}

hipError_t launch_jerk(const JerkLaunch &a, hipStream_t s)
{
    if (a.nrows <= 0) return hipSuccess;
    // a launch description missing its buffers or tile is refused, never launched
    if (!a.rec || !a.out_acc || !a.out_jerk || (a.j_split > 1 && !a.partial) || a.j_tile <= 0 ||
        a.npad <= 0 || a.npad % kWave != 0)
        return hipErrorInvalidValue;
    const int64_t waves = a.split_dev ? a.grid_waves
                                      : (a.nrows + (int64_t)kWave * a.ipl - 1) / ((int64_t)kWave * a.ipl);
    const int64_t wpb = a.block / kWave;
    if (waves <= 0) return hipSuccess;
    const dim3 grid((unsigned)((waves + wpb - 1) / wpb), a.split_dev ? 1u : (unsigned)a.j_split);
    const bool ok = a.pot ? jerk_prec<true>(a, grid, s) : jerk_prec<false>(a, grid, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// Fixed-order sum of the j-split partials, split_group(split) lanes per row.
template <bool POT>
__global__ __launch_bounds__(256) void k_jerk_reduce(JerkLaunch a)
{
    const int64_t nrows = dev_rows(a.nrows, a.nrows_dev);
    const int64_t nsplit = dev_split(a.j_split, a.split_dev, a.partial_rows, nrows);
    if (nsplit <= 1) return;                         // the kernel wrote the rows itself
    const int G = split_group(nsplit);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((tid & ~int64_t(kWave - 1)) / G >= nrows) return;
    const int64_t r = tid / G;
    const int q = (int)(tid - r * G);
    constexpr int NC = POT ? 7 : 6;
    double v[NC];
    split_group_sum<NC>(a.partial, nrows * 8, 8, r, r < nrows, nsplit, q, G, v);
    if (q == 0 && r < nrows) {
        double w[8];
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = v[c];
        jerk_finish(a, r, w, POT);
    }
}

hipError_t launch_jerk_reduce(const JerkLaunch &a, hipStream_t s)
{
    if (a.nrows <= 0 || a.j_split <= 1) return hipSuccess;
    const int64_t threads = a.nrows * split_group(a.j_split);
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (a.pot) hipLaunchKernelGGL(k_jerk_reduce<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_jerk_reduce<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

int jerk_blocks_per_cu(int prec, int ipl, int pot, int js, int block)
{
    const void *fn = nullptr;
    auto pick = [&](auto prec_c, auto pot_c) {
        constexpr int P = decltype(prec_c)::value;
        constexpr bool O = decltype(pot_c)::value;
        if (ipl == 1) fn = js ? (const void *)&k_jerk<P, 1, O, 1> : (const void *)&k_jerk<P, 1, O, 0>;
        else if (ipl == 2) fn = js ? (const void *)&k_jerk<P, 2, O, 1> : (const void *)&k_jerk<P, 2, O, 0>;
    };
    auto by_pot = [&](auto prec_c) {
        if (pot) pick(prec_c, std::true_type{});
        else pick(prec_c, std::false_type{});
    };
    switch (prec) {
    case P_FP64: by_pot(std::integral_constant<int, P_FP64>{}); break;
    case P_KAHAN: by_pot(std::integral_constant<int, P_KAHAN>{}); break;
    case P_FP64ACC: by_pot(std::integral_constant<int, P_FP64ACC>{}); break;
    default: break;
    }
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0) != hipSuccess) return 0;
    return nb;
}

// ------------------------------------------------------ Hermite corrector ----
// h divides t (both are dyadic: dt_max is a power of two), tested exactly
__device__ __forceinline__ bool divides(double h, double t)
{
    const double q = t / h;
    return __builtin_floor(q) == q;
}

// The block step for a particle at time t: the largest dt_max / 2^k not
// above the criterion value dts, at most twice the previous step (h_old > 0)
// and dividing t.
__device__ double quantised_step(double dts, double dt_max, double t, double h_old)
{
    double h = dt_max;
    int k = 0;
    while (h > dts && k < 60) {
        h *= 0.5;
        ++k;
    }
    if (h_old > 0.0 && h > 2.0 * h_old) h = 2.0 * h_old;
    while (!divides(h, t) && k < 60) {
        h *= 0.5;
        ++k;
    }
    return h;
}

__device__ __forceinline__ double norm3(const double *v)
{
    return __builtin_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// For each active row (particle i = rows[r], or r): the corrector over its
// step h (recomputing the prediction the pack kernel made), then the new
// acceleration and jerk are stored; in block mode the particle's time moves
// to t_next and its next step follows from Aarseth's criterion:
//   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2,  a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3
//   x1 = xp + a2 h^4/24 + a3 h^5/120,  v1 = vp + a2 h^3/6 + a3 h^4/24
//   dt* = sqrt(eta (|a1| |a2 + a3 h| + |j1|^2) / (|j1| |a3| + |a2 + a3 h|^2))
__global__ __launch_bounds__(256) void k_hermite_correct(HermiteLaunch a)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nrows = dev_rows(a.nrows, a.nrows_dev);
    // with the split partials: first their fixed-order sum, split_group lanes a row
    const int64_t nsplit = a.partial ? dev_split(a.split_max, a.split_dev, a.partial_rows, nrows) : 1;
    const int G = nsplit > 1 ? split_group(nsplit) : 1;
    if ((tid & ~int64_t(kWave - 1)) / G >= nrows) return;
    const int64_t r = tid / G;
    const int q = (int)(tid - r * G);
    // the particle's state first (every lane of the group loads the same
    // addresses), so that its loads overlap the split sum's
    const int64_t i = r < nrows ? (a.rows ? a.rows[r] : r) : 0;
    const double h = a.dt_i ? a.dt_i[i] : a.h;
    double x0[3], v0[3], a0[3], j0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x0[c] = a.pos[3 * i + c];
        v0[c] = a.vel[3 * i + c];
        a0[c] = a.acc[3 * i + c];
        j0[c] = a.jerk[3 * i + c];
    }
    double a1[3], j1[3];
    if (nsplit > 1) {
        double v[6];
        split_group_sum<6>(a.partial, nrows * 8, 8, r, r < nrows, nsplit, q, G, v);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a1[c] = a.Gc * v[c];
            j1[c] = a.Gc * v[3 + c];
        }
    }
    if (q != 0 || r >= nrows) return;
    if (nsplit <= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a1[c] = a.a1[3 * r + c];
            j1[c] = a.j1[3 * r + c];
        }
    double xp[3], vp[3], a2[3], a3[3];
    predict(x0, v0, a0, j0, h, xp, vp);
    const double h2 = h * h, h3 = h2 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double da = a0[c] - a1[c];
        const double s2 = (-6.0 * da - h * (4.0 * j0[c] + 2.0 * j1[c])) / h2;
        const double s3 = (12.0 * da + 6.0 * h * (j0[c] + j1[c])) / h3;
        a.pos[3 * i + c] = xp[c] + h2 * h2 * (s2 / 24.0 + h * s3 / 120.0);
        a.vel[3 * i + c] = vp[c] + h3 * (s2 / 6.0 + h * s3 / 24.0);
        a.acc[3 * i + c] = a1[c];
        a.jerk[3 * i + c] = j1[c];
        a2[c] = s2 + s3 * h;
        a3[c] = s3;
    }
    if (a.dt_i) {
        const double t = *a.t_next;
        const double na1 = norm3(a1), nj1 = norm3(j1), na2 = norm3(a2), na3 = norm3(a3);
        const double den = nj1 * na3 + na2 * na2;
        const double dts = den > 0.0 ? __builtin_sqrt(a.eta * (na1 * na2 + nj1 * nj1) / den) : a.dt_max;
        a.t_i[i] = t;
        a.dt_i[i] = quantised_step(dts, a.dt_max, t, h);
    }
}

hipError_t launch_hermite_correct(const HermiteLaunch &a, hipStream_t s)
{
    if (a.nrows <= 0) return hipSuccess;
    if (!a.pos || !a.vel || !a.acc || !a.jerk || !a.a1 || !a.j1 || (a.dt_i && (!a.t_i || !a.t_next)))
        return hipErrorInvalidValue;
    const int64_t threads = a.partial ? a.grid_threads : a.nrows;
    hipLaunchKernelGGL(k_hermite_correct, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Initial block steps: t_i = 0, dt_i from eta_s |a| / |jerk| quantised at t = 0.
__global__ __launch_bounds__(256) void k_block_init(const double *acc, const double *jerk, int64_t n,
                                                    double eta_s, double dt_max, double *t_i, double *dt_i)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nj = norm3(jerk + 3 * i);
    const double dts = nj > 0.0 ? eta_s * norm3(acc + 3 * i) / nj : dt_max;
    t_i[i] = 0.0;
    dt_i[i] = quantised_step(dts, dt_max, 0.0, 0.0);
}

hipError_t launch_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                             double dt_max, double *t_i, double *dt_i, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, jerk, n,
                       eta_s, dt_max, t_i, dt_i);
    return hipGetLastError();
}

// ------------------------------------------------------ block scheduling ----
// Each of the nb scheduling blocks owns the contiguous particle range
// [b chunk, (b + 1) chunk).  Three launches, no atomics, so the active list
// is in increasing particle order:
//   k_sched_min    per-block minimum of t_i + dt_i
//   k_sched_count  the global minimum t_next (every block reduces the nb
//                  partials itself) and the per-block number of due particles
//   k_sched_write  each block writes its due particles, in order, after the
//                  due particles of the blocks before it; the last block
//                  stores the total
constexpr int kSchedThreads = 256;

__device__ double block_min(double v, double *sm)
{
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = kSchedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = __builtin_fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sm[0];
    __syncthreads();
    return r;
}

__device__ int64_t block_sum(int64_t v, int64_t *sm)
{
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = kSchedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    const int64_t r = sm[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kSchedThreads) void k_sched_min(SchedLaunch a)
{
    __shared__ double sm[kSchedThreads];
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t b1 = b0 + a.chunk < a.n ? b0 + a.chunk : a.n;
    double m = __builtin_inf();
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kSchedThreads) m = __builtin_fmin(m, a.t_i[i] + a.dt_i[i]);
    m = block_min(m, sm);
    if (threadIdx.x == 0) a.part_min[blockIdx.x] = m;
}

__global__ __launch_bounds__(kSchedThreads) void k_sched_count(SchedLaunch a)
{
    __shared__ double sm[kSchedThreads];
    __shared__ int64_t sc[kSchedThreads];
    double m = __builtin_inf();
    for (int k = threadIdx.x; k < a.nb; k += kSchedThreads) m = __builtin_fmin(m, a.part_min[k]);
    const double t = block_min(m, sm);
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t b1 = b0 + a.chunk < a.n ? b0 + a.chunk : a.n;
    int64_t c = 0;
    if (t <= a.t_end)        // past t_end nothing is due: the block step is a no-op
        for (int64_t i = b0 + threadIdx.x; i < b1; i += kSchedThreads) c += (a.t_i[i] + a.dt_i[i] == t) ? 1 : 0;
    c = block_sum(c, sc);
    if (threadIdx.x == 0) {
        a.part_cnt[blockIdx.x] = c;
        if (blockIdx.x == 0) a.state->t = t;
    }
}

template <typename T, bool PACK>
__global__ __launch_bounds__(kSchedThreads) void k_sched_write(SchedLaunch a)
{
    __shared__ int64_t sc[kSchedThreads];
    __shared__ int64_t flag[kSchedThreads];
    const double t = a.state->t;
    const bool live = t <= a.t_end;
    int64_t before = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kSchedThreads) before += a.part_cnt[k];
    int64_t base = block_sum(before, sc);
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t b1 = b0 + a.chunk < a.n ? b0 + a.chunk : a.n;
    for (int64_t g = b0; g < b1; g += kSchedThreads) {
        const int64_t i = g + threadIdx.x;
        const int64_t f = (live && i < b1 && a.t_i[i] + a.dt_i[i] == t) ? 1 : 0;
        // inclusive scan of the flags (Hillis-Steele over the block)
        flag[threadIdx.x] = f;
        __syncthreads();
        for (int s = 1; s < kSchedThreads; s <<= 1) {
            const int64_t add = (int)threadIdx.x >= s ? flag[threadIdx.x - s] : 0;
            __syncthreads();
            flag[threadIdx.x] += add;
            __syncthreads();
        }
        if (f) a.list[base + flag[threadIdx.x] - 1] = i;
        base += flag[kSchedThreads - 1];
        __syncthreads();
    }
    if (PACK && live) {
        // the records of this block's particles predicted to t (and the padding)
        for (int64_t i = b0 + threadIdx.x; i < b1; i += kSchedThreads) pack_record<T>(a.pack, i);
        if (blockIdx.x == gridDim.x - 1)
            for (int64_t i = a.n + threadIdx.x; i < a.pack.npad; i += kSchedThreads) pack_record<T>(a.pack, i);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        int64_t split = 1;
        if (a.split_table && a.table_len > 0 && base > 0) {
            int64_t rw = (base + a.rows_per_wave - 1) / a.rows_per_wave;
            rw = rw < a.table_len ? rw : a.table_len;
            split = a.split_table[rw - 1];
        }
        a.state->count = base;
        a.state->split = split;
        if (a.count_log) {
            a.count_log[a.log_index] = base;
            a.time_log[a.log_index] = t;
        }
    }
}

hipError_t launch_schedule(const SchedLaunch &a, hipStream_t s)
{
    if (a.n <= 0 || a.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sched_min, dim3((unsigned)a.nb), dim3(kSchedThreads), 0, s, a);
    hipLaunchKernelGGL(k_sched_count, dim3((unsigned)a.nb), dim3(kSchedThreads), 0, s, a);
    if (!a.fuse_pack)
        hipLaunchKernelGGL((k_sched_write<double, false>), dim3((unsigned)a.nb), dim3(kSchedThreads), 0, s, a);
    else if (a.pack.prec != P_FP64)
        hipLaunchKernelGGL((k_sched_write<float, true>), dim3((unsigned)a.nb), dim3(kSchedThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_sched_write<double, true>), dim3((unsigned)a.nb), dim3(kSchedThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace nbk
