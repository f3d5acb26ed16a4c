// Adjoint (backward) all-pairs kernels.  Not in the paper: the derivative of
// the same pair laws, evaluated with the same tiled, SGPR-streamed j loop as
// the forward kernels.
//
// Gravity (Eq. 1), g_i = dL/da_i, d = r_j - r_k, s^2 = |d|^2 + eps^2:
//   dL/dr_k = G sum_{j!=k} [ w / s^3 - 3 (d.w) d / s^5 ],   w = m_k g_j - m_j g_k
// LJC(linear) with F_i = sum_j w(r) d_ij,
//   w = -x (C x + 24 e s6 (2 s6 - 1)),   x = 1/r^2, C = qs_i qs_j, e = se_i se_j,
//   s6 = (sigma_ij^2 x)^3,
//   w'/r = x^2 (4 C x + 24 e s6 (28 s6 - 8)),
//   u = g_j - g_k, du = d.u:
//   dL/dr_k     = sum_j [ w u + (w'/r) du d ]
//   dL/dq_k     = sqrt(2k/D) sum_j qs_j x^2 du
//   dL/dsigma_k = 72 sum_j e s6 (4 s6 - 1) x du / sigma_kj
//   dL/deps_k   = (12 / se_k) sum_j se_j s6 (2 s6 - 1) x du
#include <type_traits>

#include "allpairs.h"
#include "kernels.h"
#include "adjoint.h"

namespace nbk {

template <typename T> struct alignas(4 * sizeof(T)) LjcAdjRec {
    T x, y, z, qs, sh, se, gx, gy, gz, p0, p1, p2, p3, p4, p5, p6;   // padded to 16 values
};

// ------------------------------------------------------------------- pack ----
template <typename T>
__device__ __forceinline__ void adj_put(GravAdjRec<T> *rec, int64_t i, const double *x,
                                        const double *par, const double *g, double)
{
    GravAdjRec<T> r;
    r.x = (T)x[0];
    r.y = (T)x[1];
    r.z = (T)x[2];
    r.m = (T)par[0];
    r.gx = (T)g[0];
    r.gy = (T)g[1];
    r.gz = (T)g[2];
    r.p0 = T(0);
    rec[i] = r;
}
template <typename T>
__device__ __forceinline__ void adj_put(LjcAdjRec<T> *rec, int64_t i, const double *x,
                                        const double *par, const double *g, double qscale)
{
    LjcAdjRec<T> r;
    r.x = (T)x[0];
    r.y = (T)x[1];
    r.z = (T)x[2];
    r.qs = (T)(par[0] * qscale);
    r.sh = (T)(0.5 * par[1]);
    r.se = (T)__builtin_sqrt(24.0 * par[2]);     // se_i se_j = 24 eps_ij, as the forward records
    r.gx = (T)g[0];
    r.gy = (T)g[1];
    r.gz = (T)g[2];
    r.p0 = r.p1 = r.p2 = r.p3 = r.p4 = r.p5 = r.p6 = T(0);
    rec[i] = r;
}
template <typename T> __device__ __forceinline__ void adj_pad(GravAdjRec<T> *rec, int64_t i)
{
    GravAdjRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.m = r.gx = r.gy = r.gz = r.p0 = T(0);
    rec[i] = r;
}
template <typename T> __device__ __forceinline__ void adj_pad(LjcAdjRec<T> *rec, int64_t i)
{
    LjcAdjRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.qs = r.sh = r.se = r.gx = r.gy = r.gz = T(0);
    r.p0 = r.p1 = r.p2 = r.p3 = r.p4 = r.p5 = r.p6 = T(0);
    rec[i] = r;
}

template <typename R, int P>
__global__ __launch_bounds__(256) void k_pack_adj(AdjPackLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.npad) return;
    R *rec = (R *)a.rec;
    if (i < a.n) adj_put(rec, i, a.pos + 3 * i, a.params + (int64_t)P * i, a.g + 3 * i, a.qscale);
    else adj_pad(rec, i);
}

hipError_t launch_pack_adjoint(const AdjPackLaunch &p, hipStream_t s)
{
    if (p.npad <= 0) return hipSuccess;
    const dim3 grid((unsigned)((p.npad + 255) / 256)), block(256);
    const bool f32 = p.prec != P_FP64;
    if (p.law == GRAVITY) {
        if (f32) hipLaunchKernelGGL((k_pack_adj<GravAdjRec<float>, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_adj<GravAdjRec<double>, 1>), grid, block, 0, s, p);
    } else {
        if (f32) hipLaunchKernelGGL((k_pack_adj<LjcAdjRec<float>, 3>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_adj<LjcAdjRec<double>, 3>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- pair math ----
// Gravity adjoint, per pair: 3 sub, 3 fma, 1 rsq, 4 mul, 3 mul + 3 fma (w),
// 1 mul + 2 fma (d.w), 1 mul, 6 fma: 41 flops (multiply-add = 2).
template <bool MASK, typename T>
__device__ __forceinline__ void grav_adj_pair(const GravAdjRec<T> &i, const GravAdjRec<T> &j, T eps2,
                                              bool self, T (&o)[8])
{
    const T dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
    T r2 = fma_(dx, dx, eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    if (MASK) r2 = self ? T(1) : r2;
    T ri = rsqrt_(r2);
    if (MASK) ri = self ? T(0) : ri;
    const T ri2 = ri * ri;
    const T ri3 = ri2 * ri;
    const T wx = fma_(-j.m, i.gx, i.m * j.gx);
    const T wy = fma_(-j.m, i.gy, i.m * j.gy);
    const T wz = fma_(-j.m, i.gz, i.m * j.gz);
    T dw = dx * wx;
    dw = fma_(dy, wy, dw);
    dw = fma_(dz, wz, dw);
    // K(d) w = s^-3 (w - 3 s^-2 (d.w) d)
    const T u = (ri2 * T(3)) * dw;
    o[0] = fma_(ri3, fma_(-u, dx, wx), o[0]);
    o[1] = fma_(ri3, fma_(-u, dy, wy), o[1]);
    o[2] = fma_(ri3, fma_(-u, dz, wz), o[2]);
}

// LJC adjoint, per pair (position and parameter adjoints together).
template <bool MASK, typename T>
__device__ __forceinline__ void ljc_adj_pair(const LjcAdjRec<T> &i, const LjcAdjRec<T> &j, T,
                                             bool self, T (&o)[8])
{
    const T dx = j.x - i.x, dy = j.y - i.y, dz = j.z - i.z;
    T r2 = dx * dx;
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    T qq = i.qs * j.qs;
    T e = i.se * j.se;
    if (MASK) {
        r2 = self ? T(1) : r2;
        qq = self ? T(0) : qq;
        e = self ? T(0) : e;
    }
    const T x = rcp_(r2);
    const T sg = i.sh + j.sh;
    const T sgx = sg * x;
    const T s2 = sg * sgx;                                         // (sigma_ij / r)^2
    const T s4 = s2 * s2;
    const T s6 = s4 * s2;
    const T lj = e * s6;                                           // 24 eps_ij s^6
    const T t = fma_(s6, T(2), T(-1));
    const T cx = qq * x;
    const T W = fma_(lj, t, cx) * x;                               // w = -W
    const T x2 = x * x;
    const T wpr = fma_(lj, fma_(s6, T(28), T(-8)), cx * T(4)) * x2;
    const T ux = j.gx - i.gx, uy = j.gy - i.gy, uz = j.gz - i.gz;
    T du = dx * ux;
    du = fma_(dy, uy, du);
    du = fma_(dz, uz, du);
    // a masked pair must contribute nothing: its qq and e are zeroed above, and
    // d.u is zeroed here because the charge and epsilon terms below do not
    // carry qq or e (for the self pair d = 0 anyway; an excluded pair has d != 0)
    if (MASK) du = self ? T(0) : du;
    const T tt = wpr * du;
    o[0] = fma_(-W, ux, o[0]);
    o[1] = fma_(-W, uy, o[1]);
    o[2] = fma_(-W, uz, o[2]);
    o[0] = fma_(tt, dx, o[0]);
    o[1] = fma_(tt, dy, o[1]);
    o[2] = fma_(tt, dz, o[2]);
    const T xdu = x * du;
    o[3] = fma_(j.qs, x * xdu, o[3]);
    // 24 eps_ij s^6 / sigma_ij = e s^4 (sigma_ij / r^2): no reciprocal of sigma
    o[4] = fma_((e * (s4 * sgx)) * fma_(s6, T(4), T(-1)), xdu, o[4]);
    o[5] = fma_(j.se, s6 * t * xdu, o[5]);
}

template <bool MASK, typename T>
__device__ __forceinline__ void adj_pair(const GravAdjRec<T> &i, const GravAdjRec<T> &j, T eps2,
                                         bool self, T (&o)[8])
{
    grav_adj_pair<MASK>(i, j, eps2, self, o);
}
template <bool MASK, typename T>
__device__ __forceinline__ void adj_pair(const LjcAdjRec<T> &i, const LjcAdjRec<T> &j, T eps2,
                                         bool self, T (&o)[8])
{
    ljc_adj_pair<MASK>(i, j, eps2, self, o);
}

// The pair operation of the adjoint kernels for the shared j loop.
template <int LAW> struct AdjOp {
    static constexpr int NC = LAW == GRAVITY ? 3 : 6;
    static constexpr int NP = 8;
    template <bool MASK, typename R, typename T>
    static __device__ __forceinline__ void run(const R &i, const R &j, const PairK<T> &k, bool self,
                                               T (&o)[NP])
    {
        adj_pair<MASK>(i, j, k.eps2, self, o);
    }
};

template <typename T> __device__ __forceinline__ void settle(const GravAdjRec<T> &s)
{
    asm volatile("" ::"v"(s.x), "v"(s.y), "v"(s.z), "v"(s.m), "v"(s.gx), "v"(s.gy), "v"(s.gz));
}
template <typename T> __device__ __forceinline__ void settle(const LjcAdjRec<T> &s)
{
    asm volatile("" ::"v"(s.x), "v"(s.y), "v"(s.z), "v"(s.qs), "v"(s.sh), "v"(s.se), "v"(s.gx),
                 "v"(s.gy), "v"(s.gz));
}

__device__ __forceinline__ void adj_finish(const AdjLaunch &a, int law, int64_t k, const double *v)
{
    if (law == GRAVITY) {
        if (a.grad_pos) {
            a.grad_pos[3 * k] = a.G * v[0];
            a.grad_pos[3 * k + 1] = a.G * v[1];
            a.grad_pos[3 * k + 2] = a.G * v[2];
        }
        return;
    }
    if (a.grad_pos) {
        a.grad_pos[3 * k] = v[0];
        a.grad_pos[3 * k + 1] = v[1];
        a.grad_pos[3 * k + 2] = v[2];
    }
    if (a.grad_params) {
        // the sums carry the records' factor 24 in eps (v[4]) and sqrt(24) in se_j (v[5])
        const double se_k = __builtin_sqrt(24.0 * a.params[3 * k + 2]);
        a.grad_params[3 * k] = a.qscale * v[3];
        a.grad_params[3 * k + 1] = 3.0 * v[4];
        a.grad_params[3 * k + 2] = (12.0 / se_k) * v[5];
    }
}

template <int LAW, int PREC>
using AdjRecOf = typename std::conditional<LAW == GRAVITY, GravAdjRec<typename RealOf<PREC>::type>,
                                           LjcAdjRec<typename RealOf<PREC>::type>>::type;

// One wave's rows against its j split (EX: with exclusion lists, LDS staging only).
template <int LAW, int PREC, int I, int JS, bool EX>
__device__ __forceinline__ void adjoint_body(const AdjRecOf<LAW, PREC> *__restrict__ rec, const AdjLaunch &a)
{
    using T = typename RealOf<PREC>::type;
    using R = typename std::conditional<LAW == GRAVITY, GravAdjRec<T>, LjcAdjRec<T>>::type;
    using Op = AdjOp<LAW>;
    constexpr int NC = Op::NC;
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rbase = wave * (int64_t)(kWave * I);
    if (rbase >= a.n) return;
    const int64_t jb = (int64_t)blockIdx.y * a.split_len;
    const int64_t je = (jb + a.split_len < a.npad) ? jb + a.split_len : a.npad;

    R is[I];
    int64_t pid[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
        int64_t r = rbase + lane + (int64_t)kWave * k;
        pid[k] = r < a.n ? r : a.n - 1;
        is[k] = rec[pid[k]];
    }
    RunSum<PREC> acc[I][NC];
    T p[I][Op::NP];
    __shared__ R lds_j[JS ? 4 : 1][2][kWave];
    R(*wl)[kWave] = lds_j[JS ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    PairK<T> kc{};
    kc.eps2 = (T)a.eps2;
    if constexpr (EX) {
        static_assert(JS == 1, "exclusion lists use the LDS staging");
        ExclMask<I> mask;
#pragma unroll
        for (int k = 0; k < I; ++k) mask.pid[k] = pid[k];
        mask.init(a.excl, pid, 0);
        j_range_masked<JS, Op, PREC, I>(rec, jb, je, a.j_tile, is, mask, kc, acc, p, wl);
    } else {
        j_range<JS, Op, PREC, I>(rec, jb, je, a.j_tile, is, pid, kc, acc, p, wl);
    }
#pragma unroll
    for (int k = 0; k < I; ++k) {
        const int64_t r = rbase + lane + (int64_t)kWave * k;
        if (r >= a.n) continue;
        double v[8];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = acc[k][c].value();
        if (a.j_split > 1) {
            double *o = a.partial + ((int64_t)blockIdx.y * a.n + r) * 8;
#pragma unroll
            for (int c = 0; c < NC; ++c) o[c] = v[c];
        } else {
            adj_finish(a, LAW, r, v);
        }
    }
}

template <int LAW, int PREC, int I, int JS>
__global__ __launch_bounds__(256) void k_adjoint(const AdjRecOf<LAW, PREC> *__restrict__ rec, AdjLaunch a)
{
    adjoint_body<LAW, PREC, I, JS, false>(rec, a);
}

template <int PREC, int I>
__global__ __launch_bounds__(256) void k_adjoint_excl(const AdjRecOf<LJC, PREC> *__restrict__ rec, AdjLaunch a)
{
    adjoint_body<LJC, PREC, I, 1, true>(rec, a);
}

template <int LAW, int PREC, int I>
static void launch_adj_one(const AdjLaunch &a, dim3 grid, hipStream_t s)
{
    using T = typename RealOf<PREC>::type;
    using R = typename std::conditional<LAW == GRAVITY, GravAdjRec<T>, LjcAdjRec<T>>::type;
    if (a.excl.off) {
        if constexpr (LAW == LJC && I <= 2)
            hipLaunchKernelGGL((k_adjoint_excl<PREC, I>), grid, dim3(a.block), 0, s, (const R *)a.rec, a);
        return;
    }
    if (a.j_stage == 1)
        hipLaunchKernelGGL((k_adjoint<LAW, PREC, I, 1>), grid, dim3(a.block), 0, s, (const R *)a.rec, a);
    else
        hipLaunchKernelGGL((k_adjoint<LAW, PREC, I, 0>), grid, dim3(a.block), 0, s, (const R *)a.rec, a);
}

template <int LAW, int PREC>
static bool adj_ipl(const AdjLaunch &a, dim3 grid, hipStream_t s)
{
    switch (a.ipl) {
    case 1: launch_adj_one<LAW, PREC, 1>(a, grid, s); return true;
    case 2: launch_adj_one<LAW, PREC, 2>(a, grid, s); return true;
    case 4: launch_adj_one<LAW, PREC, 4>(a, grid, s); return true;
    default: return false;
    }
}

template <int LAW>
static bool adj_prec(const AdjLaunch &a, dim3 grid, hipStream_t s)
{
    switch (a.prec) {
    case P_FP64: return adj_ipl<LAW, P_FP64>(a, grid, s);
    case P_KAHAN: return adj_ipl<LAW, P_KAHAN>(a, grid, s);
    case P_FP64ACC: return adj_ipl<LAW, P_FP64ACC>(a, grid, s);
    default: return false;
    }
}

hipError_t launch_adjoint(const AdjLaunch &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (a.excl.off && (a.law != LJC || a.ipl > 2)) return hipErrorInvalidValue;
    const int64_t waves = (a.n + (int64_t)kWave * a.ipl - 1) / ((int64_t)kWave * a.ipl);
    const int64_t wpb = a.block / kWave;
    const dim3 grid((unsigned)((waves + wpb - 1) / wpb), (unsigned)a.j_split);
    const bool ok = a.law == GRAVITY ? adj_prec<GRAVITY>(a, grid, s) : adj_prec<LJC>(a, grid, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// Fixed-order sum of the j-split partials, split_group(j_split) lanes per row
// (NC = 3 sums for gravity, 6 for LJC).
template <int NC>
__global__ __launch_bounds__(256) void k_adj_reduce(AdjLaunch a)
{
    const int G = split_group(a.j_split);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((tid & ~int64_t(kWave - 1)) / G >= a.n) return;     // the whole wave is past the rows
    const int64_t r = tid / G;
    const int q = (int)(tid - r * G);
    double v[NC];
    split_group_sum<NC>(a.partial, a.n * 8, 8, r, r < a.n, a.j_split, q, G, v);
    if (q == 0 && r < a.n) {
        double out[8];
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] = v[c];
        adj_finish(a, NC == 3 ? (int)GRAVITY : a.law, r, out);
    }
}

hipError_t launch_adjoint_reduce(const AdjLaunch &a, hipStream_t s)
{
    if (a.n <= 0 || a.j_split <= 1) return hipSuccess;
    const int64_t threads = a.n * split_group(a.j_split);
    const dim3 grid((unsigned)((threads + 255) / 256));
    if (a.law == GRAVITY) hipLaunchKernelGGL(k_adj_reduce<3>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_adj_reduce<6>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ----------------------------------------------------------- batched adjoint ----
// Many independent systems in one persistent launch, as the batched forward:
// (system, row-block) units in decreasing order of cost, pulled with an
// integer ticket; each unit runs the adjoint j loop over its own system's
// records (padded per system) and writes its rows' adjoints.
template <typename R, int P>
__global__ __launch_bounds__(256) void k_pack_adj_batched(AdjBatchLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.ticket_zeroed && i < 64) a.ticket[i] = 0;     // the work ticket of the launch that follows
    if (i >= a.npad_total) return;
    int64_t lo = 0, hi = a.n_systems;          // poff[lo] <= i < poff[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.poff[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int64_t l = i - a.poff[lo];
    R *rec = (R *)a.rec;
    if (l < a.off[lo + 1] - a.off[lo]) {
        const int64_t src = a.off[lo] + l;
        adj_put(rec, i, a.pos + 3 * src, a.params + (int64_t)P * src, a.g + 3 * src, a.qscale);
    } else {
        adj_pad(rec, i);
    }
}

hipError_t launch_pack_adjoint_batched(const AdjBatchLaunch &p, hipStream_t s)
{
    if (p.npad_total <= 0 || p.n_systems <= 0) return hipSuccess;
    const dim3 grid((unsigned)((p.npad_total + 255) / 256)), block(256);
    const bool f32 = p.prec != P_FP64;
    if (p.law == GRAVITY) {
        if (f32) hipLaunchKernelGGL((k_pack_adj_batched<GravAdjRec<float>, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_adj_batched<GravAdjRec<double>, 1>), grid, block, 0, s, p);
    } else {
        if (f32) hipLaunchKernelGGL((k_pack_adj_batched<LjcAdjRec<float>, 3>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_adj_batched<LjcAdjRec<double>, 3>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

__device__ __forceinline__ void adj_finish_b(const AdjBatchLaunch &a, int law, int64_t k, const double *v)
{
    AdjLaunch t{};
    t.G = a.G;
    t.qscale = a.qscale;
    t.grad_pos = a.grad_pos;
    t.grad_params = a.grad_params;
    t.params = a.params;
    adj_finish(t, law, k, v);
}

template <int LAW, int PREC, int I, int JS, bool EX>
__global__ __launch_bounds__(256) void k_adjoint_batched(const AdjRecOf<LAW, PREC> *__restrict__ rec,
                                                         AdjBatchLaunch a)
{
    using T = typename RealOf<PREC>::type;
    using R = AdjRecOf<LAW, PREC>;
    using Op = AdjOp<LAW>;
    constexpr int NC = Op::NC;
    const int lane = lane_id();
    __shared__ R lds_j[JS ? 4 : 1][2][kWave];
    R(*wl)[kWave] = lds_j[JS ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    PairK<T> kc{};
    kc.eps2 = (T)a.eps2;
    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(a.ticket, 1);
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= a.n_units) break;      // every wave leaves once the list is drained
        const int s = a.units[4 * (int64_t)u];
        if (s < 0 || (int64_t)s >= a.n_systems) continue;   // never index outside the tables
        const int64_t rb = a.units[4 * (int64_t)u + 1];
        const int64_t part = a.units[4 * (int64_t)u + 2];
        const int64_t o = a.off[s], ns = a.off[s + 1] - o;
        const int64_t po = a.poff[s], pe = a.poff[s + 1];
        const int64_t nparts = a.systab[3 * (int64_t)s], plen = a.systab[3 * (int64_t)s + 1];
        const int64_t jb = po + part * plen;
        const int64_t je = jb + plen < pe ? jb + plen : pe;
        const int64_t lbase = rb * (int64_t)(kWave * I);
        R is[I];
        int64_t pid[I], gid[I];
#pragma unroll
        for (int k = 0; k < I; ++k) {
            int64_t l = lbase + lane + (int64_t)kWave * k;
            l = l < ns ? l : ns - 1;
            pid[k] = po + l;
            gid[k] = o + l;
            is[k] = rec[pid[k]];
        }
        RunSum<PREC> acc[I][NC];
        T p[I][Op::NP];
        if constexpr (EX) {
            static_assert(JS == 1, "exclusion lists use the LDS staging");
            ExclMask<I> mask;
#pragma unroll
            for (int k = 0; k < I; ++k) mask.pid[k] = pid[k];
            mask.init(a.excl, gid, po - o);
            j_range_masked<JS, Op, PREC, I>(rec, jb, je, a.j_tile, is, mask, kc, acc, p, wl);
        } else {
            j_range<JS, Op, PREC, I>(rec, jb, je, a.j_tile, is, pid, kc, acc, p, wl);
        }
        const int64_t slot = a.systab[3 * (int64_t)s + 2] + rb * nparts + part;
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const int64_t l = lbase + lane + (int64_t)kWave * k;
            if (l >= ns) continue;
            double v[8];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = acc[k][c].value();
            if (nparts > 1) {            // partial sums of this part, added by the reduction
                double *q = a.partial + (slot * (kWave * I) + lane + kWave * k) * 8;
#pragma unroll
                for (int c = 0; c < NC; ++c) q[c] = v[c];
                continue;
            }
            adj_finish_b(a, LAW, o + l, v);
        }
    }
}

template <int LAW, int PREC, int I>
static bool adjb_one(const AdjBatchLaunch &a, hipStream_t s, const void **fn)
{
    using R = AdjRecOf<LAW, PREC>;
    const dim3 grid((unsigned)a.grid), block((unsigned)a.block);
    if (a.excl.off) {
        if constexpr (LAW == LJC) {
            if (fn) *fn = (const void *)&k_adjoint_batched<LAW, PREC, I, 1, true>;
            else hipLaunchKernelGGL((k_adjoint_batched<LAW, PREC, I, 1, true>), grid, block, 0, s, (const R *)a.rec, a);
            return true;
        }
        return false;
    }
    if (a.j_stage == 1) {
        if (fn) *fn = (const void *)&k_adjoint_batched<LAW, PREC, I, 1, false>;
        else hipLaunchKernelGGL((k_adjoint_batched<LAW, PREC, I, 1, false>), grid, block, 0, s, (const R *)a.rec, a);
    } else {
        if (fn) *fn = (const void *)&k_adjoint_batched<LAW, PREC, I, 0, false>;
        else hipLaunchKernelGGL((k_adjoint_batched<LAW, PREC, I, 0, false>), grid, block, 0, s, (const R *)a.rec, a);
    }
    return true;
}

template <int LAW, int PREC>
static bool adjb_ipl(const AdjBatchLaunch &a, hipStream_t s, const void **fn)
{
    switch (a.ipl) {
    case 1: return adjb_one<LAW, PREC, 1>(a, s, fn);
    case 2: return adjb_one<LAW, PREC, 2>(a, s, fn);
    default: return false;
    }
}

template <int LAW>
static bool adjb_prec(const AdjBatchLaunch &a, hipStream_t s, const void **fn)
{
    switch (a.prec) {
    case P_FP64: return adjb_ipl<LAW, P_FP64>(a, s, fn);
    case P_KAHAN: return adjb_ipl<LAW, P_KAHAN>(a, s, fn);
    case P_FP64ACC: return adjb_ipl<LAW, P_FP64ACC>(a, s, fn);
    default: return false;
    }
}

static bool adjb_dispatch(const AdjBatchLaunch &a, hipStream_t s, const void **fn)
{
    return a.law == GRAVITY ? adjb_prec<GRAVITY>(a, s, fn) : (a.law == LJC ? adjb_prec<LJC>(a, s, fn) : false);
}

// Row block red[blockIdx.x] of a system cut into several j parts: each thread adds its
// row's part sums in part order (NC = 3 sums for gravity, 6 for LJC).
template <int NC>
__global__ __launch_bounds__(128) void k_adjoint_batched_reduce(AdjBatchLaunch a)
{
    const int64_t s = a.red[2 * blockIdx.x], rb = a.red[2 * blockIdx.x + 1];
    const int64_t rows = (int64_t)kWave * a.ipl;
    const int64_t l = rb * rows + threadIdx.x;
    if (l >= a.off[s + 1] - a.off[s]) return;
    const int64_t nparts = a.systab[3 * s];
    const int64_t slot0 = a.systab[3 * s + 2] + rb * nparts;
    NSum v[NC];
    for (int64_t p = 0; p < nparts; ++p) {
        const double *q = a.partial + ((slot0 + p) * rows + threadIdx.x) * 8;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c].add(q[c]);
    }
    double out[8];
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = v[c].value();
    adj_finish_b(a, NC == 3 ? (int)GRAVITY : a.law, a.off[s] + l, out);
}

hipError_t launch_adjoint_batched(const AdjBatchLaunch &a, hipStream_t s)
{
    if (a.n_units <= 0) return hipSuccess;
    if (a.ipl < 1 || a.ipl > 2) return hipErrorInvalidValue;     // the reduction's 128-thread bound
    hipError_t e = a.ticket_zeroed ? hipSuccess : launch_fill_zero(a.ticket, 256, s);
    if (e != hipSuccess) return e;
    if (!adjb_dispatch(a, s, nullptr)) return hipErrorInvalidValue;
    e = hipGetLastError();
    if (e != hipSuccess || !a.any_parts || a.n_red <= 0) return e;
    const dim3 grid((unsigned)a.n_red), block((unsigned)(kWave * a.ipl));
    if (a.law == GRAVITY) hipLaunchKernelGGL(k_adjoint_batched_reduce<3>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_adjoint_batched_reduce<6>, grid, block, 0, s, a);
    return hipGetLastError();
}

int adjoint_batched_blocks_per_cu(const AdjBatchLaunch &a)
{
    const void *fn = nullptr;
    if (!adjb_dispatch(a, nullptr, &fn) || !fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, a.block, 0) != hipSuccess) return 0;
    return nb;
}

// ------------------------------------------------------ per-type reduction ----
// Per-type sums of the sigma and epsilon gradients (params columns 1 and 2) in
// two passes, each in a fixed order, so that the sums repeat bit for bit:
//   k_type_partial  block b owns the atoms [b chunk, (b + 1) chunk); for eight
//                   types at a time every lane sums its strided atoms
//                   (Neumaier; other types' atoms add an exact zero), the wave
//                   merges its lanes in a butterfly and thread 0 the waves in
//                   wave order, into partial[b][t][2];
//   k_type_final    a group of 64 lanes per type sums the nb partials
//                   (split_group_sum).
// Types outside [0, n_types) are not counted.
constexpr int kTypeGroup = 8;
constexpr int kTypeThreads = 256;

__global__ __launch_bounds__(kTypeThreads) void k_type_partial(const double *__restrict__ gp,
                                                               const int32_t *__restrict__ types, int64_t n,
                                                               int n_types, int64_t chunk,
                                                               double *__restrict__ partial)
{
    __shared__ double sm[kTypeThreads / kWave][kTypeGroup][2][2];   // [wave][type][column][s, c]
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    const int w = threadIdx.x >> 6;
    for (int tg = 0; tg < n_types; tg += kTypeGroup) {
        NSum acc[kTypeGroup][2];
        for (int64_t i = b0 + threadIdx.x; i < b1; i += kTypeThreads) {
            const int t = types[i] - tg;
            const double x1 = gp[3 * i + 1], x2 = gp[3 * i + 2];
#pragma unroll
            for (int k = 0; k < kTypeGroup; ++k) {
                acc[k][0].add(t == k ? x1 : 0.0);
                acc[k][1].add(t == k ? x2 : 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < kTypeGroup; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                for (int m = 1; m < kWave; m <<= 1) {
                    const double s2 = __shfl_xor(acc[k][c].s, m);
                    const double c2 = __shfl_xor(acc[k][c].c, m);
                    acc[k][c].merge(s2, c2);
                }
                if ((threadIdx.x & (kWave - 1)) == 0) {
                    sm[w][k][c][0] = acc[k][c].s;
                    sm[w][k][c][1] = acc[k][c].c;
                }
            }
        __syncthreads();
        if (threadIdx.x < 2 * kTypeGroup) {
            const int k = threadIdx.x >> 1, c = threadIdx.x & 1;
            NSum v;
            for (int ww = 0; ww < kTypeThreads / kWave; ++ww) v.merge(sm[ww][k][c][0], sm[ww][k][c][1]);
            if (tg + k < n_types) partial[((int64_t)blockIdx.x * n_types + tg + k) * 2 + c] = v.value();
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_type_final(const double *__restrict__ partial, int n_types,
                                                    int64_t nb, double *__restrict__ out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = tid >> 6;
    const int q = (int)(tid & (kWave - 1));
    if ((tid & ~int64_t(kWave - 1)) >> 6 >= n_types) return;
    double v[2];
    split_group_sum<2>(partial, (int64_t)n_types * 2, 2, t, t < n_types, nb, q, kWave, v);
    if (q == 0 && t < n_types) {
        out[2 * t] = v[0];
        out[2 * t + 1] = v[1];
    }
}

hipError_t launch_type_reduce(const double *grad_params, const int32_t *types, int64_t n,
                              int32_t n_types, double *out, double *partial, int64_t partial_doubles,
                              hipStream_t s)
{
    if (n_types <= 0) return hipSuccess;
    // blocks: about 2048 atoms each, at most 1024, and as many as the partial buffer holds
    int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + 2047) / 2048, 1024));
    nb = std::min<int64_t>(nb, partial_doubles / (2 * (int64_t)n_types));
    if (nb < 1) return hipErrorInvalidValue;
    const int64_t chunk = (std::max<int64_t>(n, 1) + nb - 1) / nb;
    hipLaunchKernelGGL(k_type_partial, dim3((unsigned)nb), dim3(kTypeThreads), 0, s, grad_params, types, n,
                       (int)n_types, chunk, partial);
    const int64_t threads = (int64_t)n_types * kWave;
    hipLaunchKernelGGL(k_type_final, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, partial,
                       (int)n_types, nb, out);
    return hipGetLastError();
}

}  // namespace nbk
