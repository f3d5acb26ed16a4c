// All-pairs force / potential kernels for one system (gfx950).
//
// Structure (Section 2's stream formulation: one output per i, the j loop
// inside; Section 3.3's i-unrolling; Section 3.4's replication of the i
// stream over disjoint j ranges):
//   pack          FP64 inputs -> padded records (FP32 or FP64), optionally
//                 after the kick-drift half of a leapfrog step;
//   k_forces      each wave owns 64*I output rows (I per lane, in VGPRs) and
//                 streams the records of its j range through SGPRs, tile by
//                 tile; FP32 tile partials are folded into FP64 / Kahan sums;
//   reduce_split  when the j range is split over several waves, the split
//                 partials are added in a fixed order (deterministic).
#include "allpairs.h"
#include "kernels.h"

namespace nbk {

// ------------------------------------------------------------------ pack ----
template <typename R, int P>
__global__ __launch_bounds__(256) void k_pack(PackLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.npad) return;
    R *rec = (R *)a.rec;
    if (i >= a.n) {
        store_pad(rec, i);
        return;
    }
    double x = a.pos[3 * i], y = a.pos[3 * i + 1], z = a.pos[3 * i + 2];
    if (a.kick_drift) {
        const double vx = a.vel[3 * i] + a.half_dt * a.acc[3 * i];
        const double vy = a.vel[3 * i + 1] + a.half_dt * a.acc[3 * i + 1];
        const double vz = a.vel[3 * i + 2] + a.half_dt * a.acc[3 * i + 2];
        x += a.dt * vx;
        y += a.dt * vy;
        z += a.dt * vz;
        a.vel[3 * i] = vx;
        a.vel[3 * i + 1] = vy;
        a.vel[3 * i + 2] = vz;
        a.pos[3 * i] = x;
        a.pos[3 * i + 1] = y;
        a.pos[3 * i + 2] = z;
    }
    store_rec(rec, i, x, y, z, a.params + (int64_t)P * i, a.qscale);
}

hipError_t launch_pack(const PackLaunch &p, hipStream_t s)
{
    if (p.npad <= 0) return hipSuccess;
    const dim3 grid((unsigned)((p.npad + 255) / 256)), block(256);
    const bool f32 = p.prec != P_FP64;
    if (p.law == GRAVITY) {
        if (f32) hipLaunchKernelGGL((k_pack<GravRec<float>, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack<GravRec<double>, 1>), grid, block, 0, s, p);
    } else {
        if (f32) hipLaunchKernelGGL((k_pack<LjcRec<float>, 3>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack<LjcRec<double>, 3>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- epilogue ----
__device__ __forceinline__ void finish_row(const Epilogue &e, int64_t r, double v0, double v1,
                                           double v2, double v3, bool pot)
{
    double f0 = e.fscale * v0, f1 = e.fscale * v1, f2 = e.fscale * v2;
    if (e.kick) {
        const double w = e.inv_mass ? e.inv_mass[r] : 1.0;
        f0 *= w;
        f1 *= w;
        f2 *= w;
        e.vel[3 * r] += e.half_dt * f0;
        e.vel[3 * r + 1] += e.half_dt * f1;
        e.vel[3 * r + 2] += e.half_dt * f2;
    }
    e.out_force[3 * r] = f0;
    e.out_force[3 * r + 1] = f1;
    e.out_force[3 * r + 2] = f2;
    if (pot && e.out_pot) e.out_pot[r] = e.pscale * v3;
}

// ------------------------------------------------------------- all pairs ----
// Block -> (row block, j part).  The dispatcher hands workgroups to the eight
// XCDs in turn (linear block id mod 8), each XCD with its own L2.  When the part
// count S is a multiple of 8, XCD x owns the S/8 parts x, x + 8, x + 16, ...,
// and takes them for one row block after another: its L2 then holds those
// parts' j segments (npad/8 records, 2 MiB at N = 2^20 in FP32, whatever S)
// and each row block's i records, so both are fetched from HBM about once per
// XCD.  Otherwise the grid is taken as (row block, part) directly.  Either way
// each (row block, part) pair is visited once, and the sums do not depend on
// the mapping.
constexpr int kXcds = 8;

__device__ __forceinline__ void block_tile(int64_t &rblock, int64_t &part)
{
    const int64_t gx = gridDim.x, gy = gridDim.y;
    if (gy % kXcds != 0) {
        rblock = blockIdx.x;
        part = blockIdx.y;
        return;
    }
    const int64_t L = (int64_t)blockIdx.y * gx + blockIdx.x;
    const int64_t k = L / kXcds, per_xcd = gy / kXcds;
    part = L % kXcds + kXcds * (k % per_xcd);
    rblock = k / per_xcd;
}

// One wave's rows against the j range of its split (EX: with exclusion lists,
// LDS staging only).
template <int LAW, int PREC, int I, bool POT, int JS, bool EX>
__device__ __forceinline__ void forces_body(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec, int64_t npad,
    int64_t nrows, const int64_t *__restrict__ rows, int64_t split_len, int j_tile,
    PairK<typename RealOf<PREC>::type> kc, double *__restrict__ partial, const Epilogue &epi,
    const ExclArgs &ex)
{
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    using IS = typename IStateOf<R>::type;
    constexpr int NC = POT ? 4 : 3;

    const int lane = lane_id();
    int64_t rblock, part;
    block_tile(rblock, part);
    const int64_t wave = rblock * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rbase = wave * (int64_t)(kWave * I);
    if (rbase >= nrows) return;
    const int64_t jb = part * split_len;
    const int64_t je = (jb + split_len < npad) ? jb + split_len : npad;

    IS is[I];
    int64_t pid[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
        int64_t r = rbase + lane + (int64_t)kWave * k;
        r = r < nrows ? r : nrows - 1;
        int64_t q = rows ? rows[r] : r;
        q = q < 0 ? 0 : (q < npad ? q : npad - 1);        // never read outside the records
        pid[k] = q;
        load_i(rec, pid[k], is[k]);
    }

    RunSum<PREC> acc[I][NC];
    T p[I][4];
#pragma unroll
    for (int k = 0; k < I; ++k) p[k][3] = T(0);

    __shared__ R lds_j[JS ? 4 : 1][2][kWave];
    R(*wl)[kWave] = lds_j[JS ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
    if constexpr (EX) {
        static_assert(JS == 1, "exclusion lists use the LDS staging");
        ExclMask<I> mask;
#pragma unroll
        for (int k = 0; k < I; ++k) mask.pid[k] = pid[k];
        mask.init(ex, pid, 0);
        j_range_masked<JS, ForceOp<POT, LAW>, PREC, I>(rec, jb, je, j_tile, is, mask, kc, acc, p, wl);
    } else {
        j_range<JS, ForceOp<POT, LAW>, PREC, I>(rec, jb, je, j_tile, is, pid, kc, acc, p, wl);
    }

#pragma unroll
    for (int k = 0; k < I; ++k) {
        const int64_t r = rbase + lane + (int64_t)kWave * k;
        if (r >= nrows) continue;
        const double v0 = acc[k][0].value(), v1 = acc[k][1].value(), v2 = acc[k][2].value();
        const double v3 = POT ? acc[k][NC - 1].value() : 0.0;
        if (partial) {
            double *o = partial + (part * nrows + r) * 4;
            o[0] = v0;
            o[1] = v1;
            o[2] = v2;
            o[3] = v3;
        } else {
            finish_row(epi, r, v0, v1, v2, v3, POT);
        }
    }
}

template <int LAW, int PREC, int I, bool POT, int JS>
__global__ __launch_bounds__(256) void k_forces(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec, int64_t npad,
    int64_t nrows, const int64_t *__restrict__ rows, int64_t split_len, int j_tile,
    PairK<typename RealOf<PREC>::type> kc, double *__restrict__ partial, Epilogue epi)
{
    forces_body<LAW, PREC, I, POT, JS, false>(rec, npad, nrows, rows, split_len, j_tile, kc, partial,
                                              epi, ExclArgs{});
}

// The same with per-particle exclusion lists (the particle of row r is rows[r]
// or r, and its records are the particle indices themselves).
template <int LAW, int PREC, int I, bool POT>
__global__ __launch_bounds__(256) void k_forces_excl(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec, int64_t npad,
    int64_t nrows, const int64_t *__restrict__ rows, int64_t split_len, int j_tile,
    PairK<typename RealOf<PREC>::type> kc, double *__restrict__ partial, Epilogue epi, ExclArgs ex)
{
    forces_body<LAW, PREC, I, POT, 1, true>(rec, npad, nrows, rows, split_len, j_tile, kc, partial,
                                            epi, ex);
}

template <typename T> static PairK<T> pair_constants(const FwdLaunch &f)
{
    PairK<T> k;
    k.eps2 = (T)f.eps2;
    k.za = (T)f.zeta[0];
    k.zb = (T)f.zeta[1];
    k.zc = (T)f.zeta[2];
    k.zd = (T)f.zeta[3];
    k.za3 = (T)(3.0 * f.zeta[0]);
    k.zb2 = (T)(2.0 * f.zeta[1]);
    return k;
}

// rows per lane instantiated for each law: the two dielectric variants beyond
// the linear one are built for up to 2 rows per lane
template <int LAW> constexpr int kMaxIpl = LAW >= LJC_CONST ? 2 : 8;

template <int LAW, int PREC, int I, bool POT>
static bool launch_one(const FwdLaunch &f, dim3 grid, hipStream_t s)
{
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    if constexpr (I > kMaxIpl<LAW>) {
        return false;
    } else {
        const PairK<T> kc = pair_constants<T>(f);
        if (f.excl.off) {           // exclusion lists: LJC laws, LDS staging, up to 2 rows per lane
            if constexpr (LAW != GRAVITY && I <= 2 && PREC != P_PLAIN) {
                hipLaunchKernelGGL((k_forces_excl<LAW, PREC, I, POT>), grid, dim3(f.block), 0, s,
                                   (const R *)f.rec, f.npad, f.nrows, f.rows, f.split_len, f.j_tile,
                                   kc, f.j_split > 1 ? f.partial : nullptr, f.epi, f.excl);
                return true;
            }
            return false;
        }
        if constexpr (I <= 4) {     // LDS staging is instantiated up to 4 rows per lane
            if (f.j_stage == 1) {
                hipLaunchKernelGGL((k_forces<LAW, PREC, I, POT, 1>), grid, dim3(f.block), 0, s,
                                   (const R *)f.rec, f.npad, f.nrows, f.rows, f.split_len,
                                   f.j_tile, kc, f.j_split > 1 ? f.partial : nullptr, f.epi);
                return true;
            }
        }
        hipLaunchKernelGGL((k_forces<LAW, PREC, I, POT, 0>), grid, dim3(f.block), 0, s,
                           (const R *)f.rec, f.npad, f.nrows, f.rows, f.split_len, f.j_tile, kc,
                           f.j_split > 1 ? f.partial : nullptr, f.epi);
        return true;
    }
}

template <int LAW, int PREC, bool POT>
static bool dispatch_ipl(const FwdLaunch &f, dim3 grid, hipStream_t s)
{
    switch (f.ipl) {
    case 1: return launch_one<LAW, PREC, 1, POT>(f, grid, s);
    case 2: return launch_one<LAW, PREC, 2, POT>(f, grid, s);
    case 4: return launch_one<LAW, PREC, 4, POT>(f, grid, s);
    case 8: return launch_one<LAW, PREC, 8, POT>(f, grid, s);
    default: return false;
    }
}

template <int LAW, bool POT>
static bool dispatch_prec(const FwdLaunch &f, dim3 grid, hipStream_t s)
{
    switch (f.prec) {
    case P_FP64: return dispatch_ipl<LAW, P_FP64, POT>(f, grid, s);
    case P_KAHAN: return dispatch_ipl<LAW, P_KAHAN, POT>(f, grid, s);
    case P_FP64ACC: return dispatch_ipl<LAW, P_FP64ACC, POT>(f, grid, s);
    case P_PLAIN:
        if constexpr (LAW <= LJC) return dispatch_ipl<LAW, P_PLAIN, POT>(f, grid, s);
        return false;
    default: return false;
    }
}

// Resident workgroups per CU of the all-pairs kernel a launch would use
// (from the compiled register and LDS footprint), 0 if unknown.
template <int LAW, int PREC, int I, bool POT>
static const void *forces_ptr(int js)
{
    if constexpr (I > kMaxIpl<LAW> || (LAW > LJC && PREC == P_PLAIN)) {
        return nullptr;
    } else {
        if constexpr (I <= 4) {
            if (js == 1) return (const void *)&k_forces<LAW, PREC, I, POT, 1>;
        }
        return (const void *)&k_forces<LAW, PREC, I, POT, 0>;
    }
}

template <int LAW, int PREC, bool POT>
static const void *forces_ptr_ipl(int ipl, int js)
{
    switch (ipl) {
    case 1: return forces_ptr<LAW, PREC, 1, POT>(js);
    case 2: return forces_ptr<LAW, PREC, 2, POT>(js);
    case 4: return forces_ptr<LAW, PREC, 4, POT>(js);
    case 8: return forces_ptr<LAW, PREC, 8, POT>(js);
    default: return nullptr;
    }
}

template <int LAW, bool POT>
static const void *forces_ptr_prec(int prec, int ipl, int js)
{
    switch (prec) {
    case P_FP64: return forces_ptr_ipl<LAW, P_FP64, POT>(ipl, js);
    case P_KAHAN: return forces_ptr_ipl<LAW, P_KAHAN, POT>(ipl, js);
    case P_FP64ACC: return forces_ptr_ipl<LAW, P_FP64ACC, POT>(ipl, js);
    case P_PLAIN: return forces_ptr_ipl<LAW, P_PLAIN, POT>(ipl, js);
    default: return nullptr;
    }
}

int forces_blocks_per_cu(int law, int prec, int ipl, int pot, int js, int block)
{
    const void *fn = nullptr;
    switch (law) {
    case GRAVITY:
        fn = pot ? forces_ptr_prec<GRAVITY, true>(prec, ipl, js) : forces_ptr_prec<GRAVITY, false>(prec, ipl, js);
        break;
    case LJC: fn = pot ? forces_ptr_prec<LJC, true>(prec, ipl, js) : forces_ptr_prec<LJC, false>(prec, ipl, js); break;
    case LJC_CONST:
        fn = pot ? forces_ptr_prec<LJC_CONST, true>(prec, ipl, js)
                 : forces_ptr_prec<LJC_CONST, false>(prec, ipl, js);
        break;
    case LJC_SIG:
        fn = pot ? forces_ptr_prec<LJC_SIG, true>(prec, ipl, js) : forces_ptr_prec<LJC_SIG, false>(prec, ipl, js);
        break;
    default: break;
    }
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0) != hipSuccess) return 0;
    return nb;
}

template <bool POT>
static bool dispatch_law(const FwdLaunch &f, dim3 grid, hipStream_t s)
{
    switch (f.law) {
    case GRAVITY: return dispatch_prec<GRAVITY, POT>(f, grid, s);
    case LJC: return dispatch_prec<LJC, POT>(f, grid, s);
    case LJC_CONST: return dispatch_prec<LJC_CONST, POT>(f, grid, s);
    case LJC_SIG: return dispatch_prec<LJC_SIG, POT>(f, grid, s);
    default: return false;
    }
}

hipError_t launch_forces(const FwdLaunch &f, hipStream_t s)
{
    if (f.block < 64 || f.block > 256 || f.block % 64 != 0) return hipErrorInvalidValue;   // launch bounds
    if (f.nrows <= 0) return hipSuccess;
    const int64_t waves = (f.nrows + (int64_t)kWave * f.ipl - 1) / ((int64_t)kWave * f.ipl);
    const int64_t wpb = f.block / kWave;
    const dim3 grid((unsigned)((waves + wpb - 1) / wpb), (unsigned)f.j_split);
    const bool ok = f.pot ? dispatch_law<true>(f, grid, s) : dispatch_law<false>(f, grid, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------- fixed-order split sum ----
// split_group(j_split) lanes per row (split_group_sum: a fixed order for a
// given split, so results repeat bit for bit)
__global__ __launch_bounds__(256) void k_reduce_split(const double *__restrict__ partial,
                                                      int64_t nrows, int j_split, int pot,
                                                      Epilogue epi)
{
    const int G = split_group(j_split);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((tid & ~int64_t(kWave - 1)) / G >= nrows) return;   // the whole wave is past the rows
    const int64_t r = tid / G;
    const int q = (int)(tid - r * G);
    double v[4];
    split_group_sum<4>(partial, nrows * 4, 4, r, r < nrows, j_split, q, G, v);
    if (q == 0 && r < nrows) finish_row(epi, r, v[0], v[1], v[2], v[3], pot != 0);
}

hipError_t launch_reduce_split(const FwdLaunch &f, hipStream_t s)
{
    if (f.nrows <= 0 || f.j_split <= 1) return hipSuccess;
    const int64_t threads = f.nrows * split_group(f.j_split);
    hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (const double *)f.partial, f.nrows, f.j_split, f.pot, f.epi);
    return hipGetLastError();
}

// ------------------------------------------------------------- zero fill ----
__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *p, int64_t words)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t words = (int64_t)(bytes / 4);
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                       (uint32_t *)p, words);
    return hipGetLastError();
}

}  // namespace nbk
