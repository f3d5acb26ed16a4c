// Many independent systems of uneven size in one persistent launch.
//
// The paper's small-system problem (Section 3.4: too few i-particles to fill
// the machine, fixed per-kernel overhead) is addressed here by batching: the
// host lists (system, row-block, j-part) work units in decreasing order of
// cost (longest-processing-time first), and a persistent grid sized to the
// chip's resident-wave capacity pulls units with an integer ticket until the
// list is exhausted.  Each unit is the same tiled j loop as the single-system
// kernel, restricted to one part of the records of its own system.  A system
// whose j range is cut into P > 1 parts (Section 3.4's replication, applied
// per system so that there are enough units to balance the machine) writes
// per-part partial sums, which k_batched_reduce adds in part order (one
// workgroup per row block of such a system, from the plan's list).
#include <type_traits>

#include "allpairs.h"
#include "kernels.h"

namespace nbk {

// EX: with per-particle exclusion lists over the caller's (global) particle
// indices; only partners in the particle's own system can match.
template <int LAW, int PREC, int I, bool POT, int JS, bool EX>
__device__ __forceinline__ void batched_body(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec,
    const BatchLaunch &b, PairK<typename RealOf<PREC>::type> kc)
{
    const int32_t *__restrict__ units = b.units;
    const int64_t *__restrict__ off = b.off;
    const int64_t *__restrict__ poff = b.poff;
    const Epilogue &epi = b.epi;
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    using IS = typename IStateOf<R>::type;
    constexpr int NC = POT ? 4 : 3;
    const int lane = lane_id();
    __shared__ R lds_j[JS ? 4 : 1][2][kWave];
    R(*wl)[kWave] = lds_j[JS ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];

    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(b.ticket, 1);
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= b.n_units) break;    // every wave leaves once the list is drained
        const int s = units[4 * (int64_t)u];
        if (s < 0 || (int64_t)s >= b.n_systems) continue;   // never index outside the tables
        const int64_t rb = units[4 * (int64_t)u + 1];
        const int64_t part = units[4 * (int64_t)u + 2];
        const int64_t o = off[s], ns = off[s + 1] - o;
        const int64_t po = poff[s], pe = poff[s + 1];
        const int64_t nparts = b.systab[3 * (int64_t)s], plen = b.systab[3 * (int64_t)s + 1];
        const int64_t jb = po + part * plen;
        const int64_t je = jb + plen < pe ? jb + plen : pe;
        const int64_t lbase = rb * (int64_t)(kWave * I);

        IS is[I];
        int64_t pid[I], gid[I];
#pragma unroll
        for (int k = 0; k < I; ++k) {
            int64_t l = lbase + lane + (int64_t)kWave * k;
            l = l < ns ? l : ns - 1;
            pid[k] = po + l;
            gid[k] = o + l;
            load_i(rec, pid[k], is[k]);
        }
        RunSum<PREC> acc[I][NC];
        T p[I][4];
#pragma unroll
        for (int k = 0; k < I; ++k) p[k][3] = T(0);
        if constexpr (EX) {
            static_assert(JS == 1, "exclusion lists use the LDS staging");
            ExclMask<I> mask;
#pragma unroll
            for (int k = 0; k < I; ++k) mask.pid[k] = pid[k];
            mask.init(b.excl, gid, po - o);
            j_range_masked<JS, ForceOp<POT, LAW>, PREC, I>(rec, jb, je, b.j_tile, is, mask, kc, acc, p, wl);
        } else {
            j_range<JS, ForceOp<POT, LAW>, PREC, I>(rec, jb, je, b.j_tile, is, pid, kc, acc, p, wl);
        }
        const int64_t slot = b.systab[3 * (int64_t)s + 2] + rb * nparts + part;
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const int64_t l = lbase + lane + (int64_t)kWave * k;
            if (l >= ns) continue;
            if (nparts > 1) {            // partial sums of this part, added by k_batched_reduce
                double *q = b.partial + (slot * (kWave * I) + lane + kWave * k) * 4;
                q[0] = acc[k][0].value();
                q[1] = acc[k][1].value();
                q[2] = acc[k][2].value();
                q[3] = POT ? acc[k][NC - 1].value() : 0.0;
                continue;
            }
            const int64_t r = o + l;
            epi.out_force[3 * r] = epi.fscale * acc[k][0].value();
            epi.out_force[3 * r + 1] = epi.fscale * acc[k][1].value();
            epi.out_force[3 * r + 2] = epi.fscale * acc[k][2].value();
            if (POT && epi.out_pot) epi.out_pot[r] = epi.pscale * acc[k][NC - 1].value();
        }
    }
}

// The rows of systems cut into several j parts: the part sums in part order
// (Neumaier, so the result does not depend on the schedule).
// Row block red[blockIdx.x] of a system cut into P > 1 parts: each thread adds its row's P
// part sums in part order (FP64, Neumaier) and writes the row.  The P loads of a row are
// issued before the sums, four parts at a time.
__global__ __launch_bounds__(256) void k_batched_reduce(BatchLaunch b)
{
    const int64_t s = b.red[2 * blockIdx.x], rb = b.red[2 * blockIdx.x + 1];
    const int64_t rows = (int64_t)kWave * b.ipl;
    const int64_t l = rb * rows + threadIdx.x;
    if (l >= b.off[s + 1] - b.off[s]) return;
    const int64_t r = b.off[s] + l;
    const int64_t nparts = b.systab[3 * s];
    const int64_t slot0 = b.systab[3 * s + 2] + rb * nparts;
    const double4 *__restrict__ q = (const double4 *)b.partial + slot0 * rows + threadIdx.x;
    NSum v[4];
    int64_t p = 0;
    for (; p + 4 <= nparts; p += 4) {
        double4 x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = q[(p + k) * rows];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[0].add(x[k].x);
            v[1].add(x[k].y);
            v[2].add(x[k].z);
            v[3].add(x[k].w);
        }
    }
    for (; p < nparts; ++p) {
        const double4 x = q[p * rows];
        v[0].add(x.x);
        v[1].add(x.y);
        v[2].add(x.z);
        v[3].add(x.w);
    }
    const Epilogue &e = b.epi;
    e.out_force[3 * r] = e.fscale * v[0].value();
    e.out_force[3 * r + 1] = e.fscale * v[1].value();
    e.out_force[3 * r + 2] = e.fscale * v[2].value();
    if (b.pot && e.out_pot) e.out_pot[r] = e.pscale * v[3].value();
}

template <int LAW, int PREC, int I, bool POT, int JS>
__global__ __launch_bounds__(256) void k_batched(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec, BatchLaunch b,
    PairK<typename RealOf<PREC>::type> kc)
{
    batched_body<LAW, PREC, I, POT, JS, false>(rec, b, kc);
}

template <int LAW, int PREC, int I, bool POT>
__global__ __launch_bounds__(256) void k_batched_excl(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec, BatchLaunch b,
    PairK<typename RealOf<PREC>::type> kc)
{
    batched_body<LAW, PREC, I, POT, 1, true>(rec, b, kc);
}

// ---------------------------------------------------------------- packing ----
// One thread per padded slot; the owning system is found by binary search
// over the padded offsets.
template <typename R, int P>
__global__ __launch_bounds__(256) void k_pack_batched(BatchPackLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.ticket && i < 64) a.ticket[i] = 0;     // the work ticket of the launch that follows
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
        store_rec(rec, i, a.pos[3 * src], a.pos[3 * src + 1], a.pos[3 * src + 2],
                  a.params + (int64_t)P * src, a.qscale);
    } else {
        store_pad(rec, i);
    }
}

hipError_t launch_pack_batched(const BatchPackLaunch &p, hipStream_t s)
{
    if (p.npad_total <= 0 || p.n_systems <= 0) return hipSuccess;
    const dim3 grid((unsigned)((p.npad_total + 255) / 256)), block(256);
    const bool f32 = p.prec != P_FP64;
    if (p.law == GRAVITY) {
        if (f32) hipLaunchKernelGGL((k_pack_batched<GravRec<float>, 1>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_batched<GravRec<double>, 1>), grid, block, 0, s, p);
    } else {
        if (f32) hipLaunchKernelGGL((k_pack_batched<LjcRec<float>, 3>), grid, block, 0, s, p);
        else hipLaunchKernelGGL((k_pack_batched<LjcRec<double>, 3>), grid, block, 0, s, p);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------- dispatch ----
template <int LAW, int PREC, int I, bool POT>
static const void *batched_ptr(int js, bool excl)
{
    if (excl) {
        if constexpr (LAW != GRAVITY && I <= 2 && PREC != P_PLAIN)
            return (const void *)&k_batched_excl<LAW, PREC, I, POT>;
        return nullptr;
    }
    if (js == 1) return (const void *)&k_batched<LAW, PREC, I, POT, 1>;
    return (const void *)&k_batched<LAW, PREC, I, POT, 0>;
}

template <int LAW, int PREC, int I, bool POT>
static void launch_b(const BatchLaunch &b, hipStream_t s)
{
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    PairK<T> kc;
    kc.eps2 = (T)b.eps2;
    kc.za = (T)b.zeta[0];
    kc.zb = (T)b.zeta[1];
    kc.zc = (T)b.zeta[2];
    kc.zd = (T)b.zeta[3];
    kc.za3 = (T)(3.0 * b.zeta[0]);
    kc.zb2 = (T)(2.0 * b.zeta[1]);
    if (b.excl.off) {
        if constexpr (LAW != GRAVITY && I <= 2 && PREC != P_PLAIN) {
            hipLaunchKernelGGL((k_batched_excl<LAW, PREC, I, POT>), dim3(b.grid), dim3(b.block), 0, s,
                               (const R *)b.rec, b, kc);
        }
        return;
    }
    if (b.j_stage == 1)
        hipLaunchKernelGGL((k_batched<LAW, PREC, I, POT, 1>), dim3(b.grid), dim3(b.block), 0, s,
                           (const R *)b.rec, b, kc);
    else
        hipLaunchKernelGGL((k_batched<LAW, PREC, I, POT, 0>), dim3(b.grid), dim3(b.block), 0, s,
                           (const R *)b.rec, b, kc);
}

// Calls f.run<LAW, PREC, I, POT>() for the runtime selectors (I in {1, 2, 4});
// false for an unsupported combination.
template <typename F>
static bool batched_dispatch(int law, int prec, int ipl, bool pot, F &f)
{
    auto by_ipl = [&](auto law_c, auto prec_c, auto pot_c) -> bool {
        constexpr int L = decltype(law_c)::value, P = decltype(prec_c)::value;
        constexpr bool O = decltype(pot_c)::value;
        if constexpr (L > LJC && P == P_PLAIN) {
            return false;            // the ablation precision exists for gravity and LJC(linear)
        } else {
            switch (ipl) {
            case 1: f.template run<L, P, 1, O>(); return true;
            case 2: f.template run<L, P, 2, O>(); return true;
            case 4:
                if constexpr (L <= LJC) {
                    f.template run<L, P, 4, O>();
                    return true;
                }
                return false;
            default: return false;
            }
        }
    };
    auto by_pot = [&](auto law_c, auto prec_c) -> bool {
        return pot ? by_ipl(law_c, prec_c, std::true_type{}) : by_ipl(law_c, prec_c, std::false_type{});
    };
    auto by_prec = [&](auto law_c) -> bool {
        switch (prec) {
        case P_FP64: return by_pot(law_c, std::integral_constant<int, P_FP64>{});
        case P_KAHAN: return by_pot(law_c, std::integral_constant<int, P_KAHAN>{});
        case P_FP64ACC: return by_pot(law_c, std::integral_constant<int, P_FP64ACC>{});
        case P_PLAIN: return by_pot(law_c, std::integral_constant<int, P_PLAIN>{});
        default: return false;
        }
    };
    switch (law) {
    case GRAVITY: return by_prec(std::integral_constant<int, GRAVITY>{});
    case LJC: return by_prec(std::integral_constant<int, LJC>{});
    case LJC_CONST: return by_prec(std::integral_constant<int, LJC_CONST>{});
    case LJC_SIG: return by_prec(std::integral_constant<int, LJC_SIG>{});
    default: return false;
    }
}

struct LaunchB {
    const BatchLaunch &b;
    hipStream_t s;
    template <int L, int P, int I, bool O> void run() { launch_b<L, P, I, O>(b, s); }
};

struct PtrB {
    int js;
    bool excl;
    const void *fn = nullptr;
    template <int L, int P, int I, bool O> void run() { fn = batched_ptr<L, P, I, O>(js, excl); }
};

hipError_t launch_batched(const BatchLaunch &b, hipStream_t s)
{
    if (b.n_units <= 0) return hipSuccess;
    hipError_t e = b.ticket_zeroed ? hipSuccess : launch_fill_zero(b.ticket, 256, s);
    if (e != hipSuccess) return e;
    if (b.excl.off && (b.law == GRAVITY || b.ipl > 2 || b.prec == P_PLAIN)) return hipErrorInvalidValue;
    LaunchB l{b, s};
    if (!batched_dispatch(b.law, b.prec, b.ipl, b.pot != 0, l)) return hipErrorInvalidValue;
    e = hipGetLastError();
    if (e != hipSuccess || !b.any_parts || b.n_red <= 0) return e;
    hipLaunchKernelGGL(k_batched_reduce, dim3((unsigned)b.n_red), dim3((unsigned)(kWave * b.ipl)), 0, s, b);
    return hipGetLastError();
}

int batched_max_blocks_per_cu(int law, int prec, int ipl, int pot, int js, int block, int excl)
{
    PtrB g{js, excl != 0};
    if (!batched_dispatch(law, prec, ipl, pot != 0, g) || !g.fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, g.fn, block, 0) != hipSuccess) return 0;
    return nb;
}

}  // namespace nbk
