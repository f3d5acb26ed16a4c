// Many independent systems of uneven size in one persistent launch.
//
// The paper's small-system problem (Section 3.4: too few i-particles to fill
// the machine, fixed per-kernel overhead) is addressed here by batching: the
// host lists (system, row-block) work units in decreasing order of cost
// (longest-processing-time first), and a persistent grid sized to the chip's
// resident-wave capacity pulls units with an integer ticket until the list
// is exhausted.  Each unit is the same tiled j loop as the single-system
// kernel, restricted to the records of its own system.
#include "device.h"
#include "kernels.h"

namespace nbk {

template <typename T> struct IStateB;
template <typename T> struct IStateB<GravRec<T>> { using type = GravI<T>; };
template <typename T> struct IStateB<LjcRec<T>> { using type = LjcI<T>; };

template <typename T>
__device__ __forceinline__ void load_ib(const GravRec<T> *rec, int64_t p, GravI<T> &s)
{
    const GravRec<T> r = rec[p];
    s.x = r.x;
    s.y = r.y;
    s.z = r.z;
}

template <typename T>
__device__ __forceinline__ void load_ib(const LjcRec<T> *rec, int64_t p, LjcI<T> &s)
{
    const LjcRec<T> r = rec[p];
    s.x = r.x;
    s.y = r.y;
    s.z = r.z;
    s.qs = r.qs;
    s.sh = r.sh;
    s.se = r.se;
}

template <bool MASK, bool POT, typename T>
__device__ __forceinline__ void pair_b(const GravI<T> &i, const GravRec<T> &j, T eps2, bool self,
                                       T (&p)[4])
{
    grav_pair<MASK, POT>(i, j.x, j.y, j.z, j.m, eps2, self, p);
}

template <bool MASK, bool POT, typename T>
__device__ __forceinline__ void pair_b(const LjcI<T> &i, const LjcRec<T> &j, T, bool self, T (&p)[4])
{
    ljc_pair<MASK, POT>(i, j.x, j.y, j.z, j.qs, j.sh, j.se, self, p);
}

template <bool MASK, bool POT, int I, typename R, typename IS, typename T>
__device__ __forceinline__ void tile_loop_b(const R *__restrict__ rec, int64_t t0, int64_t t1,
                                            const IS (&is)[I], const int64_t (&pid)[I], T eps2,
                                            T (&p)[I][4])
{
    constexpr int U = 8;
    for (int64_t j = t0; j < t1; j += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const R r = rec[j + u];
#pragma unroll
            for (int k = 0; k < I; ++k)
                pair_b<MASK, POT>(is[k], r, eps2, MASK && (pid[k] == j + u), p[k]);
        }
    }
}

__device__ __forceinline__ void finish_row_b(const Epilogue &e, int64_t r, double v0, double v1,
                                             double v2, double v3, bool pot)
{
    e.out_force[3 * r] = e.fscale * v0;
    e.out_force[3 * r + 1] = e.fscale * v1;
    e.out_force[3 * r + 2] = e.fscale * v2;
    if (pot && e.out_pot) e.out_pot[r] = e.pscale * v3;
}

template <int LAW, int PREC, int I, bool POT>
__global__ __launch_bounds__(256) void k_batched(
    const typename RecOf<typename RealOf<PREC>::type, LAW>::type *__restrict__ rec,
    const int32_t *__restrict__ units, int64_t n_units, const int64_t *__restrict__ off,
    const int64_t *__restrict__ poff, int j_tile, typename RealOf<PREC>::type eps2, int *ticket,
    Epilogue epi)
{
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    using IS = typename IStateB<R>::type;
    constexpr int NC = POT ? 4 : 3;
    const int lane = lane_id();

    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(ticket, 1);
        u = __builtin_amdgcn_readfirstlane(u);
        if ((int64_t)u >= n_units) break;      // every wave leaves once the list is drained
        const int s = units[2 * (int64_t)u];
        const int64_t rb = units[2 * (int64_t)u + 1];
        const int64_t o = off[s], ns = off[s + 1] - o;
        const int64_t po = poff[s], pe = poff[s + 1];
        const int64_t lbase = rb * (int64_t)(kWave * I);

        IS is[I];
        int64_t pid[I];
#pragma unroll
        for (int k = 0; k < I; ++k) {
            int64_t l = lbase + lane + (int64_t)kWave * k;
            l = l < ns ? l : ns - 1;
            pid[k] = po + l;
            load_ib(rec, pid[k], is[k]);
        }
        RunSum<PREC> acc[I][NC];
        T p[I][4];
#pragma unroll
        for (int k = 0; k < I; ++k) p[k][3] = T(0);

        for (int64_t t0 = po; t0 < pe; t0 += j_tile) {
            const int64_t t1 = (t0 + j_tile < pe) ? t0 + j_tile : pe;
            bool near = false;
#pragma unroll
            for (int k = 0; k < I; ++k) near |= (pid[k] >= t0) & (pid[k] < t1);
#pragma unroll
            for (int k = 0; k < I; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[k][c].begin(p[k][c]);
            if (wave_any(near))
                tile_loop_b<true, POT, I>(rec, t0, t1, is, pid, (T)eps2, p);
            else
                tile_loop_b<false, POT, I>(rec, t0, t1, is, pid, (T)eps2, p);
#pragma unroll
            for (int k = 0; k < I; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[k][c].fold(p[k][c]);
        }
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const int64_t l = lbase + lane + (int64_t)kWave * k;
            if (l >= ns) continue;
            finish_row_b(epi, o + l, acc[k][0].value(), acc[k][1].value(), acc[k][2].value(),
                         POT ? acc[k][NC - 1].value() : 0.0, POT);
        }
    }
}

// ---------------------------------------------------------------- packing ----
template <typename T>
__device__ __forceinline__ void put(GravRec<T> *rec, int64_t i, const double *x, const double *par,
                                    double)
{
    GravRec<T> r;
    r.x = (T)x[0];
    r.y = (T)x[1];
    r.z = (T)x[2];
    r.m = (T)par[0];
    rec[i] = r;
}
template <typename T>
__device__ __forceinline__ void put(LjcRec<T> *rec, int64_t i, const double *x, const double *par,
                                    double qscale)
{
    LjcRec<T> r;
    r.x = (T)x[0];
    r.y = (T)x[1];
    r.z = (T)x[2];
    r.qs = (T)(par[0] * qscale);
    r.sh = (T)(0.5 * par[1]);
    r.se = (T)__builtin_sqrt(par[2]);
    r.p0 = r.p1 = T(0);
    rec[i] = r;
}
template <typename T> __device__ __forceinline__ void put_pad(GravRec<T> *rec, int64_t i)
{
    GravRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.m = T(0);
    rec[i] = r;
}
template <typename T> __device__ __forceinline__ void put_pad(LjcRec<T> *rec, int64_t i)
{
    LjcRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.qs = r.sh = r.se = r.p0 = r.p1 = T(0);
    rec[i] = r;
}

// One thread per padded slot; the owning system is found by binary search
// over the padded offsets.
template <typename R, int P>
__global__ __launch_bounds__(256) void k_pack_batched(BatchPackLaunch a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
        put(rec, i, a.pos + 3 * src, a.params + (int64_t)P * src, a.qscale);
    } else {
        put_pad(rec, i);
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
static const void *kernel_ptr()
{
    return (const void *)&k_batched<LAW, PREC, I, POT>;
}

template <int LAW, int PREC, int I, bool POT>
static void launch_b(const BatchLaunch &b, hipStream_t s)
{
    using T = typename RealOf<PREC>::type;
    using R = typename RecOf<T, LAW>::type;
    hipLaunchKernelGGL((k_batched<LAW, PREC, I, POT>), dim3(b.grid), dim3(b.block), 0, s,
                       (const R *)b.rec, b.units, b.n_units, b.off, b.poff, b.j_tile, (T)b.eps2,
                       b.ticket, b.epi);
}

// Calls F<LAW, PREC, I, POT>::run(args...) for the runtime selectors.
#define NBK_BATCH_SWITCH(LAWV, PRECV, IPLV, POTV, CALL)                                           \
    do {                                                                                         \
        switch ((LAWV) * 1000 + (PRECV) * 100 + (IPLV) * 10 + ((POTV) ? 1 : 0)) {               \
        NBK_BCASE(0, 0, 1, CALL) NBK_BCASE(0, 0, 2, CALL) NBK_BCASE(0, 0, 4, CALL)               \
        NBK_BCASE(0, 1, 1, CALL) NBK_BCASE(0, 1, 2, CALL) NBK_BCASE(0, 1, 4, CALL)               \
        NBK_BCASE(0, 2, 1, CALL) NBK_BCASE(0, 2, 2, CALL) NBK_BCASE(0, 2, 4, CALL)               \
        NBK_BCASE(0, 3, 1, CALL) NBK_BCASE(0, 3, 2, CALL) NBK_BCASE(0, 3, 4, CALL)               \
        NBK_BCASE(1, 0, 1, CALL) NBK_BCASE(1, 0, 2, CALL) NBK_BCASE(1, 0, 4, CALL)               \
        NBK_BCASE(1, 1, 1, CALL) NBK_BCASE(1, 1, 2, CALL) NBK_BCASE(1, 1, 4, CALL)               \
        NBK_BCASE(1, 2, 1, CALL) NBK_BCASE(1, 2, 2, CALL) NBK_BCASE(1, 2, 4, CALL)               \
        NBK_BCASE(1, 3, 1, CALL) NBK_BCASE(1, 3, 2, CALL) NBK_BCASE(1, 3, 4, CALL)               \
        default: break;                                                                          \
        }                                                                                        \
    } while (0)
#define NBK_BCASE(L, P, I, CALL)                                                                 \
    case L * 1000 + P * 100 + I * 10 + 1: CALL(L, P, I, true); break;                            \
    case L * 1000 + P * 100 + I * 10 + 0: CALL(L, P, I, false); break;

hipError_t launch_batched(const BatchLaunch &b, hipStream_t s)
{
    if (b.n_units <= 0) return hipSuccess;
    hipError_t e = launch_fill_zero(b.ticket, 256, s);
    if (e != hipSuccess) return e;
    bool launched = false;
#define NBK_DO_LAUNCH(L, P, I, POT) (launch_b<L, P, I, POT>(b, s), launched = true)
    NBK_BATCH_SWITCH(b.law, b.prec, b.ipl, b.pot, NBK_DO_LAUNCH);
#undef NBK_DO_LAUNCH
    if (!launched) return hipErrorInvalidValue;
    return hipGetLastError();
}

int batched_max_blocks_per_cu(int law, int prec, int ipl, int pot, int block)
{
    const void *fn = nullptr;
#define NBK_GET_PTR(L, P, I, POT) (fn = kernel_ptr<L, P, I, POT>())
    NBK_BATCH_SWITCH(law, prec, ipl, pot, NBK_GET_PTR);
#undef NBK_GET_PTR
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0) != hipSuccess) return 0;
    return nb;
}

}  // namespace nbk
