// The tiled all-pairs j loop shared by the single-system and batched kernels.
//
// A wave holds I rows per lane (i state in VGPRs) and walks a j range
// [jb, je) (a multiple of 64 records) in tiles of j_tile records; each
// tile's FP32 partial sums are folded into the running sums (RunSum) at the
// tile's end.  Two ways of bringing the j records to the arithmetic:
//   JS = 0  wave-uniform scalar loads into SGPRs (the VALU instructions read
//           one SGPR operand each);
//   JS = 1  a wave-private, double-buffered LDS slot of 64 records, read back
//           as broadcasts into VGPRs (all-VGPR arithmetic, which gfx950 issues
//           at a higher rate than instructions with an SGPR operand).
// The self pair (j == i), and with exclusion lists the listed pairs, are
// neutralised only in tiles or chunks that may hold them (a wave-uniform test).
#pragma once
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace nbk {

// ------------------------------------------------------------ record packing
template <typename T>
__device__ __forceinline__ void store_rec(GravRec<T> *rec, int64_t i, double x, double y, double z,
                                          const double *par, double)
{
    GravRec<T> r;
    r.x = (T)x;
    r.y = (T)y;
    r.z = (T)z;
    r.m = (T)par[0];
    rec[i] = r;
}

template <typename T>
__device__ __forceinline__ void store_rec(LjcRec<T> *rec, int64_t i, double x, double y, double z,
                                          const double *par, double qscale)
{
    LjcRec<T> r;
    r.x = (T)x;
    r.y = (T)y;
    r.z = (T)z;
    r.qs = (T)(par[0] * qscale);
    r.sh = (T)(0.5 * par[1]);
    r.se = (T)__builtin_sqrt(24.0 * par[2]);
    r.p0 = T(0);
    r.p1 = T(0);
    rec[i] = r;
}

template <typename T>
__device__ __forceinline__ void store_pad(GravRec<T> *rec, int64_t i)
{
    GravRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.m = T(0);
    rec[i] = r;
}

template <typename T>
__device__ __forceinline__ void store_pad(LjcRec<T> *rec, int64_t i)
{
    LjcRec<T> r;
    r.x = r.y = r.z = (T)kPadCoord;
    r.qs = r.sh = r.se = r.p0 = r.p1 = T(0);
    rec[i] = r;
}

// ------------------------------------------------------- per-law i / j I/O ----
template <typename T>
__device__ __forceinline__ void load_i(const GravRec<T> *rec, int64_t p, GravI<T> &s)
{
    const GravRec<T> r = rec[p];
    s.x = r.x;
    s.y = r.y;
    s.z = r.z;
}

template <typename T>
__device__ __forceinline__ void load_i(const LjcRec<T> *rec, int64_t p, LjcI<T> &s)
{
    const LjcRec<T> r = rec[p];
    s.x = r.x;
    s.y = r.y;
    s.z = r.z;
    s.qs = r.qs;
    s.sh = r.sh;
    s.se = r.se;
}

// Make the i-state loads complete here (an empty asm that reads the values),
// so that no wait for them is left pending into the j loop.
template <typename T> __device__ __forceinline__ void settle(const GravI<T> &s)
{
    asm volatile("" ::"v"(s.x), "v"(s.y), "v"(s.z));
}
template <typename T> __device__ __forceinline__ void settle(const LjcI<T> &s)
{
    asm volatile("" ::"v"(s.x), "v"(s.y), "v"(s.z), "v"(s.qs), "v"(s.sh), "v"(s.se));
}

template <typename T> struct IStateOf;
template <typename T> struct IStateOf<GravRec<T>> { using type = GravI<T>; };
template <typename T> struct IStateOf<LjcRec<T>> { using type = LjcI<T>; };

template <bool MASK, bool POT, int LAW, typename T>
__device__ __forceinline__ void pair(const GravI<T> &i, const GravRec<T> &j, const PairK<T> &k,
                                     bool self, T (&p)[4])
{
    grav_pair<MASK, POT>(i, j.x, j.y, j.z, j.m, k, self, p);
}

template <bool MASK, bool POT, int LAW, typename T>
__device__ __forceinline__ void pair(const LjcI<T> &i, const LjcRec<T> &j, const PairK<T> &k,
                                     bool self, T (&p)[4])
{
    ljc_pair<MASK, POT, LAW>(i, j.x, j.y, j.z, j.qs, j.sh, j.se, k, self, p);
}

// The pair operation of the forward kernels: Op::NC running sums
// (force and, with POT, potential) from the pair functions above.
template <bool POT, int LAW> struct ForceOp {
    static constexpr int NC = POT ? 4 : 3;
    static constexpr int NP = 4;
    template <bool MASK, typename IS, typename R, typename T>
    static __device__ __forceinline__ void run(const IS &i, const R &j, const PairK<T> &k, bool self,
                                               T (&p)[NP])
    {
        pair<MASK, POT, LAW>(i, j, k, self, p);
    }
};

// The j loop over one tile [t0, t1) (a multiple of 8 records).  `rec` is a
// restrict-qualified read-only pointer and j is wave-uniform, so each record
// load is a scalar load shared by the 64 lanes.
template <bool MASK, typename Op, int I, typename R, typename IS, typename T>
__device__ __forceinline__ void tile_loop(const R *__restrict__ rec, int64_t t0, int64_t t1,
                                          const IS (&is)[I], const int64_t (&pid)[I],
                                          const PairK<T> &kc, T (&p)[I][Op::NP])
{
    constexpr int U = 8;
    R cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = rec[t0 + u];
    for (int64_t j = t0; j < t1; j += U) {
        // prefetch the next group (the last group re-reads itself: always in bounds)
        const int64_t jn = (j + U < t1) ? j + U : j;
        R nxt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = rec[jn + u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < I; ++k)
                Op::template run<MASK>(is[k], cur[u], kc, MASK && (pid[k] == j + u), p[k]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
}

// ------------------------------------------------------------ pair masks
// Which pairs of a 64-record chunk [c, c + 64) are left out of row k's sums.
// SelfMask: only j == i.  ExclMask: j == i and the particles on the row's
// exclusion list (Section 5: the LJC kernels read an exclusion list per
// particle).  `near` is the lane's test of whether the chunk may hold an
// excluded pair (the wave runs the masked loop when any lane says so); `load`
// prepares the chunk's masks; `excluded` is the per-pair test.
// SelfMask keeps, per row, the row's offset in the chunk being masked (a
// 32-bit value, so that the per-pair test compares with an inline constant
// rather than holding 64-bit j indices in registers).
template <int I> struct SelfMask {
    int64_t pid[I];
    int32_t rel[I];
    __device__ __forceinline__ bool near(int64_t c) const
    {
        bool b = false;
#pragma unroll
        for (int k = 0; k < I; ++k) b |= (pid[k] >= c) & (pid[k] < c + kWave);
        return b;
    }
    __device__ __forceinline__ void load(int64_t c)
    {
#pragma unroll
        for (int k = 0; k < I; ++k) {
            const int64_t d = pid[k] - c;
            rel[k] = (d >= 0 && d < kWave) ? (int32_t)d : -1;
        }
    }
    __device__ __forceinline__ bool excluded(int k, int64_t, int jj) const { return rel[k] == jj; }
};

// Row k is particle g[k] of the caller's arrays and record pid[k]; the
// record of particle x is x + shift.  List entries are only compared, never
// used as addresses, and the list ranges are clamped to [0, count), so any
// content of the lists is safe to read.
template <int I> struct ExclMask {
    const int64_t *idx;
    int64_t shift;
    int64_t pid[I], lo[I], hi[I], b[I], e[I];
    uint64_t m[I];
    __device__ __forceinline__ void init(const ExclArgs &ex, const int64_t (&g)[I], int64_t sh)
    {
        idx = ex.idx;
        shift = sh;
#pragma unroll
        for (int k = 0; k < I; ++k) {
            int64_t e0 = ex.off[g[k] + 1];
            e0 = e0 < ex.count ? (e0 > 0 ? e0 : 0) : ex.count;
            int64_t b0 = ex.off[g[k]];
            b0 = b0 < e0 ? (b0 > 0 ? b0 : 0) : e0;
            b[k] = b0;
            e[k] = e0;
            lo[k] = hi[k] = pid[k];
            for (int64_t t = b0; t < e0; ++t) {
                const int64_t r = idx[t] + shift;
                lo[k] = r < lo[k] ? r : lo[k];
                hi[k] = r > hi[k] ? r : hi[k];
            }
            m[k] = 0;
        }
    }
    __device__ __forceinline__ bool near(int64_t c) const
    {
        bool x = false;
#pragma unroll
        for (int k = 0; k < I; ++k) x |= (lo[k] < c + kWave) & (hi[k] >= c);
        return x;
    }
    __device__ __forceinline__ void load(int64_t c)
    {
#pragma unroll
        for (int k = 0; k < I; ++k) {
            uint64_t bits = 0;
            if ((lo[k] < c + kWave) & (hi[k] >= c)) {
                const int64_t d0 = pid[k] - c;
                if (d0 >= 0 && d0 < kWave) bits |= uint64_t(1) << d0;
                for (int64_t t = b[k]; t < e[k]; ++t) {
                    const int64_t d = idx[t] + shift - c;
                    if (d >= 0 && d < kWave) bits |= uint64_t(1) << d;
                }
            }
            m[k] = bits;
        }
    }
    __device__ __forceinline__ bool excluded(int k, int64_t, int jj) const { return (m[k] >> jj) & 1; }
};

// The j loop over one 64-record chunk held in the wave's LDS slot (j_stage 1).
// Every lane reads the same record (an LDS broadcast) into VGPRs, so the pair
// arithmetic has only VGPR operands.
template <bool MASK, typename Op, int I, typename R, typename IS, typename T, typename M>
__device__ __forceinline__ void chunk_loop(const R *wl, int64_t c, const IS (&is)[I], const M &mask,
                                           const PairK<T> &kc, T (&p)[I][Op::NP])
{
#pragma unroll 16
    for (int jj = 0; jj < kWave; ++jj) {
        const R r = wl[jj];
#pragma unroll
        for (int k = 0; k < I; ++k)
            Op::template run<MASK>(is[k], r, kc, MASK && mask.excluded(k, c, jj), p[k]);
    }
}

// Run the j range [jb, je) for one wave's rows.  `wl` is the wave's pair of
// 64-record LDS slots (used when JS == 1).  `mask` decides which pairs are
// left out (SelfMask, or ExclMask with JS == 1 only).
template <int JS, typename Op, int PREC, int I, typename R, typename IS, typename T, typename M>
__device__ __forceinline__ void j_range_masked(const R *__restrict__ rec, int64_t jb, int64_t je,
                                               int j_tile, const IS (&is)[I], M &mask,
                                               const PairK<T> &kc, RunSum<PREC> (&acc)[I][Op::NC],
                                               T (&p)[I][Op::NP], R (*wl)[kWave])
{
    constexpr int NC = Op::NC;
    const int lane = lane_id();
    if constexpr (JS == 0) {
        static_assert(std::is_same<M, SelfMask<I>>::value, "scalar staging masks the self pair only");
        const int64_t(&pid)[I] = mask.pid;
        for (int64_t t0 = jb; t0 < je; t0 += j_tile) {
            const int64_t t1 = (t0 + j_tile < je) ? t0 + j_tile : je;
            bool near = false;
#pragma unroll
            for (int k = 0; k < I; ++k) near |= (pid[k] >= t0) & (pid[k] < t1);
#pragma unroll
            for (int k = 0; k < I; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[k][c].begin(p[k][c]);
            if (wave_any(near))
                tile_loop<true, Op, I>(rec, t0, t1, is, pid, kc, p);
            else
                tile_loop<false, Op, I>(rec, t0, t1, is, pid, kc, p);
#pragma unroll
            for (int k = 0; k < I; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[k][c].fold(p[k][c]);
        }
    } else {
        // Two wave-private LDS slots of 64 records.  Lane l stages record l of
        // each chunk (a coalesced vector load, then an LDS store), and the wave
        // reads the slot back as 64 broadcasts.  No block barrier is needed: one
        // wave writes and reads its own slots, and LDS executes a wave's
        // accesses in order; the wave barriers only keep the compiler from
        // reordering them (a memory fence here would also wait for the
        // prefetch load in flight).
        // softening in a VGPR so that r^2 + eps^2 is an all-VGPR multiply-add
        PairK<T> kv = kc;
        if constexpr (sizeof(T) == 4) asm volatile("v_mov_b32 %0, %1" : "=v"(kv.eps2) : "s"(kc.eps2));
        // Prefetch distance: the record stored into the free slot at the end of
        // chunk c was loaded at the end of chunk c - 64, one full chunk of
        // arithmetic earlier (the value is carried across the loop back-edge,
        // so the load cannot be sunk next to its store).  Indices past the
        // range are clamped to the last chunk: always in bounds, never read.
        // records move as native vectors (SSA values, never a stack object)
        using V = T __attribute__((ext_vector_type(sizeof(R) / sizeof(T))));
        const V *vrec = reinterpret_cast<const V *>(rec);
        V *vwl0 = reinterpret_cast<V *>(wl[0]);
        V *vwl1 = reinterpret_cast<V *>(wl[1]);
#pragma unroll
        for (int k = 0; k < I; ++k) settle(is[k]);
        if (jb < je) {
            const int64_t last = je - kWave;
            vwl0[lane] = vrec[jb + lane];
            V g = vrec[(jb + kWave < je ? jb + kWave : last) + lane];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < I; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[k][c].begin(p[k][c]);
            int64_t tile_end = (jb + j_tile < je) ? jb + j_tile : je;
            int buf = 0;
            for (int64_t c = jb; c < je; c += kWave) {
                if (wave_any(mask.near(c))) {
                    mask.load(c);
                    chunk_loop<true, Op, I>(wl[buf], c, is, mask, kv, p);
                } else {
                    chunk_loop<false, Op, I>(wl[buf], c, is, mask, kv, p);
                }
                if (c + kWave >= tile_end) {
#pragma unroll
                    for (int k = 0; k < I; ++k)
#pragma unroll
                        for (int cc = 0; cc < NC; ++cc) {
                            acc[k][cc].fold(p[k][cc]);
                            acc[k][cc].begin(p[k][cc]);
                        }
                    tile_end = (tile_end + j_tile < je) ? tile_end + j_tile : je;
                }
                (buf ? vwl0 : vwl1)[lane] = g;                               // chunk c + 64
                g = vrec[(c + 2 * kWave < je ? c + 2 * kWave : last) + lane];   // chunk c + 128
                __builtin_amdgcn_wave_barrier();
                buf ^= 1;
            }
        }
    }

}

// j_range with the self pair as the only exclusion.
template <int JS, typename Op, int PREC, int I, typename R, typename IS, typename T>
__device__ __forceinline__ void j_range(const R *__restrict__ rec, int64_t jb, int64_t je,
                                        int j_tile, const IS (&is)[I], const int64_t (&pid)[I],
                                        const PairK<T> &kc, RunSum<PREC> (&acc)[I][Op::NC],
                                        T (&p)[I][Op::NP], R (*wl)[kWave])
{
    SelfMask<I> mask;
#pragma unroll
    for (int k = 0; k < I; ++k) mask.pid[k] = pid[k];
    j_range_masked<JS, Op, PREC, I>(rec, jb, je, j_tile, is, mask, kc, acc, p, wl);
}

}  // namespace nbk
