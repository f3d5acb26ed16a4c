// Symmetric pair tiles for the batched entry points: in every system of an
// ensemble each unordered pair {i, j} is evaluated once and its force applied
// to both particles (Newton's third law), the small-system setting of Section
// 3.4 with the pair arithmetic of Eq. 1 (gravity) or one of Table 1's LJC laws.
//
// Decomposition.  The records of system s are padded to nb_s blocks of 256
// (four chunks of 64).  A work unit is one tile (s, b1, b2), b1 <= b2, and one
// wave evaluates it alone (no barriers): it holds the four i chunks of block
// b1 in registers and sweeps the four j chunks of block b2.  For j chunk q a
// 64-step mini-sweep pairs lane l's i particles with j = l + t (mod 64), the
// chunk staged twice in a wave-private LDS slot so that each lane reads its
// record at a constant offset.  The j sums travel with their particle from
// lane to lane (three through the LDS crossbar, the potential's by a DPP
// rotation); after 64 steps lane l holds the sums of j = l, complete for this
// tile, and writes them.  On the diagonal (b1 == b2) i chunk k meets j chunk q
// symmetrically when q > k, one-sidedly (i side only) when q == k, and not at
// all when q < k: the wave holding chunk k evaluated that pair already.
//
// Sums.  The i sums are FP32 mini-sweep partials (4 pairs per step, 64 steps)
// folded into Kahan or FP64 running sums over the tile; the j sums are FP32
// over a mini-sweep (256 terms, the one-sided kernels' tile length).  Tile
// (s, b1, b2) writes one FP32 partial (x, y, z, potential) per row of b1 into
// slot b2 and one per row of b2 into slot b1 of system s's slot buffer
// [nb_s][npad_s] (a diagonal tile adds both into slot b1), so every (slot,
// row) is written exactly once; k_bsym_reduce adds a row's nb_s slots in slot
// order in FP64 (Neumaier) and applies the epilogue.
#include "allpairs.h"
#include "kernels.h"

namespace nbk {

constexpr int kBSymWaves = 4;                       // waves (independent tiles) per workgroup
constexpr int kBSymChunks = kBSymRecords / kWave;   // chunks per block = i chunks per lane

// i-particle state of a lane (position and the law's own parameters; every LJC dielectric has
// the same)
template <int LAW> struct BsI { float x, y, z, qs, sh, se; };
template <> struct BsI<GRAVITY> { float x, y, z, m; };

__device__ __forceinline__ void bs_load(const GravRec<float> *rec, int64_t p, BsI<GRAVITY> &s)
{
    const GravRec<float> r = rec[p];
    s = BsI<GRAVITY>{r.x, r.y, r.z, r.m};
}
template <int LAW>
__device__ __forceinline__ void bs_load(const LjcRec<float> *rec, int64_t p, BsI<LAW> &s)
{
    const LjcRec<float> r = rec[p];
    s = BsI<LAW>{r.x, r.y, r.z, r.qs, r.sh, r.se};
}

// One unordered pair (i of this lane, j of the step): i-side sums p, j-side sums jv.
// SELF: the i side only (a pair of the chunk with itself, seen from both lanes), with the
// particle's own pair (step 0) neutralised.  JSIDE: add the j side.
template <bool POT, bool JSIDE>
__device__ __forceinline__ void bs_pair(const BsI<GRAVITY> &i, const GravRec<float> &J, const PairK<float> &k,
                                        bool self0, float (&p)[4], float (&jv)[4])
{
    const float dx = J.x - i.x, dy = J.y - i.y, dz = J.z - i.z;
    float r2 = fma_(dx, dx, k.eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    float mj = J.m;
    r2 = self0 ? 1.0f : r2;
    mj = self0 ? 0.0f : mj;
    const float ri = rsqrt_(r2);
    const float ri3 = (ri * ri) * ri;
    const float cj = mj * ri3;
    p[0] = fma_(cj, dx, p[0]);
    p[1] = fma_(cj, dy, p[1]);
    p[2] = fma_(cj, dz, p[2]);
    if (POT) p[3] = fma_(mj, ri, p[3]);
    if (JSIDE) {
        const float ci = i.m * ri3;
        jv[0] = fma_(-ci, dx, jv[0]);
        jv[1] = fma_(-ci, dy, jv[1]);
        jv[2] = fma_(-ci, dz, jv[2]);
        if (POT) jv[3] = fma_(i.m, ri, jv[3]);
    }
}

// LJC: F_i += W (r_i - r_j), F_j -= W (r_i - r_j); both get the pair's energy term (2 u_ij for
// the linear dielectric, halved by the epilogue; u_ij for the others), from the scalar part
// of the pair that the one-sided ljc_pair uses (ljc_terms).
template <bool POT, bool JSIDE, int LAW>
__device__ __forceinline__ void bs_pair(const BsI<LAW> &i, const LjcRec<float> &J, const PairK<float> &k,
                                        bool self0, float (&p)[4], float (&jv)[4])
{
    const float dx = J.x - i.x, dy = J.y - i.y, dz = J.z - i.z;
    float r2 = dx * dx;
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    float qq = i.qs * J.qs;
    float e = i.se * J.se;
    r2 = self0 ? 1.0f : r2;
    qq = self0 ? 0.0f : qq;
    e = self0 ? 0.0f : e;
    float W, u = 0.0f;
    ljc_terms<POT, LAW>(r2, qq, e, i.sh + J.sh, k, W, u);
    p[0] = fma_(-W, dx, p[0]);
    p[1] = fma_(-W, dy, p[1]);
    p[2] = fma_(-W, dz, p[2]);
    if (POT) p[3] += u;
    if (JSIDE) {
        jv[0] = fma_(W, dx, jv[0]);
        jv[1] = fma_(W, dy, jv[1]);
        jv[2] = fma_(W, dz, jv[2]);
        if (POT) jv[3] += u;
    }
}

// One mini-sweep: the wave's four i chunks against the j chunk staged in `st`.  DIAG: i chunk
// k pairs symmetrically only when q > k, one-sidedly when q == k, and not when q < k.
template <int LAW, bool POT, bool DIAG, typename R>
__device__ __forceinline__ void bs_sweep(const R *st, const BsI<LAW> (&iv)[kBSymChunks], const PairK<float> &kc, int q,
                                         int bp_addr, float (&p)[kBSymChunks][4], float (&jv)[4])
{
    const int lane = lane_id();
#pragma unroll 4
    for (int t = 0; t < kWave; ++t) {
        const R J = st[lane + t];
#pragma unroll
        for (int k = 0; k < kBSymChunks; ++k) {
            if (!DIAG) {
                bs_pair<POT, true>(iv[k], J, kc, false, p[k], jv);
            } else if (k < q) {
                bs_pair<POT, true>(iv[k], J, kc, false, p[k], jv);
            } else if (k == q) {
                bs_pair<POT, false>(iv[k], J, kc, t == 0, p[k], jv);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) jv[c] = from_next_lane(bp_addr, jv[c]);
        if (POT) jv[3] = from_next_lane_dpp(jv[3]);
    }
}

// waves per SIMD the register allocation aims at: four with Kahan sums (128 VGPRs), three with
// FP64 sums or the sigmoidal dielectric's longer sequence
template <int LAW, int PREC> constexpr int bsym_waves_per_eu() { return PREC == P_KAHAN && LAW != LJC_SIG ? 4 : 3; }

template <int LAW, int PREC, bool POT>
__global__ __launch_bounds__(kBSymWaves * kWave) __attribute__((amdgpu_waves_per_eu(bsym_waves_per_eu<LAW, PREC>()))) void k_bsym(BSymLaunch a)
{
    using R = typename RecOf<float, LAW>::type;
    const R *__restrict__ rec = (const R *)a.rec;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t u = (int64_t)blockIdx.x * kBSymWaves + w;
    __shared__ R st_all[kBSymWaves][2 * kWave];                 // each wave's j chunk, staged twice
    __shared__ float4 jd_all[kBSymWaves][kBSymChunks][kWave];   // diagonal tiles: the j sums of block b1
    if (u >= a.n_units) return;                                 // whole wave; the kernel has no barriers
    const int32_t *un = a.units + 4 * u;
    const int64_t s = un[0], b1 = un[1], b2 = un[2];
    if (s < 0 || s >= a.n_systems) return;
    const int64_t po = a.poff[s];
    const int64_t npad = a.poff[s + 1] - po;
    const int64_t nb = npad / kBSymRecords;
    if (b1 < 0 || b2 < b1 || b2 >= nb) return;                  // never index outside the tables
    const bool diag = b1 == b2;
    const int64_t irec0 = po + b1 * kBSymRecords, jrec0 = po + b2 * kBSymRecords;
    float4 *slots = a.partial + a.systab[3 * s + 2];            // [nb][npad] of system s
    R *st = st_all[w];
    PairK<float> kc;
    kc.eps2 = (float)a.eps2;
    kc.za = (float)a.zeta[0];
    kc.zb = (float)a.zeta[1];
    kc.zc = (float)a.zeta[2];
    kc.zd = (float)a.zeta[3];
    kc.za3 = (float)(3.0 * a.zeta[0]);
    kc.zb2 = (float)(2.0 * a.zeta[1]);
    const int bp_addr = ((lane + 1) & (kWave - 1)) * 4;

    BsI<LAW> iv[kBSymChunks];
#pragma unroll
    for (int k = 0; k < kBSymChunks; ++k) bs_load(rec, irec0 + k * kWave + lane, iv[k]);
    RunSum<PREC> acc[kBSymChunks][4];
    float p[kBSymChunks][4];
    // the next chunk's record of this lane, loaded a chunk ahead as 128-bit vectors (so that it
    // stays in registers)
    constexpr int V = sizeof(R) / sizeof(float4);               // 1 (gravity) or 2 (LJC)
    static_assert(V == 1 || V == 2, "records of one or two 128-bit vectors");
    const float4 *__restrict__ rec4 = (const float4 *)a.rec;
    float4 *st4 = (float4 *)st;
    float4 g0 = rec4[(jrec0 + lane) * V], g1 = V == 2 ? rec4[(jrec0 + lane) * V + 1] : float4{0, 0, 0, 0};
    for (int q = 0; q < kBSymChunks; ++q) {
        st4[lane * V] = g0;
        st4[(lane + kWave) * V] = g0;
        if (V == 2) {
            st4[lane * V + 1] = g1;
            st4[(lane + kWave) * V + 1] = g1;
        }
        // the next chunk (the last round reloads its own, unused)
        const int64_t qn = q + 1 < kBSymChunks ? q + 1 : q;
        g0 = rec4[(jrec0 + qn * kWave + lane) * V];
        if (V == 2) g1 = rec4[(jrec0 + qn * kWave + lane) * V + 1];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < kBSymChunks; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[k][c].begin(p[k][c]);
        float jv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (!diag) bs_sweep<LAW, POT, false>(st, iv, kc, q, bp_addr, p, jv);
        else bs_sweep<LAW, POT, true>(st, iv, kc, q, bp_addr, p, jv);
#pragma unroll
        for (int k = 0; k < kBSymChunks; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[k][c].fold(p[k][c]);
        const float4 jq = float4{jv[0], jv[1], jv[2], POT ? jv[3] : 0.0f};
        if (!diag) slots[b1 * npad + b2 * kBSymRecords + q * kWave + lane] = jq;   // slot b1, rows of b2
        else jd_all[w][q][lane] = jq;
        __builtin_amdgcn_wave_barrier();                         // the slot is restaged next
    }
    // i sums: slot b2 of the rows of block b1 (on the diagonal with the j sums of the same rows)
#pragma unroll
    for (int k = 0; k < kBSymChunks; ++k) {
        float4 v = float4{(float)acc[k][0].value(), (float)acc[k][1].value(), (float)acc[k][2].value(),
                          POT ? (float)acc[k][3].value() : 0.0f};
        if (diag) {
            const float4 t = jd_all[w][k][lane];
            v = float4{v.x + t.x, v.y + t.y, v.z + t.z, v.w + t.w};
        }
        slots[b2 * npad + b1 * kBSymRecords + k * kWave + lane] = v;
    }
}

// Row block red[blockIdx.x] = (s, rb) of 256 rows: each row adds its system's nb_s slots in
// slot order (FP64, Neumaier) and applies the epilogue.
__global__ __launch_bounds__(kBSymRecords) void k_bsym_reduce(BSymLaunch a)
{
    const int64_t s = a.red[2 * blockIdx.x], rb = a.red[2 * blockIdx.x + 1];
    const int64_t l = rb * kBSymRecords + threadIdx.x;
    const int64_t o = a.off[s];
    if (l >= a.off[s + 1] - o) return;
    const int64_t npad = a.poff[s + 1] - a.poff[s];
    const int64_t nb = npad / kBSymRecords;
    const float4 *__restrict__ slots = a.partial + a.systab[3 * s + 2] + l;
    NSum v[4];
    int64_t k = 0;
    for (; k + 4 <= nb; k += 4) {            // four slots' loads in flight before their sums
        float4 x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = slots[(k + t) * npad];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v[0].add((double)x[t].x);
            v[1].add((double)x[t].y);
            v[2].add((double)x[t].z);
            v[3].add((double)x[t].w);
        }
    }
    for (; k < nb; ++k) {
        const float4 x = slots[k * npad];
        v[0].add((double)x.x);
        v[1].add((double)x.y);
        v[2].add((double)x.z);
        v[3].add((double)x.w);
    }
    const int64_t r = o + l;
    const Epilogue &e = a.epi;
    e.out_force[3 * r] = e.fscale * v[0].value();
    e.out_force[3 * r + 1] = e.fscale * v[1].value();
    e.out_force[3 * r + 2] = e.fscale * v[2].value();
    if (a.pot && e.out_pot) e.out_pot[r] = e.pscale * v[3].value();
}

template <int LAW, int PREC>
static void bsym_go(const BSymLaunch &a, const dim3 &grid, const dim3 &block, hipStream_t s)
{
    if (a.pot) hipLaunchKernelGGL((k_bsym<LAW, PREC, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_bsym<LAW, PREC, false>), grid, block, 0, s, a);
}

bool bsym_supported(int law, int prec)
{
    return (law == GRAVITY || law == LJC || law == LJC_CONST || law == LJC_SIG) &&
           (prec == P_KAHAN || prec == P_FP64ACC);
}

hipError_t launch_bsym(const BSymLaunch &a, hipStream_t s)
{
    if (a.n_units <= 0) return hipSuccess;
    if (!bsym_supported(a.law, a.prec)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.n_units + kBSymWaves - 1) / kBSymWaves)), block(kBSymWaves * kWave);
    const bool kahan = a.prec == P_KAHAN;
    switch (a.law) {
    case GRAVITY: kahan ? bsym_go<GRAVITY, P_KAHAN>(a, grid, block, s) : bsym_go<GRAVITY, P_FP64ACC>(a, grid, block, s); break;
    case LJC: kahan ? bsym_go<LJC, P_KAHAN>(a, grid, block, s) : bsym_go<LJC, P_FP64ACC>(a, grid, block, s); break;
    case LJC_CONST:
        kahan ? bsym_go<LJC_CONST, P_KAHAN>(a, grid, block, s) : bsym_go<LJC_CONST, P_FP64ACC>(a, grid, block, s);
        break;
    default: kahan ? bsym_go<LJC_SIG, P_KAHAN>(a, grid, block, s) : bsym_go<LJC_SIG, P_FP64ACC>(a, grid, block, s);
    }
    return hipGetLastError();
}

hipError_t launch_bsym_reduce(const BSymLaunch &a, hipStream_t s)
{
    if (a.n_red <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsym_reduce, dim3((unsigned)a.n_red), dim3(kBSymRecords), 0, s, a);
    return hipGetLastError();
}

}  // namespace nbk
