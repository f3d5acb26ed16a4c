// Symmetric pair tiles for the acceleration and jerk (Table 1's "Gravity (accel &
// jerk)", the GAJ kernel of Section 2, which the Hermite scheme needs): every
// unordered pair {i, j} of a whole system is evaluated once and its terms are
// applied to both particles.  With d = r_j - r_i, w = v_j - v_i and
// s^2 = |d|^2 + eps^2, particle i gets m_j d / s^3 (acceleration),
// m_j u / s^3 with u = w - 3 (d.w) d / s^2 (jerk) and m_j / s (potential).
// Swapping i and j negates d, w and u and leaves d.w and s unchanged, so j gets
// -m_i d / s^3, -m_i u / s^3 and m_i / s: one rsq, one u and the shared
// scalars serve both particles (36 FP32 instructions per unordered pair against
// 28 per ordered pair one-sided).
//
// Decomposition as the symmetric force tiles (symmetric.hip), in one shape: the
// padded records form nblk blocks of 16 chunks of 64 (1024 records); a
// workgroup takes part h of tile (b1, b2), b1 <= b2, of the block grid's upper
// triangle in the XCD-aware strip order (sym_item_of), the tile's j chunks cut
// into `split` parts (1 or 2).  Its 8 waves hold 2 i chunks of b1 each (the 16
// chunks of the block) and sweep the part's j chunks of b2 in rounds: in round
// r wave w takes chunk (w + r) mod jr, and a barrier closes the round.  A
// 64 x 64 mini-tile takes 64 steps; at step t lane l pairs its i particles with
// j = l + t (mod 64) from the wave's LDS slot (the chunk staged twice), and the
// six or seven j sums travel with their particle from lane to lane (four through
// the LDS crossbar, the others by DPP rotations); between rounds they wait in
// LDS.  Diagonal tiles evaluate i chunk k against j chunk q symmetrically when
// q > k, one-sidedly when q == k (the particle's own pair masked) and not at all
// when q < k.
//
// Sums.  The i sums are FP32 mini-tile partials folded into Kahan or FP64 tile
// sums, the j sums FP32 over the part.  Part h of tile (b1, b2) writes one FP32
// partial of the seven sums per row of b1 into slot split b2 + h and one per row
// of its chunks of b2 into slot split b1 + h (a diagonal tile adds both where
// they meet), so every (slot, row) is written once; k_symjerk_reduce adds a
// row's slots in slot order in FP64 (Neumaier) and scales by G (-G for the
// potential), as the one-sided kernel's finish does.
#include "allpairs.h"
#include "kernels.h"
#include "jerk.h"

namespace nbk {

namespace {

constexpr int kSjWaves = 8;                              // waves per workgroup
constexpr int kSjIch = 2;                                // i chunks per wave
constexpr int kSjCrossbar = 4;                           // j sums moved through the LDS crossbar
static_assert(kSjWaves * kSjIch == kSymJerkBlk, "one pass of the waves' i chunks covers a block");

struct alignas(16) SjRec { float x, y, z, m, vx, vy, vz, p0; };

// One unordered pair: i sums p, j sums jv.  MASK (diagonal tiles): wi / wj switch the i and j
// sides on or off, sk marks the particle's own pair.
template <bool POT, bool MASK>
__device__ __forceinline__ void sj_pair(const SjRec &I, const SjRec &J, float eps2, bool sk, float wi, float wj,
                                        float (&p)[7], float (&jv)[7])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
    const float wx = J.vx - I.vx, wy = J.vy - I.vy, wz = J.vz - I.vz;
    float r2 = fma_(dx, dx, eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    float mj = J.m, mi = I.m;
    if (MASK) {
        r2 = sk ? 1.0f : r2;
        mj = sk ? 0.0f : mj * wi;
        mi = mi * wj;
    }
    const float ri = rsqrt_(r2);
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    float dw = dx * wx;
    dw = fma_(dy, wy, dw);
    dw = fma_(dz, wz, dw);
    const float q = (dw * ri2) * -3.0f;
    const float ux = fma_(q, dx, wx), uy = fma_(q, dy, wy), uz = fma_(q, dz, wz);
    const float cj = mj * ri3, ci = mi * ri3;
    p[0] = fma_(cj, dx, p[0]);
    p[1] = fma_(cj, dy, p[1]);
    p[2] = fma_(cj, dz, p[2]);
    p[3] = fma_(cj, ux, p[3]);
    p[4] = fma_(cj, uy, p[4]);
    p[5] = fma_(cj, uz, p[5]);
    jv[0] = fma_(-ci, dx, jv[0]);
    jv[1] = fma_(-ci, dy, jv[1]);
    jv[2] = fma_(-ci, dz, jv[2]);
    jv[3] = fma_(-ci, ux, jv[3]);
    jv[4] = fma_(-ci, uy, jv[4]);
    jv[5] = fma_(-ci, uz, jv[5]);
    if (POT) {
        p[6] = fma_(mj, ri, p[6]);
        jv[6] = fma_(mi, ri, jv[6]);
    }
}

// The value of lane (l + 1) mod 64 by a DPP rotation of the whole wave by one lane (wave_rol:1).
// Every lane reads a valid lane, so no old value is kept and none is set up first.
__device__ __forceinline__ float sj_next_lane_dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}

// One mini-tile: the wave's i chunks (records iv, partials p) against the j chunk staged in st,
// the j sums jv entering and leaving in lane order.
template <bool POT, bool MASK>
__device__ __forceinline__ void sj_minitile(const SjRec *st, const SjRec (&iv)[kSjIch], float eps2, int bp_addr,
                                            float (&p)[kSjIch][7], float (&jv)[7], const float (&wi)[kSjIch],
                                            const float (&wj)[kSjIch], const bool (&self)[kSjIch])
{
    constexpr int NS = POT ? 7 : 6;
    const int lane = lane_id();
#pragma unroll 4
    for (int t = 0; t < kWave; ++t) {
        const SjRec J = st[lane + t];
#pragma unroll
        for (int k = 0; k < kSjIch; ++k)
            sj_pair<POT, MASK>(iv[k], J, eps2, MASK && self[k] && t == 0, MASK ? wi[k] : 1.0f,
                               MASK ? wj[k] : 1.0f, p[k], jv);
        // some sums through the LDS crossbar, the rest on the VALU, so that neither unit
        // carries all the moves
#pragma unroll
        for (int c = 0; c < NS; ++c)
            jv[c] = c < kSjCrossbar ? from_next_lane(bp_addr, jv[c]) : sj_next_lane_dpp(jv[c]);
    }
}

}  // namespace

template <int PREC, bool POT>
__global__ __launch_bounds__(kSjWaves * kWave) __attribute__((amdgpu_waves_per_eu(4)))
void k_symjerk(SymJerkLaunch a)
{
    constexpr int NS = POT ? 7 : 6;
    constexpr int kThreads = kSjWaves * kWave;
    const SjRec *__restrict__ rec = (const SjRec *)a.rec;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int split = a.split;
    const int jr = kSymJerkBlk / split;                    // j chunks of this part (rounds)
    int64_t b1, b2;
    int h;
    if (!sym_item_of(blockIdx.x, a.nblk, 0, sym_tiles(a.nblk), split, b1, b2, h)) return;   // whole workgroup
    const bool diag = b1 == b2;
    const float eps2 = (float)a.eps2;
    const int bp_addr = ((lane + 1) & (kWave - 1)) * 4;

    // j sums of the part's chunks, [jr][NS][64] floats of dynamic LDS
    extern __shared__ float jacc[];
    __shared__ SjRec st_all[kSjWaves][2 * kWave];          // each wave's j chunk, staged twice
    SjRec *st = st_all[w];
    for (int k = threadIdx.x; k < jr * NS * kWave; k += kThreads) jacc[k] = 0.0f;
    const int64_t jrec0 = ((int64_t)b2 * kSymJerkBlk + h * jr) * kWave;   // first record of the part
    const int64_t irec0 = (int64_t)b1 * kSymJerkBlk * kWave;              // first record of block b1
    float4 *const part_i = a.partial + (split * b2 + h) * a.npad * 2;
    float4 *const part_j = a.partial + (split * b1 + h) * a.npad * 2;
    __syncthreads();

    const int aloc = kSjIch * w;                           // local chunks aloc, aloc + 1 of block b1
    SjRec iv[kSjIch];
#pragma unroll
    for (int k = 0; k < kSjIch; ++k) iv[k] = rec[irec0 + (int64_t)(aloc + k) * kWave + lane];
    RunSum<PREC> acc[kSjIch][NS];
    float p[kSjIch][7];
#pragma unroll
    for (int k = 0; k < kSjIch; ++k) p[k][6] = 0.0f;
    // the next round's j record of this lane, loaded a round ahead as two 128-bit vectors
    const float4 *__restrict__ rec4 = (const float4 *)a.rec;
    float4 *st4 = (float4 *)st;
    int64_t gj = jrec0 + (int64_t)(w % jr) * kWave + lane;
    float4 g0 = rec4[2 * gj], g1 = rec4[2 * gj + 1];
    for (int r = 0; r < jr; ++r) {
        const int ql = (w + r) % jr;                       // the part's chunk of this round
        const int q = h * jr + ql;                         // the same chunk, counted in block b2
        st4[2 * lane] = g0;
        st4[2 * lane + 1] = g1;
        st4[2 * (lane + kWave)] = g0;
        st4[2 * (lane + kWave) + 1] = g1;
        gj = jrec0 + (int64_t)((w + r + 1) % jr) * kWave + lane;
        g0 = rec4[2 * gj];
        g1 = rec4[2 * gj + 1];
        float jv[7];
#pragma unroll
        for (int c = 0; c < NS; ++c) jv[c] = jacc[(ql * NS + c) * kWave + lane];
        if (!POT) jv[6] = 0.0f;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < kSjIch; ++k)
#pragma unroll
            for (int c = 0; c < NS; ++c) acc[k][c].begin(p[k][c]);
        if (!diag) {
            const float one[kSjIch] = {1.0f, 1.0f};
            const bool none[kSjIch] = {false, false};
            sj_minitile<POT, false>(st, iv, eps2, bp_addr, p, jv, one, one, none);
        } else {
            // chunk q against i chunk aloc + k: symmetric when q is after it, its own chunk's
            // pairs one-sided when q is it, nothing when q is before it (the wave holding q
            // evaluates those pairs)
            float wi[kSjIch], wj[kSjIch];
            bool self[kSjIch];
            bool any = false;
#pragma unroll
            for (int k = 0; k < kSjIch; ++k) {
                const int rel = q - (aloc + k);
                wi[k] = rel >= 0 ? 1.0f : 0.0f;
                wj[k] = rel > 0 ? 1.0f : 0.0f;
                self[k] = rel == 0;
                any = any || rel >= 0;
            }
            if (any) sj_minitile<POT, true>(st, iv, eps2, bp_addr, p, jv, wi, wj, self);
        }
#pragma unroll
        for (int c = 0; c < NS; ++c) jacc[(ql * NS + c) * kWave + lane] = jv[c];
#pragma unroll
        for (int k = 0; k < kSjIch; ++k)
#pragma unroll
            for (int c = 0; c < NS; ++c) acc[k][c].fold(p[k][c]);
        __syncthreads();
    }
    // i sums: the i-side slot of the rows of block b1, or, on the diagonal, added to the j sums
    // of the same rows where the chunk is one of the part's (no other wave touches it now)
#pragma unroll
    for (int k = 0; k < kSjIch; ++k) {
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = c < NS ? (float)acc[k][c].value() : 0.0f;
        const int c = aloc + k;
        if (!diag || c / jr != h) {
            float4 *o = part_i + 2 * (irec0 + (int64_t)c * kWave + lane);
            o[0] = float4{v[0], v[1], v[2], v[3]};
            o[1] = float4{v[4], v[5], v[6], 0.0f};
        } else {
#pragma unroll
            for (int m = 0; m < NS; ++m) jacc[((c - h * jr) * NS + m) * kWave + lane] += v[m];
        }
    }
    __syncthreads();
    // j sums: the j-side slot of the rows of the part's chunks of block b2
    for (int ql = w; ql < jr; ql += kSjWaves) {
        float v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = m < NS ? jacc[(ql * NS + m) * kWave + lane] : 0.0f;
        float4 *o = part_j + 2 * (jrec0 + (int64_t)ql * kWave + lane);
        o[0] = float4{v[0], v[1], v[2], v[3]};
        o[1] = float4{v[4], v[5], v[6], 0.0f};
    }
}

// Row r of block b: its slot partials in slot order (FP64, Neumaier), then G (and -G for the
// potential).  A tile (b, k), k >= b, holds r on its i side: each of its parts wrote a partial
// for r (slots split k .. split k + split - 1).  A tile (k, b), k < b, holds r on its j side:
// only the part whose chunks include r's wrote one (slot split k + h_r).
template <bool POT>
__global__ __launch_bounds__(256) void k_symjerk_reduce(SymJerkLaunch a)
{
    constexpr int NS = POT ? 7 : 6;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    constexpr int64_t kRows = (int64_t)kSymJerkBlk * kWave;
    const int64_t b = r / kRows;
    const int split = a.split;
    const int hr = (int)((r % kRows) / kWave) / (kSymJerkBlk / split);   // r's part
    NSum v[NS];
    for (int64_t k = 0; k < a.nblk; ++k)
        for (int hh = k < b ? hr : 0; hh < (k < b ? hr + 1 : split); ++hh) {
            const float4 *x = a.partial + 2 * ((split * k + hh) * a.npad + r);
            const float4 x0 = x[0], x1 = x[1];
            const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
            for (int m = 0; m < NS; ++m) v[m].add((double)xs[m]);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a.out_acc[3 * r + c] = a.G * v[c].value();
        a.out_jerk[3 * r + c] = a.G * v[3 + c].value();
    }
    if (POT && a.out_pot) a.out_pot[r] = -a.G * v[6].value();
}

hipError_t launch_symjerk(const SymJerkLaunch &a, hipStream_t s)
{
    if (a.nblk <= 0) return hipSuccess;
    // a launch description that does not match the tiling is refused, never launched
    if (!a.rec || !a.partial || !a.out_acc || !a.out_jerk || (a.split != 1 && a.split != 2) ||
        a.npad != a.nblk * kSymJerkBlk * kWave || a.n > a.npad)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)sym_grid(sym_tiles(a.nblk) * a.split)), block(kSjWaves * kWave);
    const size_t lds = (size_t)(kSymJerkBlk / a.split) * (a.pot ? 7 : 6) * kWave * sizeof(float);
    if (a.prec == P_KAHAN) {
        if (a.pot) hipLaunchKernelGGL((k_symjerk<P_KAHAN, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_symjerk<P_KAHAN, false>), grid, block, lds, s, a);
    } else if (a.prec == P_FP64ACC) {
        if (a.pot) hipLaunchKernelGGL((k_symjerk<P_FP64ACC, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_symjerk<P_FP64ACC, false>), grid, block, lds, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_symjerk_reduce(const SymJerkLaunch &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (a.pot) hipLaunchKernelGGL(k_symjerk_reduce<true>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_symjerk_reduce<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace nbk
