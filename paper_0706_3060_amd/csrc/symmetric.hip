// Symmetric all-pairs tiles: every unordered pair {i, j} is evaluated once
// and its force is applied to both particles (Newton's third law), so one
// reciprocal square root (or reciprocal) serves two interactions.  The pair
// operators that share the tiles: gravity's forces and potentials, gravity's
// position adjoint, and the forces and energies of the three LJC dielectrics.
//
// Decomposition.  The padded records form nblk blocks of blk chunks of 64
// (blk = 16 or 32).  Each workgroup takes one tile (b1, b2), b1 <= b2, of the
// upper triangle of the block grid (in the XCD-aware strip order of
// sym_tile_of; a launch covers the whole triangle or one share of it): the
// pairs between the rows of block b1 and the rows of block b2 (on the
// diagonal, b1 == b2, each unordered pair once).  Its waves hold the i chunks
// of a pass in registers (8 waves of 2 chunks or 4 waves of 4: 16 chunks per
// pass, two passes for blk = 32; four chunks per wave halve the cross-lane
// moves per pair at the cost of registers) and sweep the j chunks of b2 in
// rounds: in round r wave w takes j chunk (w + r) mod blk, so no two waves
// touch one j chunk in the same round, and a barrier closes every round.  The
// order in which the contributions of the waves reach a j chunk is therefore
// fixed, and the sums repeat bit for bit.
//
// A 64 x 64 mini-tile (one i chunk against one j chunk) takes 64 steps.  At
// step s lane l pairs its i particle with j = l + s (mod 64): the j records
// are staged twice in a wave-private LDS slot, so each lane reads its own
// record at a constant offset.  The j-side sums of the mini-tile travel with
// their particle: after each step every lane takes its right neighbour's four
// sums (three through the LDS crossbar with ds_bpermute, the potential's with a
// DPP wave rotation), so after 64 steps lane l holds the sums of j = l again.
// Between mini-tiles the j sums of a tile live in LDS (FP32, one slot per j of
// block b2); the i sums are FP32 mini-tile partials folded into Kahan or FP64
// running sums (the tile-level compensation of the one-sided kernels).
//
// Output.  Tile (b1, b2) writes one FP32 partial (x, y, z, potential) per row
// of b1 into slot b2 and one per row of b2 into slot b1 of the partial buffer
// [nblk][npad][4] (a diagonal tile adds its i and j sums and writes slot b1),
// so every (slot, row) is written exactly once.  k_sym_reduce then adds the
// nblk slots of each row in slot order in FP64 (Neumaier) and applies the
// epilogue (scales, leapfrog kick).
//
// Parts.  For systems that give few tiles per CU, the j chunks of each tile can
// be cut into `split` parts (2 or 4) run by workgroups of their own, so that
// the launch's last round of workgroups is shorter.  Part h sweeps chunks
// h blk/split .. (h + 1) blk/split - 1 of b2 with all the i chunks of b1; its
// i sums go to slot split b2 + h and the j sums of its chunks' rows to slot
// split b1 + h of a [split nblk][npad][4] buffer.  The reduction adds, in slot
// order, every part's slot of the tiles holding a row on their i side and the
// one part's slot of the tiles holding it on their j side.
#include "allpairs.h"
#include "kernels.h"

namespace nbk {


// The pair operators.  SYM_FORCE: Eq. 1 (i side m_j r^-3 d, j side -m_i r^-3 d, potentials
// m_j / r and m_i / r).  SYM_HVP: the position adjoint of Eq. 1 (a Hessian-vector product):
// with w = m_i g_j - m_j g_i, the i side adds t = s^-3 (w - 3 s^-2 (d.w) d) and the j side -t
// (swapping i and j negates both w and d).  wi / wj switch the i and j sides on or off (diagonal
// tiles); sk marks the particle's own pair, which contributes nothing.
template <int OP> struct SymRecOf { using type = GravRec<float>; };
template <> struct SymRecOf<SYM_HVP> { using type = GravAdjRec<float>; };
template <> struct SymRecOf<SYM_LJC> { using type = LjcRec<float>; };
template <> struct SymRecOf<SYM_LJC_CONST> { using type = LjcRec<float>; };
template <> struct SymRecOf<SYM_LJC_SIG> { using type = LjcRec<float>; };
// the Table 1 law of an LJC operator
template <int OP> constexpr int sym_ljc_law() { return OP == SYM_LJC ? LJC : (OP == SYM_LJC_CONST ? LJC_CONST : LJC_SIG); }

template <bool POT, bool MASK>
__device__ __forceinline__ void sym_pair_grav(const GravRec<float> &I, const GravRec<float> &J, float eps2, bool sk,
                                              float wi, float wj, float (&p)[4], float (&jv)[4])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
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
    const float ri3 = (ri * ri) * ri;
    const float cj = mj * ri3, ci = mi * ri3;
    p[0] = fma_(cj, dx, p[0]);
    p[1] = fma_(cj, dy, p[1]);
    p[2] = fma_(cj, dz, p[2]);
    jv[0] = fma_(-ci, dx, jv[0]);
    jv[1] = fma_(-ci, dy, jv[1]);
    jv[2] = fma_(-ci, dz, jv[2]);
    if (POT) {
        p[3] = fma_(mj, ri, p[3]);
        jv[3] = fma_(mi, ri, jv[3]);
    }
}

template <bool MASK>
__device__ __forceinline__ void sym_pair_hvp(const GravAdjRec<float> &I, const GravAdjRec<float> &J, float eps2,
                                             bool sk, float wi, float wj, float (&p)[4], float (&jv)[4])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
    float r2 = fma_(dx, dx, eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    if (MASK) r2 = sk ? 1.0f : r2;
    float ri = rsqrt_(r2);
    if (MASK) ri = sk ? 0.0f : ri;
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    const float wx = fma_(-J.m, I.gx, I.m * J.gx);
    const float wy = fma_(-J.m, I.gy, I.m * J.gy);
    const float wz = fma_(-J.m, I.gz, I.m * J.gz);
    float dw = dx * wx;
    dw = fma_(dy, wy, dw);
    dw = fma_(dz, wz, dw);
    const float u = (ri2 * 3.0f) * dw;
    float tx = ri3 * fma_(-u, dx, wx), ty = ri3 * fma_(-u, dy, wy), tz = ri3 * fma_(-u, dz, wz);
    if (MASK) {
        p[0] = fma_(wi, tx, p[0]);
        p[1] = fma_(wi, ty, p[1]);
        p[2] = fma_(wi, tz, p[2]);
        jv[0] = fma_(-wj, tx, jv[0]);
        jv[1] = fma_(-wj, ty, jv[1]);
        jv[2] = fma_(-wj, tz, jv[2]);
    } else {
        p[0] += tx;
        p[1] += ty;
        p[2] += tz;
        jv[0] -= tx;
        jv[1] -= ty;
        jv[2] -= tz;
    }
}

// The LJC operators: Table 1's LJC pair is symmetric in its two atoms (ljc_terms), so one W
// and one energy term serve both: F_i -= W d and F_j += W d (d = r_j - r_i), and both energy
// sums get the pair's term (2 u_ij for the linear dielectric, halved by the epilogue; u_ij for
// the others), as the one-sided ljc_pair computes them.
template <int LAW, bool POT, bool MASK>
__device__ __forceinline__ void sym_pair_ljc(const LjcRec<float> &I, const LjcRec<float> &J, const PairK<float> &k,
                                             bool sk, float wi, float wj, float (&p)[4], float (&jv)[4])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
    float r2 = dx * dx;
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    float qq = I.qs * J.qs;
    float e = I.se * J.se;
    if (MASK) {
        r2 = sk ? 1.0f : r2;
        qq = sk ? 0.0f : qq;
        e = sk ? 0.0f : e;
    }
    float W, u = 0.0f;
    ljc_terms<POT, LAW>(r2, qq, e, I.sh + J.sh, k, W, u);
    if (MASK) {
        const float Wi = W * wi, Wj = W * wj;
        p[0] = fma_(-Wi, dx, p[0]);
        p[1] = fma_(-Wi, dy, p[1]);
        p[2] = fma_(-Wi, dz, p[2]);
        jv[0] = fma_(Wj, dx, jv[0]);
        jv[1] = fma_(Wj, dy, jv[1]);
        jv[2] = fma_(Wj, dz, jv[2]);
        if (POT) {
            p[3] = fma_(u, wi, p[3]);
            jv[3] = fma_(u, wj, jv[3]);
        }
    } else {
        p[0] = fma_(-W, dx, p[0]);
        p[1] = fma_(-W, dy, p[1]);
        p[2] = fma_(-W, dz, p[2]);
        jv[0] = fma_(W, dx, jv[0]);
        jv[1] = fma_(W, dy, jv[1]);
        jv[2] = fma_(W, dz, jv[2]);
        if (POT) {
            p[3] += u;
            jv[3] += u;
        }
    }
}

template <int OP, bool POT, bool MASK, typename R>
__device__ __forceinline__ void sym_pair(const R &I, const R &J, const PairK<float> &k, bool sk, float wi, float wj,
                                         float (&p)[4], float (&jv)[4])
{
    if constexpr (OP == SYM_FORCE) sym_pair_grav<POT, MASK>(I, J, k.eps2, sk, wi, wj, p, jv);
    else if constexpr (OP == SYM_HVP) sym_pair_hvp<MASK>(I, J, k.eps2, sk, wi, wj, p, jv);
    else sym_pair_ljc<sym_ljc_law<OP>(), POT, MASK>(I, J, k, sk, wi, wj, p, jv);
}

// One mini-tile: the wave's ICH i chunks (records iv, running partials p) against the j chunk in
// the wave's LDS slot `st` (staged twice), with the j sums jv entering and leaving in lane order.
// MASK (diagonal tiles only): per i slot k, wi[k] / wj[k] switch the i and j sides on or off and
// self[k] marks a slot whose i chunk is the j chunk itself, whose pair at step 0 is the particle
// with itself.
template <int OP, int ICH, bool POT, bool MASK, typename R>
__device__ __forceinline__ void sym_minitile(const R *st, const R (&iv)[ICH], const PairK<float> &kc, int bp_addr,
                                             float (&p)[ICH][4], float (&jv)[4], const float (&wi)[ICH],
                                             const float (&wj)[ICH], const bool (&self)[ICH])
{
    const int lane = lane_id();
#pragma unroll(16 / ICH)
    for (int s = 0; s < kWave; ++s) {
        const R J = st[lane + s];
#pragma unroll
        for (int k = 0; k < ICH; ++k)
            sym_pair<OP, POT, MASK>(iv[k], J, kc, MASK && self[k] && s == 0, MASK ? wi[k] : 1.0f,
                                    MASK ? wj[k] : 1.0f, p[k], jv);
        // most sums move through the LDS crossbar, one on the VALU: the two units share the
        // moves (2 % faster at N = 2^20 than four crossbar moves; more DPP moves are slower)
        if (OP != SYM_HVP) {
#pragma unroll
            for (int c = 0; c < 3; ++c) jv[c] = from_next_lane(bp_addr, jv[c]);
            if (POT) jv[3] = from_next_lane_dpp(jv[3]);
        } else {
            jv[0] = from_next_lane(bp_addr, jv[0]);
            jv[1] = from_next_lane(bp_addr, jv[1]);
            jv[2] = from_next_lane_dpp(jv[2]);
        }
    }
}

// Waves per SIMD the register allocation aims at: 8-wave workgroups fit three per CU at six
// waves per SIMD (80 VGPRs), 4-wave ones four at four (128 VGPRs).  The longer pair sequences
// (the adjoint, the sigmoidal dielectric, and the 8-wave LJC sequences with the energy) need
// more registers than that without spilling; they aim one workgroup lower.
template <int OP, bool POT, int WAVES> constexpr int sym_waves_per_eu()
{
    if (OP == SYM_HVP || OP == SYM_LJC_SIG) return WAVES == 8 ? 4 : 3;
    if (OP >= SYM_LJC && POT && WAVES == 8) return 4;
    return WAVES == 8 ? 6 : 4;
}

// WAVES waves per workgroup hold ICH i chunks each: (8, 2) or (4, 4), a pass of 16 i chunks.
template <int OP, int PREC, bool POT, int WAVES, int ICH>
__global__ __launch_bounds__(WAVES * kWave)
__attribute__((amdgpu_waves_per_eu(sym_waves_per_eu<OP, POT, WAVES>())))
void k_sym(SymLaunch a)
{
    using R = typename SymRecOf<OP>::type;
    constexpr int kThreads = WAVES * kWave;
    constexpr int kPass = WAVES * ICH;                     // i chunks of one pass
    const R *__restrict__ rec = (const R *)a.rec;
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int blk = a.blk;
    const int split = a.split;
    const int jr = blk / split;                            // j chunks of this part (rounds of a pass)
    int64_t b1, b2;
    int h;                                                 // the part: j chunks h jr .. h jr + jr - 1 of b2
    if (!sym_item_of(blockIdx.x, a.nblk, a.t0, a.count, split, b1, b2, h)) return;   // whole workgroup
    const bool diag = b1 == b2;
    PairK<float> kc;
    kc.eps2 = (float)a.eps2;
    kc.za = (float)a.zeta[0];
    kc.zb = (float)a.zeta[1];
    kc.zc = (float)a.zeta[2];
    kc.zd = (float)a.zeta[3];
    kc.za3 = (float)(3.0 * a.zeta[0]);
    kc.zb2 = (float)(2.0 * a.zeta[1]);
    const int bp_addr = ((lane + 1) & (kWave - 1)) * 4;

    // j sums of the part's chunks of block b2: jr x 64 float4 of dynamic LDS (sized by the
    // launch, so that small parts leave room for more workgroups per CU)
    extern __shared__ float4 jacc[];
    __shared__ R st_all[WAVES][2 * kWave];                // each wave's j chunk, staged twice
    R *st = st_all[w];
    for (int k = threadIdx.x; k < jr * kWave; k += kThreads) jacc[k] = float4{0, 0, 0, 0};
    const int64_t jrec0 = (b2 * blk + h * jr) * kWave;     // first record of the part's j chunks
    const int64_t irec0 = b1 * blk * kWave;                // first record of block b1
    // slot of this part's partials: rows of b1 (the i side) in slot split b2 + h, rows of the
    // part's chunks of b2 (the j side) in slot split b1 + h
    float4 *const part_i = a.partial + (split * b2 + h) * a.npad;
    float4 *const part_j = a.partial + (split * b1 + h) * a.npad;
    __syncthreads();

    for (int pass = 0; pass < blk / kPass; ++pass) {
        const int aloc = pass * kPass + ICH * w;           // local chunks aloc .. aloc + ICH - 1 of block b1
        R iv[ICH];
#pragma unroll
        for (int k = 0; k < ICH; ++k) iv[k] = rec[irec0 + (int64_t)(aloc + k) * kWave + lane];
        RunSum<PREC> acc[ICH][4];
        float p[ICH][4];
        // the next round's j record of this lane, loaded a round ahead (as one or two 128-bit
        // vectors, so that it stays in registers)
        constexpr int V = sizeof(R) / sizeof(float4);
        static_assert(V == 1 || V == 2, "records of one or two 128-bit vectors");
        const float4 *__restrict__ rec4 = (const float4 *)a.rec;
        float4 *st4 = (float4 *)st;
        int64_t gj = jrec0 + (int64_t)(w % jr) * kWave + lane;
        float4 g0 = rec4[gj * V], g1 = V == 2 ? rec4[gj * V + 1] : float4{0, 0, 0, 0};
        for (int r = 0; r < jr; ++r) {
            const int ql = (w + r) % jr;                   // the part's chunk of this round
            const int q = h * jr + ql;                     // the same chunk, counted in block b2
            st4[lane * V] = g0;
            st4[(lane + kWave) * V] = g0;
            if (V == 2) {
                st4[lane * V + 1] = g1;
                st4[(lane + kWave) * V + 1] = g1;
            }
            gj = jrec0 + (int64_t)((w + r + 1) % jr) * kWave + lane;
            g0 = rec4[gj * V];
            if (V == 2) g1 = rec4[gj * V + 1];
            const float4 j4 = jacc[ql * kWave + lane];
            float jv[4] = {j4.x, j4.y, j4.z, j4.w};
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < ICH; ++k)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[k][c].begin(p[k][c]);
            if (!diag) {
                float one[ICH];
                bool none[ICH];
#pragma unroll
                for (int k = 0; k < ICH; ++k) {
                    one[k] = 1.0f;
                    none[k] = false;
                }
                sym_minitile<OP, ICH, POT, false>(st, iv, kc, bp_addr, p, jv, one, one, none);
            } else {
                // chunk q against i chunk aloc + k: symmetric when q is after it, its own
                // chunk's pairs one-sided when q is it, nothing when q is before it (that pair
                // is evaluated by the wave holding q)
                float wi[ICH], wj[ICH];
                bool self[ICH];
#pragma unroll
                for (int k = 0; k < ICH; ++k) {
                    const int rel = q - (aloc + k);
                    wi[k] = rel >= 0 ? 1.0f : 0.0f;
                    wj[k] = rel > 0 ? 1.0f : 0.0f;
                    self[k] = rel == 0;
                }
                sym_minitile<OP, ICH, POT, true>(st, iv, kc, bp_addr, p, jv, wi, wj, self);
            }
            jacc[ql * kWave + lane] = float4{jv[0], jv[1], jv[2], POT ? jv[3] : 0.0f};
#pragma unroll
            for (int k = 0; k < ICH; ++k)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[k][c].fold(p[k][c]);
            __syncthreads();
        }
        // i sums of this pass: the i-side slot of the rows of block b1, or, on the diagonal,
        // added to the j sums of the same rows where the chunk is one of the part's (no other
        // wave touches these chunks now); the diagonal's other chunks have i sums only
#pragma unroll
        for (int k = 0; k < ICH; ++k) {
            const float4 v = float4{(float)acc[k][0].value(), (float)acc[k][1].value(),
                                    (float)acc[k][2].value(), POT ? (float)acc[k][3].value() : 0.0f};
            const int c = aloc + k;
            if (!diag || c / jr != h) {
                part_i[irec0 + (int64_t)c * kWave + lane] = v;
            } else {
                float4 &t = jacc[(c - h * jr) * kWave + lane];
                t = float4{t.x + v.x, t.y + v.y, t.z + v.z, t.w + v.w};
            }
        }
        __syncthreads();
    }
    // j sums: the j-side slot of the rows of the part's chunks of block b2
    for (int ql = w; ql < jr; ql += WAVES) part_j[jrec0 + (int64_t)ql * kWave + lane] = jacc[ql * kWave + lane];
}

// Row r of block b: its slot partials in slot order (FP64, Neumaier), then the epilogue.  A
// tile (b, k), k >= b, holds r on its i side: each of its parts wrote a partial for r (slots
// split k .. split k + split - 1).  A tile (k, b), k < b, holds r on its j side: only the part
// whose chunks include r's wrote one (slot split k + h_r).  When the launch covered one share
// of the tiles, only the tiles in the share count (the test is the same for every row of a
// workgroup: 256 rows lie in one block).
__global__ __launch_bounds__(256) void k_sym_reduce(SymLaunch a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    NSum v[4];
    const float4 *__restrict__ part = a.partial;
    const bool whole = a.t0 == 0 && a.count == sym_tiles(a.nblk);
    const int64_t b = r / ((int64_t)a.blk * kWave);
    const int split = a.split;
    const int hr = (int)((r % ((int64_t)a.blk * kWave)) / kWave) / (a.blk / split);   // r's part
    for (int64_t k = 0; k < a.nblk; ++k) {
        if (!whole) {
            const int64_t t = b <= k ? sym_index_of(b, k, a.nblk) : sym_index_of(k, b, a.nblk);
            if (t < a.t0 || t >= a.t0 + a.count) continue;
        }
        for (int hh = k < b ? hr : 0; hh < (k < b ? hr + 1 : split); ++hh) {
            const float4 x = part[(split * k + hh) * a.npad + r];
            v[0].add((double)x.x);
            v[1].add((double)x.y);
            v[2].add((double)x.z);
            v[3].add((double)x.w);
        }
    }
    const Epilogue &e = a.epi;
    double f0 = e.fscale * v[0].value(), f1 = e.fscale * v[1].value(), f2 = e.fscale * v[2].value();
    if (e.kick) {
        const double s = e.inv_mass ? e.inv_mass[r] : 1.0;
        f0 *= s;
        f1 *= s;
        f2 *= s;
        e.vel[3 * r] += e.half_dt * f0;
        e.vel[3 * r + 1] += e.half_dt * f1;
        e.vel[3 * r + 2] += e.half_dt * f2;
    }
    e.out_force[3 * r] = f0;
    e.out_force[3 * r + 1] = f1;
    e.out_force[3 * r + 2] = f2;
    if (a.pot && e.out_pot) e.out_pot[r] = e.pscale * v[3].value();
}

template <int OP, int WAVES, int ICH>
static hipError_t launch_sym_op(const SymLaunch &a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    constexpr bool kPot = OP != SYM_HVP;                  // no potential for the adjoint
    if (a.prec == P_KAHAN) {
        if (kPot && a.pot) hipLaunchKernelGGL((k_sym<OP, P_KAHAN, kPot, WAVES, ICH>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_sym<OP, P_KAHAN, false, WAVES, ICH>), grid, block, lds, s, a);
    } else if (a.prec == P_FP64ACC) {
        if (kPot && a.pot) hipLaunchKernelGGL((k_sym<OP, P_FP64ACC, kPot, WAVES, ICH>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_sym<OP, P_FP64ACC, false, WAVES, ICH>), grid, block, lds, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int WAVES, int ICH>
static hipError_t launch_sym_shape(const SymLaunch &a, hipStream_t s)
{
    const dim3 grid((unsigned)sym_grid(a.count * a.split)), block(WAVES * kWave);
    const size_t lds = (size_t)(a.blk / a.split) * kWave * sizeof(float4);   // the j sums of one part
    switch (a.op) {
    case SYM_FORCE: return launch_sym_op<SYM_FORCE, WAVES, ICH>(a, grid, block, lds, s);
    case SYM_HVP: return launch_sym_op<SYM_HVP, WAVES, ICH>(a, grid, block, lds, s);
    case SYM_LJC: return launch_sym_op<SYM_LJC, WAVES, ICH>(a, grid, block, lds, s);
    case SYM_LJC_CONST: return launch_sym_op<SYM_LJC_CONST, WAVES, ICH>(a, grid, block, lds, s);
    case SYM_LJC_SIG: return launch_sym_op<SYM_LJC_SIG, WAVES, ICH>(a, grid, block, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sym(const SymLaunch &a, hipStream_t s)
{
    if (a.nblk <= 0 || a.count <= 0) return hipSuccess;
    if (a.blk % 16 != 0 || a.blk > kSymMaxBlk || a.npad != (int64_t)a.nblk * a.blk * kWave ||
        a.t0 < 0 || a.t0 + a.count > sym_tiles(a.nblk))
        return hipErrorInvalidValue;
    // j parts of at least as many chunks as the workgroup has waves (distinct chunks per round)
    const int waves = a.ich == 2 ? 8 : 4;
    if ((a.split != 1 && a.split != 2 && a.split != 4) || a.blk % a.split != 0 || a.blk / a.split < waves)
        return hipErrorInvalidValue;
    if (a.ich == 2) return launch_sym_shape<8, 2>(a, s);
    if (a.ich == 4) return launch_sym_shape<4, 4>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sym_reduce(const SymLaunch &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sym_reduce, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nbk
