// Symmetric pair tiles for the batched adjoint (the backward of the batched
// forces under a loss L(F), with g_i = dL/dF_i): in every system of an ensemble
// each unordered pair {i, j} is evaluated once and its adjoint terms are applied
// to both particles.  Not in the paper: the derivatives of Eq. 1 (gravity's
// position adjoint, a Hessian-vector product) and of Table 1's LJC(linear)
// (positions, charges, sigma and epsilon).
//
// Both are symmetric per pair.  Gravity: with w = m_i g_j - m_j g_i and
// d = r_j - r_i, the term t = s^-3 (w - 3 s^-2 (d.w) d) of particle i is minus
// that of particle j.  LJC: with u = g_j - g_i, the position term
// P = -W u + W' (d.u) d (W the force factor, W' its r^2 derivative factor) of i
// is minus that of j; the charge, sigma and epsilon terms share the scalar
// x (d.u): i gets qs_j A, B and se_j C, j gets qs_i A, B and se_i C.
//
// Decomposition as the batched forward tiles (bsym.hip): one wave per tile
// (s, b1, b2) of two 256-record blocks of a system, listed by the host plan, no
// barriers.  The wave holds i chunks of b1 in registers (all four for gravity's
// three sums, two at a time for LJC's six) and sweeps the four j chunks of b2
// in 64-step mini-sweeps: lane l pairs its i particles with j = l + t (mod 64),
// the chunk staged twice in a wave-private LDS slot; the j sums travel with
// their particle from lane to lane and wait in LDS between chunks and passes.
// Diagonal tiles evaluate i chunk k against j chunk q symmetrically when q > k,
// one-sidedly when q == k, not at all when q < k.
//
// Sums.  The i sums are FP32 mini-sweep partials folded into Kahan or FP64 sums
// over the tile; the j sums are FP32 over the tile.  Tile (s, b1, b2) writes
// one FP32 partial of each sum per row of b1 into slot b2 and one per row of b2
// into slot b1 of system s's slots (a diagonal tile adds both into slot b1);
// k_bsym_adj_reduce adds a row's slots in slot order in FP64 (Neumaier) and
// writes the gradients.
#include "allpairs.h"
#include "kernels.h"
#include "adjoint.h"

namespace nbk {

namespace {

constexpr int kWaves = 4;                          // waves (independent tiles) per workgroup
constexpr int kChunks = kBSymRecords / kWave;      // chunks per block

// The records as the tiles stage them: the adjoint pack's records begin with
// {x, y, z, m, gx, gy, gz, 0} (gravity, 32 bytes) or {x, y, z, qs, sh, se, gx,
// gy, gz, ...} (LJC, 64 bytes, of which the first 48 are staged).
template <int LAW> struct alignas(16) BaRec { float x, y, z, qs, sh, se, gx, gy, gz, p0, p1, p2; };
template <> struct alignas(16) BaRec<GRAVITY> { float x, y, z, m, gx, gy, gz, p0; };

// sums per particle, i chunks per pass, staged and stored 128-bit vectors per record
template <int LAW> struct BaShape {
    static constexpr int NS = 6, ICH = 2, V = 3, RS = 4;
};
template <> struct BaShape<GRAVITY> {
    static constexpr int NS = 3, ICH = 4, V = 2, RS = 2;
};

// One unordered pair: i sums p, j sums jv (JSIDE); self0 neutralises the particle's own pair.
template <bool JSIDE>
__device__ __forceinline__ void ba_pair(const BaRec<GRAVITY> &I, const BaRec<GRAVITY> &J, float eps2, bool self0,
                                        float (&p)[3], float (&jv)[3])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
    float r2 = fma_(dx, dx, eps2);
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    r2 = self0 ? 1.0f : r2;
    float ri = rsqrt_(r2);
    ri = self0 ? 0.0f : ri;
    const float ri2 = ri * ri;
    const float ri3 = ri2 * ri;
    const float wx = fma_(-J.m, I.gx, I.m * J.gx);
    const float wy = fma_(-J.m, I.gy, I.m * J.gy);
    const float wz = fma_(-J.m, I.gz, I.m * J.gz);
    float dw = dx * wx;
    dw = fma_(dy, wy, dw);
    dw = fma_(dz, wz, dw);
    const float u = (ri2 * 3.0f) * dw;
    const float tx = ri3 * fma_(-u, dx, wx), ty = ri3 * fma_(-u, dy, wy), tz = ri3 * fma_(-u, dz, wz);
    p[0] += tx;
    p[1] += ty;
    p[2] += tz;
    if (JSIDE) {
        jv[0] -= tx;
        jv[1] -= ty;
        jv[2] -= tz;
    }
}

template <bool JSIDE>
__device__ __forceinline__ void ba_pair(const BaRec<LJC> &I, const BaRec<LJC> &J, float, bool self0, float (&p)[6],
                                        float (&jv)[6])
{
    const float dx = J.x - I.x, dy = J.y - I.y, dz = J.z - I.z;
    float r2 = dx * dx;
    r2 = fma_(dy, dy, r2);
    r2 = fma_(dz, dz, r2);
    float qq = I.qs * J.qs;
    float e = I.se * J.se;
    r2 = self0 ? 1.0f : r2;
    qq = self0 ? 0.0f : qq;
    e = self0 ? 0.0f : e;
    const float x = rcp_(r2);
    const float sg = I.sh + J.sh;
    const float sgx = sg * x;
    const float s2 = sg * sgx;                                     // (sigma_ij / r)^2
    const float s4 = s2 * s2;
    const float s6 = s4 * s2;
    const float lj = e * s6;                                       // 24 eps_ij s^6
    const float t = fma_(s6, 2.0f, -1.0f);
    const float cx = qq * x;
    const float W = fma_(lj, t, cx) * x;
    const float wpr = fma_(lj, fma_(s6, 28.0f, -8.0f), cx * 4.0f) * (x * x);
    const float ux = J.gx - I.gx, uy = J.gy - I.gy, uz = J.gz - I.gz;
    float du = dx * ux;
    du = fma_(dy, uy, du);
    du = fma_(dz, uz, du);
    du = self0 ? 0.0f : du;                                        // the own pair contributes nothing
    const float tt = wpr * du;
    const float px = fma_(tt, dx, -W * ux), py = fma_(tt, dy, -W * uy), pz = fma_(tt, dz, -W * uz);
    const float xdu = x * du;
    const float A = x * xdu;                                       // charge: times the other's qs
    const float B = ((e * (s4 * sgx)) * fma_(s6, 4.0f, -1.0f)) * xdu;   // sigma: the same for both
    const float C = (s6 * t) * xdu;                                // epsilon: times the other's se
    p[0] += px;
    p[1] += py;
    p[2] += pz;
    p[3] = fma_(J.qs, A, p[3]);
    p[4] += B;
    p[5] = fma_(J.se, C, p[5]);
    if (JSIDE) {
        jv[0] -= px;
        jv[1] -= py;
        jv[2] -= pz;
        jv[3] = fma_(I.qs, A, jv[3]);
        jv[4] += B;
        jv[5] = fma_(I.se, C, jv[5]);
    }
}

// One mini-sweep: the wave's ICH i chunks k0 .. k0 + ICH - 1 against j chunk q staged in st.
template <int LAW, bool DIAG>
__device__ __forceinline__ void ba_sweep(const BaRec<LAW> *st, const BaRec<LAW> (&iv)[BaShape<LAW>::ICH], float eps2,
                                         int q, int k0, int bp_addr,
                                         float (&p)[BaShape<LAW>::ICH][BaShape<LAW>::NS],
                                         float (&jv)[BaShape<LAW>::NS])
{
    constexpr int NS = BaShape<LAW>::NS, ICH = BaShape<LAW>::ICH;
    const int lane = lane_id();
#pragma unroll 2
    for (int t = 0; t < kWave; ++t) {
        const BaRec<LAW> J = st[lane + t];
#pragma unroll
        for (int kk = 0; kk < ICH; ++kk) {
            const int k = k0 + kk;
            if (!DIAG) {
                ba_pair<true>(iv[kk], J, eps2, false, p[kk], jv);
            } else if (k < q) {
                ba_pair<true>(iv[kk], J, eps2, false, p[kk], jv);
            } else if (k == q) {
                ba_pair<false>(iv[kk], J, eps2, t == 0, p[kk], jv);
            }
        }
#pragma unroll
        for (int c = 0; c < NS - 1; ++c) jv[c] = from_next_lane(bp_addr, jv[c]);
        jv[NS - 1] = from_next_lane_dpp(jv[NS - 1]);
    }
}

template <int LAW>
__device__ __forceinline__ BaRec<LAW> ba_make(const float4 &a, const float4 &b, const float4 &c)
{
    BaRec<LAW> r;
    float4 *v = (float4 *)&r;
    v[0] = a;
    v[1] = b;
    if constexpr (BaShape<LAW>::V == 3) v[2] = c;
    return r;
}

// waves per SIMD the register allocation aims at
template <int LAW, int PREC> constexpr int ba_waves_per_eu() { return LAW == GRAVITY && PREC == P_KAHAN ? 4 : 3; }

}  // namespace

template <int LAW, int PREC>
__global__ __launch_bounds__(kWaves * kWave) __attribute__((amdgpu_waves_per_eu(ba_waves_per_eu<LAW, PREC>())))
void k_bsym_adj(BSymAdjLaunch a)
{
    using R = BaRec<LAW>;
    constexpr int NS = BaShape<LAW>::NS, ICH = BaShape<LAW>::ICH, V = BaShape<LAW>::V, RS = BaShape<LAW>::RS;
    constexpr int NV = (NS + 3) / 4;                              // 128-bit vectors per slot row
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ R st_all[kWaves][2 * kWave];                      // each wave's j chunk, staged twice
    __shared__ float jd_all[kWaves][kChunks][NS][kWave];         // the j sums of block b2, per wave
    int64_t b1, b2, po, npad, slot0;
    if (a.units) {
        const int64_t u = (int64_t)blockIdx.x * kWaves + w;
        if (u >= a.n_units) return;                              // whole wave; the kernel has no barriers
        const int32_t *un = a.units + 4 * u;
        const int64_t s = un[0];
        b1 = un[1];
        b2 = un[2];
        if (s < 0 || s >= a.n_systems) return;
        po = a.poff[s];
        npad = a.poff[s + 1] - po;
        slot0 = a.systab[3 * s + 2];
    } else {
        // one system: the workgroups reach the XCDs in turn, so each XCD is given a contiguous
        // run of workgroups, four consecutive tiles of the strip order each
        npad = a.single_npad;
        const int64_t nbs = npad / kBSymRecords, tiles = sym_tiles(nbs);
        const int64_t per = sym_grid((tiles + kWaves - 1) / kWaves) / kSymXcds;
        const int64_t u = ((int64_t)(blockIdx.x % kSymXcds) * per + blockIdx.x / kSymXcds) * kWaves + w;
        if (u >= tiles) return;
        sym_tile_at(u, nbs, b1, b2);
        po = 0;
        slot0 = 0;
    }
    const int64_t nb = npad / kBSymRecords;
    if (b1 < 0 || b2 < b1 || b2 >= nb) return;                   // never index outside the tables
    const bool diag = b1 == b2;
    const int64_t irec0 = po + b1 * kBSymRecords, jrec0 = po + b2 * kBSymRecords;
    float4 *slots = a.partial + slot0 * NV;                      // [nb][npad][NV] of the system
    R *st = st_all[w];
    float(*jd)[NS][kWave] = jd_all[w];
    const float eps2 = (float)a.eps2;
    const int bp_addr = ((lane + 1) & (kWave - 1)) * 4;
    const float4 *__restrict__ rec4 = (const float4 *)a.rec;
    float4 *st4 = (float4 *)st;
#pragma unroll
    for (int q = 0; q < kChunks; ++q)
#pragma unroll
        for (int c = 0; c < NS; ++c) jd[q][c][lane] = 0.0f;

    for (int pass = 0; pass < kChunks / ICH; ++pass) {
        const int k0 = pass * ICH;
        R iv[ICH];
#pragma unroll
        for (int kk = 0; kk < ICH; ++kk) {
            const int64_t r = (irec0 + (int64_t)(k0 + kk) * kWave + lane) * RS;
            iv[kk] = ba_make<LAW>(rec4[r], rec4[r + 1], V == 3 ? rec4[r + 2] : float4{0, 0, 0, 0});
        }
        RunSum<PREC> acc[ICH][NS];
        float p[ICH][NS];
        // the next chunk's record of this lane, loaded a chunk ahead as 128-bit vectors
        int64_t rj = (jrec0 + lane) * RS;
        float4 g0 = rec4[rj], g1 = rec4[rj + 1], g2 = V == 3 ? rec4[rj + 2] : float4{0, 0, 0, 0};
        for (int q = 0; q < kChunks; ++q) {
            const int qn = q + 1 < kChunks ? q + 1 : q;          // the last chunk reloads itself
            if (diag && q < k0) {                                // no pair of these i chunks with q
                rj = (jrec0 + (int64_t)qn * kWave + lane) * RS;
                g0 = rec4[rj];
                g1 = rec4[rj + 1];
                if (V == 3) g2 = rec4[rj + 2];
                continue;
            }
            st4[lane * V] = g0;
            st4[lane * V + 1] = g1;
            st4[(lane + kWave) * V] = g0;
            st4[(lane + kWave) * V + 1] = g1;
            if (V == 3) {
                st4[lane * V + 2] = g2;
                st4[(lane + kWave) * V + 2] = g2;
            }
            rj = (jrec0 + (int64_t)qn * kWave + lane) * RS;
            g0 = rec4[rj];
            g1 = rec4[rj + 1];
            if (V == 3) g2 = rec4[rj + 2];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int kk = 0; kk < ICH; ++kk)
#pragma unroll
                for (int c = 0; c < NS; ++c) acc[kk][c].begin(p[kk][c]);
            float jv[NS];
#pragma unroll
            for (int c = 0; c < NS; ++c) jv[c] = jd[q][c][lane];
            if (!diag) ba_sweep<LAW, false>(st, iv, eps2, q, k0, bp_addr, p, jv);
            else ba_sweep<LAW, true>(st, iv, eps2, q, k0, bp_addr, p, jv);
#pragma unroll
            for (int c = 0; c < NS; ++c) jd[q][c][lane] = jv[c];
#pragma unroll
            for (int kk = 0; kk < ICH; ++kk)
#pragma unroll
                for (int c = 0; c < NS; ++c) acc[kk][c].fold(p[kk][c]);
            __builtin_amdgcn_wave_barrier();                     // the slot is restaged next
        }
        // i sums of this pass: slot b2 of the rows of block b1 (on the diagonal with the j sums
        // of the same rows, complete once the pass holding their chunk is done)
#pragma unroll
        for (int kk = 0; kk < ICH; ++kk) {
            const int c = k0 + kk;
            float v[4 * NV];
#pragma unroll
            for (int m = 0; m < 4 * NV; ++m) v[m] = 0.0f;
#pragma unroll
            for (int m = 0; m < NS; ++m) v[m] = (float)acc[kk][m].value() + (diag ? jd[c][m][lane] : 0.0f);
            float4 *dst = slots + (b2 * npad + b1 * kBSymRecords + c * kWave + lane) * NV;
#pragma unroll
            for (int j = 0; j < NV; ++j) dst[j] = float4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        }
    }
    // j sums: slot b1 of the rows of block b2
    if (!diag) {
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            float v[4 * NV];
#pragma unroll
            for (int m = 0; m < 4 * NV; ++m) v[m] = m < NS ? jd[q][m][lane] : 0.0f;
            float4 *dst = slots + (b1 * npad + b2 * kBSymRecords + q * kWave + lane) * NV;
#pragma unroll
            for (int j = 0; j < NV; ++j) dst[j] = float4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        }
    }
}

// Row block red[blockIdx.x] = (s, rb) of 256 rows: each row adds its system's nb_s slots in
// slot order (FP64, Neumaier) and writes its gradients.
template <int LAW>
__global__ __launch_bounds__(kBSymRecords) void k_bsym_adj_reduce(BSymAdjLaunch a)
{
    constexpr int NS = BaShape<LAW>::NS, NV = (NS + 3) / 4;
    const bool one = a.red == nullptr;                           // one whole system
    const int64_t s = one ? 0 : a.red[2 * blockIdx.x], rb = one ? blockIdx.x : a.red[2 * blockIdx.x + 1];
    const int64_t l = rb * kBSymRecords + threadIdx.x;
    const int64_t o = one ? 0 : a.off[s];
    if (l >= (one ? a.single_n : a.off[s + 1] - o)) return;
    const int64_t npad = one ? a.single_npad : a.poff[s + 1] - a.poff[s];
    const int64_t nb = npad / kBSymRecords;
    const float4 *__restrict__ slots = a.partial + ((one ? 0 : a.systab[3 * s + 2]) + l) * NV;
    NSum v[NS];
    for (int64_t k = 0; k < nb; ++k) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const float4 x = slots[k * npad * NV + j];
            const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (4 * j + m < NS) v[4 * j + m].add((double)xs[m]);
        }
    }
    const int64_t r = o + l;
    if (LAW == GRAVITY) {
        if (a.grad_pos)
            for (int c = 0; c < 3; ++c) a.grad_pos[3 * r + c] = a.G * v[c].value();
        return;
    }
    if (a.grad_pos)
        for (int c = 0; c < 3; ++c) a.grad_pos[3 * r + c] = v[c].value();
    if (a.grad_params && NS == 6) {
        // the sums carry the records' factor 24 in eps (v[4]) and sqrt(24) in se_j (v[5])
        const double se_k = __builtin_sqrt(24.0 * a.params[3 * r + 2]);
        a.grad_params[3 * r] = a.qscale * v[3].value();
        a.grad_params[3 * r + 1] = 3.0 * v[4].value();
        a.grad_params[3 * r + 2] = (12.0 / se_k) * v[5].value();
    }
}

bool bsym_adj_supported(int law, int prec)
{
    return (law == GRAVITY || law == LJC) && (prec == P_KAHAN || prec == P_FP64ACC);
}

int bsym_adj_sums(int law) { return law == GRAVITY ? BaShape<GRAVITY>::NS : BaShape<LJC>::NS; }

hipError_t launch_bsym_adj(const BSymAdjLaunch &a, hipStream_t s)
{
    if (!bsym_adj_supported(a.law, a.prec)) return hipErrorInvalidValue;
    int64_t wgs;
    if (a.units) {
        if (a.n_units <= 0) return hipSuccess;
        wgs = (a.n_units + kWaves - 1) / kWaves;
    } else {
        if (a.single_n <= 0) return hipSuccess;
        if (a.single_npad % kBSymRecords != 0 || a.single_n > a.single_npad || a.red) return hipErrorInvalidValue;
        wgs = sym_grid((sym_tiles(a.single_npad / kBSymRecords) + kWaves - 1) / kWaves);
    }
    const dim3 grid((unsigned)wgs), block(kWaves * kWave);
    const bool kahan = a.prec == P_KAHAN;
    if (a.law == GRAVITY) {
        if (kahan) hipLaunchKernelGGL((k_bsym_adj<GRAVITY, P_KAHAN>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_bsym_adj<GRAVITY, P_FP64ACC>), grid, block, 0, s, a);
    } else {
        if (kahan) hipLaunchKernelGGL((k_bsym_adj<LJC, P_KAHAN>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_bsym_adj<LJC, P_FP64ACC>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_bsym_adj_reduce(const BSymAdjLaunch &a, hipStream_t s)
{
    if (!bsym_adj_supported(a.law, a.prec)) return hipErrorInvalidValue;
    const int64_t blocks = a.red ? a.n_red : (a.single_n + kBSymRecords - 1) / kBSymRecords;
    if (blocks <= 0) return hipSuccess;
    if (!a.red && (a.units || a.single_npad % kBSymRecords != 0 || a.single_n > a.single_npad))
        return hipErrorInvalidValue;
    if (a.law == GRAVITY) hipLaunchKernelGGL((k_bsym_adj_reduce<GRAVITY>), dim3((unsigned)blocks), dim3(kBSymRecords), 0, s, a);
    else hipLaunchKernelGGL((k_bsym_adj_reduce<LJC>), dim3((unsigned)blocks), dim3(kBSymRecords), 0, s, a);
    return hipGetLastError();
}

}  // namespace nbk
