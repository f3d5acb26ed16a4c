// Internal interface between the host runtime (api.cpp) and the HIP kernels.
// Not part of the public ABI (include/nbody.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nbk {

// Lanes per row of a fixed-order split reduction: the smallest power of two
// >= nsplit, at most 64 (shared by the launchers and the kernels).
__host__ __device__ inline int split_group(int64_t nsplit)
{
    int g = 1;
    while (g < 64 && g < nsplit) g <<= 1;
    return g;
}

// Per-particle exclusion lists (CSR over the caller's particle indices):
// particle x excludes idx[off[x] .. off[x+1]) (ranges clamped to [0, count)).
// off == nullptr: no exclusions.
struct ExclArgs {
    const int64_t *off;
    const int64_t *idx;
    int64_t count;
};

// What the all-pairs kernels do with the four finished sums of a row.
struct Epilogue {
    double fscale;              // out_force = fscale * sum_vec   (G for gravity, 1 for LJC)
    double pscale;              // out_pot   = pscale * sum_pot   (-G for gravity, 1/2 for LJC)
    double *out_force;          // [rows][3]
    double *out_pot;            // [rows] or null
    // leapfrog kick (kick != 0): acc = force * inv_mass; acc -> acc_out; vel += half_dt * acc
    int kick;
    double half_dt;
    double *vel;                // [rows][3]
    const double *inv_mass;     // [rows] or null
};

struct FwdLaunch {
    int law, prec, ipl, pot;     // template selectors
    int block;                   // threads per workgroup
    int64_t npad;                // padded record count (multiple of 64)
    int64_t nrows;               // output rows
    const int64_t *rows;         // row -> particle index, or null (identity)
    int64_t split_len;           // j range per split (multiple of 64)
    int j_split;
    int j_tile;
    int j_stage;                 // 0: j records through SGPRs (scalar loads); 1: through LDS into VGPRs
    double eps2;                 // gravity softening squared
    double zeta[4];              // sigmoidal dielectric exp(z0 r^3 + z1 r^2 + z2 r + z3)
    const void *rec;             // packed records
    double *partial;             // [j_split][nrows][4] when j_split > 1
    Epilogue epi;
    ExclArgs excl;               // per-particle exclusion lists, or off == nullptr
};

// Pack FP64 inputs into padded records (FP32 or FP64) for one system.
// When kick_drift != 0 the positions are first advanced in place:
//   vel += half_dt * acc;  pos += dt * vel.
struct PackLaunch {
    int law, prec;
    int64_t n, npad;
    double *pos;                 // [n][3] (written only when kick_drift)
    const double *params;        // [n][P]
    double qscale;               // sqrt(2k/D) for LJC
    void *rec;
    int kick_drift;
    double *vel;
    const double *acc;
    double half_dt, dt;
};

hipError_t launch_pack(const PackLaunch &p, hipStream_t s);
hipError_t launch_forces(const FwdLaunch &f, hipStream_t s);
hipError_t launch_reduce_split(const FwdLaunch &f, hipStream_t s);
int forces_blocks_per_cu(int law, int prec, int ipl, int pot, int js, int block);

// ---- symmetric pair tiles (symmetric.hip): gravity and the LJC laws, every unordered pair once ----
constexpr int kSymThreads = 512;           // the larger workgroup: 8 waves, 2 i chunks per wave (or 4 x 4)
constexpr int kSymMaxBlk = 32;             // largest block edge in chunks of 64 records
// gravity forces (and potentials), gravity's position adjoint, and the forces (and energies) of
// LJC with the linear, constant or sigmoidal dielectric
enum SymOp { SYM_FORCE = 0, SYM_HVP = 1, SYM_LJC = 2, SYM_LJC_CONST = 3, SYM_LJC_SIG = 4 };
struct SymLaunch {
    int op;                        // SYM_FORCE ({x, y, z, m}), SYM_HVP ({x, y, z, m, g, 0}) or an LJC
                                   // operator ({x, y, z, qs, sh, se, 0, 0}) records
    int prec, pot;                 // P_KAHAN or P_FP64ACC tile sums; potential on/off (forces)
    int blk;                       // block edge in chunks of 64 records: 16 or 32
    int ich;                       // i chunks per wave: 2 (8-wave workgroups) or 4 (4-wave workgroups)
    int split;                     // j parts per tile (1, 2 or 4), one workgroup each; blk / split
                                   // must be at least the workgroup's waves
    int64_t nblk;                  // blocks; tiles = nblk (nblk + 1) / 2
    int64_t npad;                  // records = nblk * blk * 64 (zero-mass padding past n)
    int64_t n;                     // rows finished by the reduction
    double eps2;                   // gravity softening squared
    double zeta[4];                // SYM_LJC_SIG: exp(z0 r^3 + z1 r^2 + z2 r + z3), as FwdLaunch::zeta
    const void *rec;               // FP32 records of the operator
    float4 *partial;               // [split * nblk][npad] (x, y, z, potential) FP32 slot partials
    int64_t t0, count;             // order range of the launch's tiles (whole triangle: 0, sym_tiles)
    Epilogue epi;
};
// Tile order of the symmetric launch.  The upper triangle (b1 <= b2) of the nblk x nblk block
// grid is walked in strips of kSymStrip block rows, column by column inside a strip, so that
// consecutive tiles share their blocks: sym_tile_at maps an order index to its tile and
// sym_index_of is its inverse.  A launch covers the order range [t0, t0 + count) (the whole
// triangle, or one share of it); the range is cut into kSymXcds equal portions, one per XCD
// (workgroups reach the XCDs in turn by linear id), so that each XCD's L2 sees a compact region
// of the grid at a time.  Workgroup `wg` of sym_grid(count) gets its tile from sym_tile_of,
// which returns false for the few workgroups past the last tile.
constexpr int kSymStrip = 8;
constexpr int kSymXcds = 8;
__host__ __device__ inline int64_t sym_tiles(int64_t nblk) { return nblk * (nblk + 1) / 2; }
__host__ __device__ inline int64_t sym_grid(int64_t count)
{
    return (count + kSymXcds - 1) / kSymXcds * kSymXcds;
}
// first order index of strip s (every strip before it is a full one)
__host__ __device__ inline int64_t sym_strip_start(int64_t s, int64_t nblk)
{
    const int64_t h = kSymStrip;
    return s * (h * (h + 1) / 2) + h * (s * nblk - h * s * (s + 1) / 2);
}
__host__ __device__ inline void sym_tile_at(int64_t t, int64_t nblk, int64_t &b1, int64_t &b2)
{
    int64_t lo = 0, hi = (nblk + kSymStrip - 1) / kSymStrip - 1;      // strip: last start <= t
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (sym_strip_start(mid, nblk) <= t) lo = mid;
        else hi = mid - 1;
    }
    const int64_t r0 = lo * kSymStrip, h = nblk - r0 < kSymStrip ? nblk - r0 : kSymStrip;
    const int64_t u = t - sym_strip_start(lo, nblk), tri = h * (h + 1) / 2;
    if (u < tri) {
        // columns r0 .. r0 + h - 1 hold 1 .. h tiles
        int64_t k = 0;
        while ((k + 1) * (k + 2) / 2 <= u) ++k;
        b2 = r0 + k;
        b1 = r0 + (u - k * (k + 1) / 2);
    } else {
        b2 = r0 + h + (u - tri) / h;
        b1 = r0 + (u - tri) % h;
    }
}
__host__ __device__ inline int64_t sym_index_of(int64_t b1, int64_t b2, int64_t nblk)
{
    const int64_t s = b1 / kSymStrip, r0 = s * kSymStrip;
    const int64_t h = nblk - r0 < kSymStrip ? nblk - r0 : kSymStrip;
    const int64_t k = b2 - r0;
    const int64_t u = k < h ? k * (k + 1) / 2 + (b1 - r0) : h * (h + 1) / 2 + (k - h) * h + (b1 - r0);
    return sym_strip_start(s, nblk) + u;
}
// With the j chunks of each tile cut into `split` parts, the launch's work items are the
// count * split (tile, part) pairs, the parts of a tile consecutive: workgroup wg of
// sym_grid(count * split) runs part h of tile (b1, b2).
__host__ __device__ inline bool sym_item_of(int64_t wg, int64_t nblk, int64_t t0, int64_t count, int split,
                                            int64_t &b1, int64_t &b2, int &h)
{
    const int64_t items = count * split;
    const int64_t per = sym_grid(items) / kSymXcds;
    const int64_t local = (wg % kSymXcds) * per + wg / kSymXcds;
    if (local >= items) return false;
    h = (int)(local % split);
    sym_tile_at(t0 + local / split, nblk, b1, b2);
    return true;
}
__host__ __device__ inline bool sym_tile_of(int64_t wg, int64_t nblk, int64_t t0, int64_t count, int64_t &b1,
                                            int64_t &b2)
{
    int h;
    return sym_item_of(wg, nblk, t0, count, 1, b1, b2, h);
}
// Order range of share `share` of `shares` equal shares of the triangle.
__host__ __device__ inline void sym_share_range(int64_t nblk, int64_t share, int64_t shares, int64_t &t0,
                                                int64_t &count)
{
    const int64_t T = sym_tiles(nblk);
    t0 = T * share / shares;
    count = T * (share + 1) / shares - t0;
}
hipError_t launch_sym(const SymLaunch &a, hipStream_t s);
hipError_t launch_sym_reduce(const SymLaunch &a, hipStream_t s);

// ---- batched (one persistent launch over (system, row-block) work units) ----
struct BatchLaunch {
    int law, prec, ipl, pot;
    int block;
    int grid;                    // persistent workgroups
    int64_t n_units;
    const int32_t *units;        // [n_units][4] = (system, row block, j part, 0), cost-descending
    const int64_t *off;          // [S+1] caller row offsets
    const int64_t *poff;         // [S+1] padded record offsets
    const int64_t *systab;       // [S][3] = (j parts P, records per part, first partial slot)
    double *partial;             // [slots][64 * ipl][4] part sums of systems with P > 1
    int any_parts;               // some system has P > 1 (the part sums need reducing)
    const int32_t *red;          // [n_red][2] (system, row block) of the row blocks with P > 1
    int64_t n_red;
    int64_t n_systems;
    int64_t n_total, npad_total;
    int j_tile;
    int j_stage;                 // as FwdLaunch::j_stage
    double eps2;
    double zeta[4];              // as FwdLaunch::zeta
    const void *rec;
    int *ticket;                 // zeroed by the batched pack (ticket_zeroed) or by launch_batched
    int ticket_zeroed;           // the pack of this launch has zeroed the ticket
    Epilogue epi;
    ExclArgs excl;               // exclusion lists over the caller's rows, or off == nullptr
};
struct BatchPackLaunch {
    int law, prec;
    int64_t n_systems, npad_total;
    const int64_t *off, *poff;
    const double *pos, *params;
    double qscale;
    void *rec;
    int *ticket;                 // or null: 256 bytes the pack zeroes for the batched kernel
};
hipError_t launch_pack_batched(const BatchPackLaunch &p, hipStream_t s);
hipError_t launch_batched(const BatchLaunch &b, hipStream_t s);
int batched_max_blocks_per_cu(int law, int prec, int ipl, int pot, int js, int block, int excl);

// ---- batched symmetric pair tiles (bsym.hip): gravity or an LJC law, every unordered pair of a
// system once, one wave per tile of two 256-record blocks ----
constexpr int kBSymRecords = 256;          // records per block (four chunks of 64)
constexpr int64_t kBSymMaxSystem = 8192;   // largest system of a symmetric batched launch (32 blocks)
struct BSymLaunch {
    int law, prec, pot;
    int64_t n_units;
    const int32_t *units;        // [n_units][4] = (system, b1, b2, 0), b1 <= b2
    const int64_t *off;          // [S+1] caller row offsets
    const int64_t *poff;         // [S+1] record offsets, systems padded to whole blocks
    const int64_t *systab;       // [S][3] = (blocks nb, 0, first float4 of the system's slots)
    const int32_t *red;          // [n_red][2] (system, row block of 256)
    int64_t n_red;
    int64_t n_systems;
    double eps2;
    double zeta[4];              // the sigmoidal dielectric's coefficients, as FwdLaunch::zeta
    const void *rec;             // FP32 records
    float4 *partial;             // per system [nb][npad] (x, y, z, potential) FP32 slot partials
    Epilogue epi;
};
bool bsym_supported(int law, int prec);
hipError_t launch_bsym(const BSymLaunch &a, hipStream_t s);
hipError_t launch_bsym_reduce(const BSymLaunch &a, hipStream_t s);

// zero-fill with a kernel (no memset nodes, so the calls stay capturable)
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace nbk
