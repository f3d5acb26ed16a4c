// Internal interface between the host runtime (api.cpp) and the adjoint
// kernels (adjoint.hip).  Not part of the public ABI (include/nbody.h).
#pragma once
#include "kernels.h"

namespace nbk {

// ---- adjoint ----
struct AdjLaunch {
    int law, prec, ipl;
    int block;
    int j_stage;                 // as FwdLaunch::j_stage
    int64_t n, npad;
    int64_t split_len;
    int j_split, j_tile;
    double eps2;
    double G;                    // gravity
    double qscale;               // LJC sqrt(2k/D)
    const void *rec;
    double *partial;             // [j_split][n][8] when j_split > 1
    double *grad_pos;            // [n][3] or null
    double *grad_params;         // [n][3] or null (LJC)
    const double *params;        // caller params (for the per-atom scale factors)
    ExclArgs excl;               // exclusion lists (LJC), or off == nullptr
};
// Batched adjoint: (system, row-block) units in one persistent launch.
struct AdjBatchLaunch {
    int law, prec, ipl;
    int block, grid;
    int j_stage;
    int j_tile;
    int64_t n_units;
    const int32_t *units;        // [n_units][4] (system, row block, j part, 0)
    const int64_t *off, *poff;   // [S+1] caller rows and padded record offsets
    const int64_t *systab;       // [S][3] = (j parts P, records per part, first partial slot)
    double *partial;             // [slots][64 * ipl][8] part sums of systems with P > 1
    int any_parts;
    const int32_t *red;          // [n_red][2] (system, row block) of the row blocks with P > 1
    int64_t n_red;
    int64_t n_systems, npad_total, n_total;
    double eps2, G, qscale;
    const double *pos, *params, *g;   // caller arrays (pack)
    void *rec;
    int *ticket;                 // zeroed by the pack (ticket_zeroed) or by launch_adjoint_batched
    int ticket_zeroed;
    double *grad_pos;            // [n][3] or null
    double *grad_params;         // [n][3] or null (LJC)
    ExclArgs excl;
};
hipError_t launch_pack_adjoint_batched(const AdjBatchLaunch &p, hipStream_t s);
hipError_t launch_adjoint_batched(const AdjBatchLaunch &a, hipStream_t s);
int adjoint_batched_blocks_per_cu(const AdjBatchLaunch &a);
struct AdjPackLaunch {
    int law, prec;
    int64_t n, npad;
    const double *pos, *params, *g;
    double qscale;
    void *rec;
};
hipError_t launch_pack_adjoint(const AdjPackLaunch &p, hipStream_t s);
hipError_t launch_adjoint(const AdjLaunch &a, hipStream_t s);
hipError_t launch_adjoint_reduce(const AdjLaunch &a, hipStream_t s);
// Batched adjoint over unordered pairs (bsym_adj.hip): one wave per tile (s, b1, b2) of two
// 256-record blocks of a system, the tiles and row blocks listed by the plan of the batched
// symmetric tiles (kernels.h BSymLaunch); records from the batched adjoint pack, systems padded
// to whole blocks.
struct BSymAdjLaunch {
    int law, prec;
    int64_t n_units;
    const int32_t *units;        // [n_units][4] = (system, b1, b2, 0), b1 <= b2
    const int64_t *off, *poff;   // [S+1] caller rows and record offsets (whole blocks)
    const int64_t *systab;       // [S][3] = (blocks nb, 0, first slot row of the system)
    const int32_t *red;          // [n_red][2] (system, row block of 256)
    int64_t n_red;
    int64_t n_systems;
    double eps2, G, qscale;
    const void *rec;             // FP32 adjoint records
    float4 *partial;             // per system [nb][npad][bsym_adj_sums(law) / 4 rounded up] FP32 slot sums
    const double *params;        // caller params (LJC: the epsilon gradient's scale)
    double *grad_pos;            // [n][3] or null
    double *grad_params;         // [n][3] or null (LJC)
    // or, with units and red null, one whole system of single_n rows (records padded to
    // single_npad, a multiple of 256): its nb (nb + 1) / 2 tiles taken in the XCD-aware strip
    // order, its row blocks in order, its slots from partial[0]
    int64_t single_n, single_npad;
};
bool bsym_adj_supported(int law, int prec);
int bsym_adj_sums(int law);      // sums per particle: 3 (gravity) or 6 (LJC)
hipError_t launch_bsym_adj(const BSymAdjLaunch &a, hipStream_t s);
hipError_t launch_bsym_adj_reduce(const BSymAdjLaunch &a, hipStream_t s);
// per-type sums of grad_params columns 1 and 2 into out [n_types][2], through
// partial [blocks][n_types][2] (partial_doubles doubles; at least 2 n_types)
hipError_t launch_type_reduce(const double *grad_params, const int32_t *types, int64_t n,
                              int32_t n_types, double *out, double *partial, int64_t partial_doubles,
                              hipStream_t s);

}  // namespace nbk
