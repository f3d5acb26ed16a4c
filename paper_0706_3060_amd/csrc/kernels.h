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
    int64_t n_systems;
    int64_t n_total, npad_total;
    int j_tile;
    int j_stage;                 // as FwdLaunch::j_stage
    double eps2;
    double zeta[4];              // as FwdLaunch::zeta
    const void *rec;
    int *ticket;                 // zeroed by launch_batched before the kernel
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
};
hipError_t launch_pack_batched(const BatchPackLaunch &p, hipStream_t s);
hipError_t launch_batched(const BatchLaunch &b, hipStream_t s);
int batched_max_blocks_per_cu(int law, int prec, int ipl, int pot, int js, int block, int excl);

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
    int64_t n_systems, npad_total, n_total;
    double eps2, G, qscale;
    const double *pos, *params, *g;   // caller arrays (pack)
    void *rec;
    int *ticket;
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
// per-type sums of grad_params columns 1 and 2 into out [n_types][2], through
// partial [blocks][n_types][2] (partial_doubles doubles; at least 2 n_types)
hipError_t launch_type_reduce(const double *grad_params, const int32_t *types, int64_t n,
                              int32_t n_types, double *out, double *partial, int64_t partial_doubles,
                              hipStream_t s);

// ---- acceleration + jerk and the Hermite integrator ----
struct JerkPackLaunch {
    int prec;
    int64_t n, npad;
    const double *pos, *vel, *mass;   // [n][3], [n][3], [n]
    int predict;                      // 0: records from (pos, vel); 1: Hermite-predicted state
    const double *acc, *jerk;         // [n][3] (predict)
    const double *t_i;                // [n] per-particle times, or null: tau for every particle
    double t_pred;                    // prediction time (with t_i)
    const double *t_pred_dev;         // or the prediction time in device memory (with t_i)
    const int64_t *live_dev;          // or null: when set and zero, the pack is skipped
    double tau;                       // prediction interval (without t_i)
    void *rec;                        // GajRec records [npad]
};
struct JerkLaunch {
    int prec, ipl, pot;
    int block, j_stage;
    int64_t npad;
    int64_t nrows;                    // rows (the grid is sized for this many)
    const int64_t *nrows_dev;         // or, when set, the rows to evaluate (<= nrows) in device memory
    const int64_t *rows;              // row -> particle, or null (identity)
    int64_t split_len;
    int j_split, j_tile;              // j_split: the split, or its upper bound with split_dev
    const int64_t *split_dev;         // or, when set, the split in device memory (1-D grid)
    int64_t grid_waves;               // with split_dev: waves launched (>= row waves x split)
    int64_t partial_rows;             // with split_dev: partial buffer capacity in rows (split x rows)
    double eps2, G;
    const void *rec;
    double *partial;                  // [j_split][nrows][8] when j_split > 1
    double *out_acc, *out_jerk;       // [nrows][3]
    double *out_pot;                  // [nrows] or null
};
struct HermiteLaunch {
    int64_t nrows;                    // grid size in rows
    const int64_t *nrows_dev;         // or, when set, the rows to correct (<= nrows) in device memory
    const int64_t *rows;              // active particles, or null (all)
    double *pos, *vel, *acc, *jerk;   // [n][3], updated for the rows
    const double *a1, *j1;            // [nrows][3] at the predicted state, in row order
    double h;                         // shared step (when dt_i is null)
    double *t_i, *dt_i;               // block steps: per-particle time and step, or null
    const double *t_next;             // block steps: device scalar, the block time
    double eta, dt_max;
    // or, when partial is set, a1 / j1 are G x the fixed-order sum of the j-split
    // partials [split][nrows][8] (split from split_dev, at most split_max; with a
    // split of 1 they are read from a1 / j1); the grid then has grid_threads threads
    const double *partial;
    const int64_t *split_dev;
    int64_t split_max, grid_threads;
    int64_t partial_rows;             // capacity clamp, as JerkLaunch::partial_rows
    double Gc;
};
// State of one block step, written by the scheduler and read by the kernels
// that follow it on the stream.
struct BlockState {
    double t;                         // block time: the smallest t_i + dt_i
    int64_t count;                    // due particles (0 past t_end)
    int64_t split;                    // j split of the jerk evaluation of the due rows
    int64_t pad;
};
struct SchedLaunch {
    int64_t n, chunk;
    int nb;                           // scheduling blocks, each owns `chunk` particles
    const double *t_i, *dt_i;
    double *part_min;                 // [nb]
    int64_t *part_cnt;                // [nb]
    int64_t *list;                    // [n] due particles, increasing
    BlockState *state;
    double t_end;                     // a block time beyond t_end has no due particles
    const int *split_table;           // [table_len]: split for 1.. row waves of due rows, or null (1)
    int64_t table_len;
    int rows_per_wave;
    int64_t *count_log;               // [log] due counts of successive block steps, or null
    double *time_log;                 // [log] their block times
    int64_t log_index;
    int fuse_pack;                    // also write the predicted records of the block step
    JerkPackLaunch pack;              // (t_pred_dev = &state->t, pack.n == n)
};
hipError_t launch_pack_jerk(const JerkPackLaunch &p, hipStream_t s);
hipError_t launch_jerk(const JerkLaunch &a, hipStream_t s);
hipError_t launch_jerk_reduce(const JerkLaunch &a, hipStream_t s);
int jerk_blocks_per_cu(int prec, int ipl, int pot, int js, int block);
hipError_t launch_hermite_correct(const HermiteLaunch &a, hipStream_t s);
hipError_t launch_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                             double dt_max, double *t_i, double *dt_i, hipStream_t s);
hipError_t launch_schedule(const SchedLaunch &a, hipStream_t s);

// zero-fill with a kernel (no memset nodes, so the calls stay capturable)
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace nbk
