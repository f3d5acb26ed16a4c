// Internal interface between the host runtime (api.cpp) and the acceleration-
// and-jerk and Hermite kernels (jerk.hip).  Not part of the public ABI.
#pragma once
#include "kernels.h"

namespace nbk {

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
// Symmetric pair tiles of the acceleration and jerk (symjerk.hip): each unordered pair of a
// whole system evaluated once and applied to both particles, FP32 pair arithmetic, per-row
// FP32 slot partials added in slot order in FP64.
constexpr int kSymJerkBlk = 16;       // block edge in chunks of 64 records (1024 records)
struct SymJerkLaunch {
    int prec, pot;                    // P_KAHAN or P_FP64ACC tile sums; potential on/off
    int split;                        // j parts per tile (1 or 2), one workgroup each
    int64_t nblk;                     // blocks; tiles = nblk (nblk + 1) / 2
    int64_t npad;                     // records = nblk * kSymJerkBlk * 64 (zero-mass padding past n)
    int64_t n;                        // rows finished by the reduction
    double eps2, G;
    const void *rec;                  // GajRec<float> records [npad]
    float4 *partial;                  // [split * nblk][npad][2]: (a, jerk_x) and (jerk_y, jerk_z, phi, 0)
    double *out_acc, *out_jerk;       // [n][3]
    double *out_pot;                  // [n] or null
};
hipError_t launch_symjerk(const SymJerkLaunch &a, hipStream_t s);
hipError_t launch_symjerk_reduce(const SymJerkLaunch &a, hipStream_t s);

hipError_t launch_pack_jerk(const JerkPackLaunch &p, hipStream_t s);
hipError_t launch_jerk(const JerkLaunch &a, hipStream_t s);
hipError_t launch_jerk_reduce(const JerkLaunch &a, hipStream_t s);
int jerk_blocks_per_cu(int prec, int ipl, int pot, int js, int block);
hipError_t launch_hermite_correct(const HermiteLaunch &a, hipStream_t s);
hipError_t launch_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                             double dt_max, double *t_i, double *dt_i, hipStream_t s);
hipError_t launch_schedule(const SchedLaunch &a, hipStream_t s);

}  // namespace nbk
