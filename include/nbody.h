/*
 * nbody.h -- C ABI of the MI355X (gfx950) all-pairs N-body library (libnbody.so).
 *
 * The library evaluates the O(N^2) pairwise force and potential sums that the
 * paper (Elsen et al., "N-Body Simulations on GPUs") identifies as the major
 * cost of stellar and molecular dynamics steps (Section 1; the all-pairs
 * pseudo-code and its stream form in Section 2), followed by the update step
 * (Section 1).  The pair laws are those of Table 1:
 *
 *   NBODY_LAW_GRAVITY     softened gravity, Eq. 1 (Section 3.3) and Table 1
 *                         "Gravity (accel)"; with nbody_forces_jerk also its
 *                         time derivative, Table 1 "Gravity (accel & jerk)":
 *                           a_i   =  G sum_{j!=i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}
 *                           phi_i = -G sum_{j!=i} m_j / (|r_j - r_i|^2 + eps^2)^{1/2}
 *   NBODY_LAW_LJC_LINEAR  Lennard-Jones + Coulomb with the linear distance-
 *                         dependent dielectric eps(r) = D r (Table 1
 *                         "LJC (linear)"; Section 2, continuum solvent),
 *                         read as the gradient of
 *                           u_ij = k q_i q_j / (D r^2) + 4 e_ij [(s_ij/r)^12 - (s_ij/r)^6],
 *                           s_ij = (s_i + s_j)/2,  e_ij = sqrt(e_i e_j):
 *                           F_i = sum_{j!=i} [2 k q_i q_j/(D r^4)
 *                                 + (24 e_ij/r^2)(2 (s_ij/r)^12 - (s_ij/r)^6)] (r_i - r_j)
 *                           U_i = sum_{j!=i} u_ij     (total energy = 1/2 sum_i U_i)
 *   NBODY_LAW_LJC_CONSTANT, NBODY_LAW_LJC_SIGMOIDAL   the constant and sigmoidal
 *                         dielectrics of Table 1 (see nbody_law).
 *
 * Updates: kick-drift-kick leapfrog (leapfrog_step) and the fourth-order
 * Hermite scheme on acceleration and jerk, with a shared step (hermite_step)
 * or block individual steps (hermite_block_steps).
 *
 * Every i interacts with every j != i.  The one-sided kernels evaluate all
 * N^2 ordered pairs and scatter no pair to both partners, as the paper's
 * kernels do (Section 2, the remark on Newton's third law).  For gravity and
 * the LJC laws over a whole system, FP32 pair arithmetic, the symmetric pair
 * tiles (j_stage 2,
 * the default for the forces from N = 32,768 to 2,097,152) evaluate each unordered pair once
 * and apply it to both particles through per-block partial sums that a
 * fixed-order reduction adds, without atomics; the batched entry point has
 * symmetric tiles of its own for gravity and LJC ensembles.  Either
 * way results are deterministic run to run.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (memory of the GPU that is current
 *    when the call is made) unless marked "host".  All are FP64, row-major:
 *    pos/vel/acc/force [N][3], params [N][P] with P = 1 (gravity: m_i) or
 *    P = 3 (LJC: q_i, sigma_i, epsilon_i).
 *  - The caller owns every array and the workspace `ws` (size from
 *    nbody_workspace_bytes).  The library keeps no pointer to them after
 *    the call returns.  `law`, `offsets` and `cfg` are host memory read
 *    before the call returns.  The only device memory the library allocates
 *    is the plan tables of the batched entry points: one copy per ensemble
 *    (offsets) and launch shape per device, made at that ensemble's first
 *    launch and kept until the process ends, at most 256 MiB per device
 *    (past that, tables go through the workspace at every launch).
 *  - Outputs must not alias inputs (leapfrog_step updates pos/vel/acc in
 *    place by design).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    default stream).  Outputs are valid after the stream is synchronised.
 *    Calls on different streams with different workspaces may overlap.
 *  - Inputs are FP64.  FP32 precisions round positions and parameters to FP32
 *    once (in the pack step) and compute the pair arithmetic in FP32; the
 *    per-particle sums are carried per j-tile in FP32 and folded into an FP64
 *    (NBODY_FP32_FP64ACC) or Kahan-compensated FP32 (NBODY_FP32_KAHAN) running
 *    sum (Section 3.2: double precision only where needed).  Outputs are FP64.
 *  - Return value: NBODY_OK (0) or a negative error code.  Arguments are
 *    validated before anything is enqueued, so an error leaves every output
 *    untouched.  nbody_last_error() gives the message of the last failure on
 *    the calling thread.  Device faults surface at the next synchronisation.
 *  - N = 0 is a no-op; N = 1 yields zero force and zero potential.
 *    Coincident particles with zero softening (gravity) or any two LJC atoms
 *    at distance 0 give Inf/NaN, as the mathematical definition does.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define NBODY_OK 0
#define NBODY_EINVAL (-1)      /* bad argument: NULL pointer, N < 0, bad enum, ... */
#define NBODY_ENOTSUP (-2)     /* law/precision/entry-point combination not provided */
#define NBODY_EWORKSPACE (-3)  /* workspace NULL or smaller than nbody_workspace_bytes() */
#define NBODY_EHIP (-4)        /* HIP runtime or launch error (message has the HIP text) */

/* ---- laws and precisions ---- */
enum nbody_law_kind {
    NBODY_LAW_GRAVITY = 0,       /* Eq. 1 */
    NBODY_LAW_LJC_LINEAR = 1,    /* Table 1 LJC (linear): dielectric D r */
    NBODY_LAW_LJC_CONSTANT = 2,  /* Table 1 LJC (constant): dielectric D */
    NBODY_LAW_LJC_SIGMOIDAL = 3  /* Table 1 LJC (sigmoidal): dielectric zeta(r), see nbody_law */
};

enum nbody_precision {
    NBODY_FP64 = 0,          /* FP64 pair arithmetic, compensated FP64 sums (reference pass) */
    NBODY_FP32_KAHAN = 1,    /* FP32 pairs, FP32 tile partials, Kahan-compensated FP32 running sum */
    NBODY_FP32_FP64ACC = 2,  /* FP32 pairs, FP32 tile partials, FP64 running sum */
    NBODY_FP32_PLAIN = 3     /* FP32 pairs, one plain FP32 running sum (accuracy ablation only) */
};

/* Law parameters (host struct).  `softening` is the length eps of Eq. 1 (the
 * kernel adds eps^2 to r^2, as the Appendix listing adds its constant).
 * `coulomb_k` is k (332.0637 kcal A / (mol e^2) for Angstrom/kcal/e units) and
 * `dielectric` is D in eps(r) = D r (LJC linear) or eps = D (LJC constant).
 * LJC(sigmoidal) uses zeta(r) = exp(zeta[0] r^3 + zeta[1] r^2 + zeta[2] r +
 * zeta[3]) (Table 1's exponent, whose printed "gamma + delta" is read as
 * gamma r + delta; the paper gives no constants) with the potential
 * u = k q_i q_j / (zeta(r) r) + LJ and F = -grad U:
 *   F_i = sum_j [k q_i q_j (1 + r zeta'/zeta) / (zeta r^3) + LJ] (r_i - r_j).
 * The other LJC laws: u = k q_i q_j / (D r^2) (linear), k q_i q_j / (D r)
 * (constant).  U_i = sum_j u_ij for every LJC law.  Fields a law does not
 * use are ignored. */
typedef struct nbody_law {
    int32_t kind;        /* enum nbody_law_kind */
    int32_t precision;   /* enum nbody_precision */
    double G;            /* gravity */
    double softening;    /* gravity, >= 0 */
    double coulomb_k;    /* LJC */
    double dielectric;   /* LJC linear / constant, > 0 */
    double zeta[4];      /* LJC sigmoidal, finite */
} nbody_law;

/* Entry-point ids for nbody_workspace_bytes / nbody_set_config. */
enum nbody_api {
    NBODY_API_FORCES = 0,
    NBODY_API_BATCHED = 1,
    NBODY_API_BACKWARD = 2,
    NBODY_API_LEAPFROG = 3,
    NBODY_API_JERK = 4,       /* nbody_forces_jerk */
    NBODY_API_HERMITE = 5,    /* hermite_step, hermite_block_steps */
    NBODY_API_BACKWARD_BATCHED = 6   /* nbody_forces_backward_batched */
};

/* Per-particle exclusion lists for bonded molecular systems (Section 5: the
 * LJC kernels read an exclusion list for each particle).  Particle x leaves
 * out of its sums every particle listed in index[offsets[x] .. offsets[x+1])
 * (caller particle indices; any order; repeats allowed).  Bonded topologies
 * give symmetric lists (y in x's list exactly when x is in y's), which keeps
 * Newton's third law; the adjoint assumes symmetric lists.
 *  offsets  [n + 1] device int64, non-decreasing, offsets[0] = 0;
 *  index    [count] device int64 (may be NULL when count == 0);
 *  count    number of entries of index.
 * List ranges are clamped to [0, count) and entries are only compared, never
 * dereferenced, so entries outside [0, n) (or naming another system of a
 * batch) have no effect. */
typedef struct nbody_exclusions {
    const int64_t *offsets;
    const int64_t *index;
    int64_t count;
} nbody_exclusions;

/* Launch configuration of the all-pairs kernels (see nbody_set_config).
 *  block      threads per workgroup, a multiple of 64 in [64, 256];
 *  i_per_lane i-particles held in registers by each lane: 1, 2, 4 or 8
 *             (the i-unrolling of Section 3.3, "4x4" kernels);
 *  j_tile     j-particles per FP32 partial sum before it is folded into the
 *             compensated running sum: a multiple of 64;
 *  j_split    number of disjoint j ranges evaluated by separate waves and
 *             added afterwards in a fixed order (the i-replication of
 *             Section 3.4), 1..64; a launch uses at most one part per 64
 *             j records and at most 2^25 / rows parts (the partial buffer of
 *             the workspace).  For the batched entry points, the number of
 *             work units per resident wave the planner aims at, 1..64 (the
 *             j ranges of large systems are cut into parts to reach it: more
 *             parts balance the persistent launch, fewer leave fewer part
 *             sums to add; 8 by the rule);
 *  j_stage    how j records reach the arithmetic: 0 = wave-uniform scalar
 *             loads into SGPRs, 1 = a wave-private LDS slot read back as
 *             broadcasts into VGPRs (so the pair arithmetic has only VGPR
 *             operands), 2 = symmetric pair tiles: each unordered pair is
 *             evaluated once and its force applied to both particles
 *             (Newton's third law), for gravity with FP32_KAHAN or
 *             FP32_FP64ACC through nbody_forces, leapfrog_step and
 *             nbody_forces_backward (the position adjoint, whose pair term
 *             for one particle is minus the other's), and for the three LJC
 *             laws with those precisions through nbody_forces and
 *             leapfrog_step (no exclusion lists), on whole systems of up
 *             to 2,097,152 particles (its per-block partials
 *             grow as n^2: 8.6 GB at n = 2^20, 34 GB at 2^21; elsewhere 2
 *             reads as 1).  For nbody_forces_batched, j_stage 2 selects the
 *             batched symmetric tiles (gravity and the LJC laws with
 *             FP32_KAHAN or FP32_FP64ACC, no exclusion lists, every system of
 *             at most 8192 particles; otherwise the launch runs one-sided),
 *             in a fixed shape (block 256, i_per_lane 4, j_tile 256, j_split
 *             1): one wave per pair of 256-record blocks of a system, each
 *             unordered pair once; the rule's choice when systems average 512
 *             particles or more.  With j_stage 2 (single systems), j_tile
 *             is the tile edge in records, 1024 (for n <= 262,144) or 2048;
 *             block and i_per_lane pick the workgroup shape, (512, 2) for 8
 *             waves of 2 i chunks or (256, 4) for 4 waves of 4; and j_split
 *             cuts each tile's j chunks into 1, 2 or 4 parts run by workgroups
 *             of their own (for n <= 131,072, each part at least as many
 *             64-record chunks as the workgroup has waves; otherwise 1): more
 *             parts fill the chip's last round of tiles better and leave more
 *             slot partials for the reduction to read.  The requested value is
 *             rounded down to the nearest allowed one. */
typedef struct nbody_config {
    int32_t block;
    int32_t i_per_lane;
    int32_t j_tile;
    int32_t j_split;
    int32_t j_stage;
} nbody_config;

/* Forces and potential of one system (Section 2 all-pairs loop; Eq. 1 or
 * Table 1 LJC(linear)).
 *  pos        [n][3] device, FP64 positions.
 *  params     [n][P] device, per-particle parameters (P = 1 or 3, see above).
 *  n          number of particles, >= 0.
 *  law        host, law and precision.
 *  out_force  [n][3] device: accelerations a_i (gravity) or forces F_i (LJC).
 *  out_potential [n] device or NULL: phi_i (gravity, per unit mass) or U_i (LJC).
 *  ws/ws_bytes  device workspace of at least
 *             nbody_workspace_bytes(NBODY_API_FORCES, n, 1, law) bytes.
 *  stream     hipStream_t or NULL.
 * Errors: NBODY_EINVAL (NULL pos/params/out_force/law with n > 0, n < 0,
 * negative softening, D <= 0, bad enum), NBODY_EWORKSPACE, NBODY_EHIP. */
int nbody_forces(const double *pos, const double *params, int64_t n, const nbody_law *law,
                 double *out_force, double *out_potential, void *ws, size_t ws_bytes,
                 void *stream);

/* nbody_forces without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It allocates nothing: its records and split partials
 * live in a device scratch area of 64 MiB that the library holds on each GPU
 * it runs on until the process ends (looked up once per device on the first
 * call there).  The arguments mean what they mean for nbody_forces; the
 * result is the same evaluation, up to the rounding of a j split that may be
 * smaller (so that its partials fit the scratch area).
 * Limit: n <= 67,108,864 / record bytes - 64, i.e. 4,194,240 particles for
 * FP32 gravity, 2,097,088 for FP32 LJC and FP64 gravity, 1,048,512 for FP64
 * LJC; larger n is refused with NBODY_EINVAL before anything is enqueued.
 * Every call on one GPU uses that GPU's one scratch area: calls that overlap
 * on one GPU (on different streams or from different threads) race and must
 * be serialised by the caller.  Nothing in the area needs to start at zero.
 * Errors: as nbody_forces, without NBODY_EWORKSPACE. */
int nbody_forces_noalloc(const double *pos, const double *params, int64_t n, const nbody_law *law,
                         double *out_force, double *out_potential, void *stream);

/* Forces on an active subset of particles (the block time step of
 * Section 3.4: forces on a subset of i against all j).  `ilist` [ni] device
 * int64 holds indices in [0, n) (repeats allowed); row k of the outputs is
 * the force and potential of particle ilist[k].  Outputs are [ni][3] and [ni].
 * Workspace: nbody_workspace_bytes(NBODY_API_FORCES, max(n, ni), 1, law). */
int nbody_forces_subset(const double *pos, const double *params, int64_t n, const int64_t *ilist,
                        int64_t ni, const nbody_law *law, double *out_force,
                        double *out_potential, void *ws, size_t ws_bytes, void *stream);

/* One share of a gravity or LJC evaluation, for a caller that spreads one system
 * over several GPUs (each GPU holds every particle and evaluates one share;
 * summing the shares' outputs gives the forces).  The unordered pairs are
 * cut as the symmetric pair tiles cut them (Section 2's all-pairs sum with
 * each pair applied to both particles): the upper triangle of the grid of
 * blocks of 1024 (n <= 262,144) or 2048 records, walked in a fixed order,
 * is split into n_shares ranges of equal tile count, and share `share`
 * evaluates the tiles of its range.  out_force [n][3] and out_potential [n]
 * (optional) receive, for EVERY row, the FP64 sum of that row's contributions
 * from the share's tiles, scaled as nbody_forces scales them (G, -G for
 * gravity; 1 and 1/2 or 1 for LJC); rows
 * the share does not touch get zero.  The sum over all shares equals
 * nbody_forces' result up to the rounding of the final FP64 additions; with
 * n_shares = 1 it is that result.
 *  share, n_shares   0 <= share < n_shares.
 * Law: any, with NBODY_FP32_KAHAN or NBODY_FP32_FP64ACC, n <= 2,097,152
 * (NBODY_ENOTSUP otherwise: FP64 and FP32_PLAIN shard by rows, with
 * nbody_forces_subset on a contiguous row list).  Workspace:
 * nbody_workspace_bytes(NBODY_API_FORCES, n, 1, law).  Errors: as
 * nbody_forces, and NBODY_EINVAL for a share outside [0, n_shares). */
int nbody_forces_share(const double *pos, const double *params, int64_t n, const nbody_law *law,
                       int32_t share, int32_t n_shares, double *out_force, double *out_potential,
                       void *ws, size_t ws_bytes, void *stream);

/* Forces of many independent systems of uneven size in ONE persistent launch
 * (small-system motivation of Section 3.4).  System s owns rows
 * [offsets[s], offsets[s+1]) of pos/params/out_*; particles interact only
 * within their system.
 *  offsets    host int64 [n_systems + 1], offsets[0] = 0, non-decreasing.
 *  n_systems  S >= 0 (empty systems are allowed).
 * Other arguments as nbody_forces with N = offsets[S].  Workspace:
 * nbody_workspace_bytes(NBODY_API_BATCHED, offsets[S], S, law).
 * Plan tables: the first launch of an ensemble plans its work units on the
 * host and uploads the tables once (synchronously) into device memory the
 * library keeps; later launches of the same ensemble copy nothing from the
 * host, so they can be captured in a graph (a captured launch reads those
 * tables at every replay).  A first launch inside a stream capture is
 * refused with NBODY_EINVAL before anything is enqueued.
 * Decompositions (nbody_config.j_stage): one-sided units of rows against
 * parts of their system's j range (each ordered pair evaluated), or, for
 * every law with FP32 pair arithmetic and systems of at most
 * 8192 particles, symmetric tiles of 256 x 256 records (each unordered pair
 * of a system evaluated once, per-system FP32 slot partials added in a fixed
 * order in FP64).  The workspace covers both: for those laws it holds up to
 * 512 bytes of slot partials per particle (32 slots of 16 bytes). */
int nbody_forces_batched(const int64_t *offsets, int64_t n_systems, const double *pos,
                         const double *params, const nbody_law *law, double *out_force,
                         double *out_potential, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of nbody_forces (not in the paper; the derivative of the same
 * laws).  Given g = dL/d(out_force) [n][3] device:
 *  grad_pos    [n][3] device or NULL: dL/dr_k.  For gravity this is the
 *              Hessian-vector product
 *                dL/dr_k = G sum_{j!=k} K(d)(m_k g_j - m_j g_k),
 *                K(d)v = v/s^3 - 3 (d.v) d / s^5,  d = r_j - r_k;
 *              for LJC, with F_i = sum_j w(r) d_ij,
 *                dL/dr_k = sum_{j!=k} [w u + (w'/r)(d.u) d],  u = g_j - g_k.
 *  grad_params [n][P] device or NULL: LJC only, per-atom dL/dq, dL/dsigma,
 *              dL/depsilon (gravity: must be NULL).  The mixing rule
 *              eps_ij = sqrt(eps_i eps_j) has no finite derivative at
 *              eps_k = 0: an atom with epsilon 0 gets a non-finite
 *              dL/depsilon (its other gradients are unaffected).
 *  types, n_types, grad_type_params: optional (LJC only).  When types
 *              (device int32 [n], values in [0, n_types)) is non-NULL,
 *              grad_type_params [n_types][2] device receives the sums of
 *              dL/dsigma and dL/depsilon over the atoms of each type (the
 *              gradient with respect to per-type sigma and epsilon), reduced
 *              in a fixed order.  At most 16384 types (NBODY_ENOTSUP
 *              beyond); atoms whose type is outside [0, n_types) are not
 *              counted.
 * Swapping k and j negates both d and m_k g_j - m_j g_k, so gravity's pair
 * term for j is minus its term for k: with FP32 pair arithmetic and 65,536
 * to 2,097,152 particles the rule evaluates each unordered pair once
 * (symmetric pair tiles, as the forward's).  LJC(linear)'s position terms
 * of the two atoms are likewise opposite and its charge, sigma and epsilon
 * terms share one scalar: with FP32 pair arithmetic, no exclusion lists and
 * 16,384 to 262,144 atoms the rule evaluates each unordered pair once too
 * (j_stage 2: the batched backward's tiles of 256 x 256 records over the one
 * system; any size up to 262,144 when forced).
 * Workspace: nbody_workspace_bytes(NBODY_API_BACKWARD, n, 1, law); for
 * LJC(linear) with FP32 and n <= 262,144 it covers 32 bytes of slot
 * partials per atom and 256-record block (8 GiB at 262,144).
 * Laws: gravity and LJC(linear) (other laws: NBODY_ENOTSUP).
 * Precisions: NBODY_FP64, NBODY_FP32_FP64ACC, NBODY_FP32_KAHAN. */
int nbody_forces_backward(const double *pos, const double *params, int64_t n,
                          const nbody_law *law, const double *grad_force, double *grad_pos,
                          double *grad_params, const int32_t *types, int32_t n_types,
                          double *grad_type_params, void *ws, size_t ws_bytes, void *stream);

/* nbody_forces with exclusion lists (LJC laws; NBODY_ENOTSUP for gravity and
 * NBODY_FP32_PLAIN).  `excl` (host struct, device arrays) must be non-NULL.
 * Workspace: nbody_workspace_bytes(NBODY_API_FORCES, n, 1, law). */
int nbody_forces_excl(const double *pos, const double *params, int64_t n,
                      const nbody_exclusions *excl, const nbody_law *law, double *out_force,
                      double *out_potential, void *ws, size_t ws_bytes, void *stream);

/* nbody_forces_batched with exclusion lists over the concatenated rows
 * (offsets / index name rows of pos; partners outside a row's own system are
 * ignored).  Laws and precisions as nbody_forces_excl.  Workspace:
 * nbody_workspace_bytes(NBODY_API_BATCHED, offsets[S], S, law).  Plan tables
 * as nbody_forces_batched. */
int nbody_forces_batched_excl(const int64_t *offsets, int64_t n_systems, const double *pos,
                              const double *params, const nbody_exclusions *excl,
                              const nbody_law *law, double *out_force, double *out_potential,
                              void *ws, size_t ws_bytes, void *stream);

/* nbody_forces_backward with (symmetric) exclusion lists, LJC(linear) only:
 * the adjoint of nbody_forces_excl.  Workspace as nbody_forces_backward. */
int nbody_forces_backward_excl(const double *pos, const double *params, int64_t n,
                               const nbody_exclusions *excl, const nbody_law *law,
                               const double *grad_force, double *grad_pos, double *grad_params,
                               const int32_t *types, int32_t n_types, double *grad_type_params,
                               void *ws, size_t ws_bytes, void *stream);

/* The adjoint of nbody_forces_batched (or, with excl != NULL, of
 * nbody_forces_batched_excl): many independent systems in ONE persistent
 * launch, as the batched forward.  Arguments as nbody_forces_backward over
 * the concatenated rows; with types, grad_type_params sums over the atoms of
 * each type across all systems.  Laws: gravity and LJC(linear) (exclusions:
 * LJC(linear)).  Decompositions as nbody_forces_batched: one-sided units,
 * or, with FP32 pair arithmetic, no exclusion lists and every system of at
 * most 8192 particles, symmetric tiles of 256 x 256 records (j_stage 2, the
 * rule's choice when systems average 512 particles or more): each unordered
 * pair's adjoint terms evaluated once and applied to both particles (the
 * position terms of the two are opposite; the charge, sigma and epsilon
 * terms share one scalar), per-system FP32 slot partials added in a fixed
 * order in FP64.  Workspace:
 * nbody_workspace_bytes(NBODY_API_BACKWARD_BATCHED, offsets[S], S, law).
 * Plan tables as nbody_forces_batched (shared with it for the same ensemble
 * and launch shape). */
int nbody_forces_backward_batched(const int64_t *offsets, int64_t n_systems, const double *pos,
                                  const double *params, const nbody_exclusions *excl,
                                  const nbody_law *law, const double *grad_force, double *grad_pos,
                                  double *grad_params, const int32_t *types, int32_t n_types,
                                  double *grad_type_params, void *ws, size_t ws_bytes, void *stream);

/* `nsteps` kick-drift-kick leapfrog steps in FP64 (the force-evaluation /
 * update-step cycle of Section 1):
 *   v += dt/2 a;  x += dt v;  a = accel(x);  v += dt/2 a.
 *  pos, vel    [n][3] device, updated in place.
 *  acc         [n][3] device: a(t) on entry, a(t + nsteps dt) on exit.
 *  inv_mass    [n] device or NULL: acceleration = force * inv_mass (LJC);
 *              NULL means the law's output is already an acceleration
 *              (gravity) or unit masses.
 *  out_potential [n] device or NULL: potential at the final positions.
 * Forces use `law->precision`; the update is always FP64.  nsteps >= 0.
 * Workspace: nbody_workspace_bytes(NBODY_API_LEAPFROG, n, 1, law). */
int leapfrog_step(double *pos, double *vel, double *acc, const double *params,
                  const double *inv_mass, int64_t n, const nbody_law *law, double dt,
                  int32_t nsteps, double *out_potential, void *ws, size_t ws_bytes,
                  void *stream);

/* Acceleration, jerk and potential of softened gravity (Table 1 "Gravity
 * (accel & jerk)", the GAJ kernel of Section 2), for every particle or for an
 * index list of them:
 *   a_i    =  G sum_{j!=i} m_j d / s^3
 *   jerk_i =  G sum_{j!=i} m_j [ w / s^3 - 3 (d.w) d / s^5 ]
 *   phi_i  = -G sum_{j!=i} m_j / s,
 *   d = r_j - r_i,  w = v_j - v_i,  s^2 = |d|^2 + eps^2.
 *  pos, vel   [n][3] device; mass [n] device.
 *  ilist      [ni] device int64 indices in [0, n) (repeats allowed), or NULL
 *             for every particle (then ni must equal n).  Row k of the
 *             outputs belongs to particle ilist[k].
 *  law        host; kind NBODY_LAW_GRAVITY; precision NBODY_FP64,
 *             NBODY_FP32_FP64ACC or NBODY_FP32_KAHAN (else NBODY_ENOTSUP).
 *  out_acc, out_jerk [ni][3] device; out_potential [ni] device or NULL.
 * Swapping i and j negates d, w and the bracket and leaves s unchanged, so
 * each unordered pair's terms serve both particles: for every particle
 * (ilist NULL), FP32 pair arithmetic and up to 524,288 particles,
 * nbody_config.j_stage 2 selects symmetric pair tiles (blocks of 1024
 * records, 8 waves of 2 i chunks, 1 or 2 j parts per tile; FP32 slot
 * partials per row and block added in a fixed order in FP64), the rule's
 * choice from 32,768 particles; an index list runs one-sided.
 * Workspace: nbody_workspace_bytes(NBODY_API_JERK, max(n, ni), 1, law); for
 * FP32 and n <= 524,288 it covers the tiles' records padded to whole blocks
 * and 32 bytes of slot partials per particle, block and part (1 GiB at
 * 2^17, 8 GiB at 2^19). */
int nbody_forces_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                      const int64_t *ilist, int64_t ni, const nbody_law *law, double *out_acc,
                      double *out_jerk, double *out_potential, void *ws, size_t ws_bytes,
                      void *stream);

/* `nsteps` shared steps h = dt of the fourth-order Hermite predictor-
 * corrector (Makino & Aarseth 1992), the integrator that acceleration and
 * jerk serve (the paper names none):
 *   predict  xp = x + v h + a h^2/2 + j h^3/6,  vp = v + a h + j h^2/2
 *   a1, j1 = acceleration and jerk at (xp, vp) of every particle
 *   a2 = (-6 (a - a1) - h (4 j + 2 j1)) / h^2,  a3 = (12 (a - a1) + 6 h (j + j1)) / h^3
 *   correct  x = xp + a2 h^4/24 + a3 h^5/120,  v = vp + a2 h^3/6 + a3 h^4/24,
 *            a = a1, jerk = j1.
 *  pos, vel, acc, jerk [n][3] device, updated in place; acc and jerk hold
 *  the values at the entry state (e.g. from nbody_forces_jerk).  mass [n]
 *  device.  law as nbody_forces_jerk.  dt > 0 finite, nsteps >= 0.  The
 *  update is FP64; the pair arithmetic follows law->precision.  Each step
 *  evaluates every particle as nbody_forces_jerk would for the whole system
 *  where its configuration (NBODY_API_JERK) selects the symmetric tiles,
 *  and otherwise with the NBODY_API_HERMITE configuration.
 * Workspace: nbody_workspace_bytes(NBODY_API_HERMITE, n, 1, law). */
int hermite_step(double *pos, double *vel, double *acc, double *jerk, const double *mass,
                 int64_t n, const nbody_law *law, double dt, int32_t nsteps, void *ws,
                 size_t ws_bytes, void *stream);

/* Initial block time steps for hermite_block_steps: t_i = 0 and dt_i = the
 * largest dt_max / 2^k not above eta_s |a_i| / |jerk_i| (dt_max where
 * jerk_i = 0).  acc, jerk [n][3] device; t_i, dt_i [n] device outputs.
 * dt_max must be a power of two; eta_s > 0. */
int hermite_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                       double dt_max, double *t_i, double *dt_i, void *stream);

/* Up to `nblocks` block steps of the Hermite scheme with individual block
 * time steps: the setting in which Section 3.4 evaluates forces on a subset
 * of the particles.  One block step:
 *   t = min_i (t_i + dt_i); the due set A = { i : t_i + dt_i == t };
 *   every particle is predicted to t from its own t_i (predictor above);
 *   acceleration and jerk of each i in A against all predicted particles;
 *   each i in A is corrected over h = dt_i, gets t_i = t and the next step
 *     dt* = sqrt(eta (|a1| |a2'| + |j1|^2) / (|j1| |a3| + |a2'|^2)),
 *     a2' = a2 + a3 h (Aarseth's criterion), quantised to the largest
 *     dt_max / 2^k <= dt* that is at most 2 h and divides t.
 * A block step whose time t would exceed t_end is not taken: it and every
 * later one leave all state untouched (pass +Inf for no bound).
 *  pos, vel, acc, jerk [n][3], t_i, dt_i [n]: device, updated in place
 *    (t_i, dt_i from hermite_block_init or a previous call).
 *  mass [n] device; law as nbody_forces_jerk; eta > 0; dt_max as given to
 *    hermite_block_init (a power of two); t_end not NaN.
 *  active_counts host int64 [nblocks] or NULL: |A| of each block step, 0 for
 *    the steps not taken.
 *  t_now host or NULL: the time of the last block step taken (left as it is
 *    when none is).
 * The scheduling (the next time, the due list in increasing index order and
 * the j split for |A| rows) runs on the device, and the launches read |A|
 * from device memory, so block steps are enqueued without waiting for one
 * another.  The call reads the due counts back (one synchronisation of
 * `stream` per batch of up to 1024 block steps, batches growing from 8) and
 * returns once a step is not taken or nblocks steps are done.
 * Workspace: nbody_workspace_bytes(NBODY_API_HERMITE, n, 1, law). */
int hermite_block_steps(double *pos, double *vel, double *acc, double *jerk, double *t_i,
                        double *dt_i, const double *mass, int64_t n, const nbody_law *law,
                        double eta, double dt_max, double t_end, int32_t nblocks,
                        int64_t *active_counts, double *t_now, void *ws, size_t ws_bytes,
                        void *stream);

/* Workspace size in bytes needed by entry point `api` for `n_total`
 * particles in `n_systems` systems (1 for the single-system entry points).
 * For every law with FP32_KAHAN or FP32_FP64ACC through the forces and
 * leapfrog entry points (and gravity's backward), n <= 2,097,152,
 * it covers the symmetric pair tiles (j_stage
 * 2), whose FP32 partial buffer holds one partial per row and block of 2048
 * records: about n^2 / 128 bytes (8.6 GB at n = 2^20); up to n = 262,144 it
 * covers blocks of 1024 records (n^2 / 64 bytes), and up to n = 131,072 tiles
 * in 4 j parts (n^2 / 16 bytes, 1.1 GB at n = 2^17).  Returns 0 when the
 * arguments are invalid. */
size_t nbody_workspace_bytes(int32_t api, int64_t n_total, int64_t n_systems,
                             const nbody_law *law);

/* Message of the last non-OK return on the calling thread ("" if none). */
const char *nbody_last_error(void);

/* ---- tuning (the unroll sweep of Section 3.3 and the replication sweep of
 * Section 3.4, done by measurement) ---- */

/* Force the launch configuration used by entry point `api` (cfg != NULL), or
 * return to the automatic choice (cfg == NULL).  Host struct.  Returns
 * NBODY_EINVAL for a configuration outside the documented ranges. */
int nbody_set_config(int32_t api, const nbody_config *cfg);

/* The configuration entry point `api` would use for n particles in
 * n_systems systems under `law`, written to *out (host). */
int nbody_get_config(int32_t api, int64_t n, int64_t n_systems, const nbody_law *law,
                     nbody_config *out);

/* Time candidate configurations on the given problem with HIP events on
 * `stream` and remember the fastest for this (device, law, precision, entry
 * point, size class).  Arguments as nbody_forces (api = NBODY_API_FORCES) or
 * nbody_forces_batched (api = NBODY_API_BATCHED, offsets/n_systems used);
 * the outputs are overwritten with the result of the winning configuration.
 * Synchronises the stream.  `out_best` (host, may be NULL) receives the
 * winner and `out_ms` (host, may be NULL) its time in milliseconds. */
int nbody_autotune(int32_t api, const int64_t *offsets, int64_t n_systems, const double *pos,
                   const double *params, int64_t n, const nbody_law *law, double *out_force,
                   double *out_potential, void *ws, size_t ws_bytes, void *stream,
                   nbody_config *out_best, double *out_ms);

/* As nbody_autotune for nbody_forces_jerk over all n particles (arguments as
 * nbody_forces_jerk with ilist = NULL); the winner is remembered for
 * NBODY_API_JERK and used by the Hermite steps of the same size class. */
int nbody_autotune_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                        const nbody_law *law, double *out_acc, double *out_jerk,
                        double *out_potential, void *ws, size_t ws_bytes, void *stream,
                        nbody_config *out_best, double *out_ms);

/* Save / load the tuning cache as a small JSON file (host path).  The file
 * records the device's architecture name and compute-unit count; loading a
 * file written for another architecture or CU count returns NBODY_EINVAL and
 * loads nothing (tuned launch shapes do not carry over between devices).
 * Saving writes a temporary file beside `path` and renames it over `path`, so
 * a concurrent reader sees the old file or the new one, never part of one.
 *
 * Environment: when NBODY_TUNE_CACHE names a file, the library loads it at
 * the first configuration lookup of the process (if the file exists; a file
 * for another device is skipped with one line on stderr) and saves the whole
 * cache to it after every successful nbody_autotune / nbody_autotune_jerk, so
 * tuned shapes carry over between processes on the same device. */
int nbody_tune_save(const char *path);
int nbody_tune_load(const char *path);

/* ---- measurement hooks ---- */

/* When enabled, every launch of the all-pairs kernel is bracketed by HIP
 * events on the launch stream and its duration is accumulated. */
int nbody_timing_enable(int32_t on);
/* Total milliseconds and number of all-pairs kernel launches recorded since
 * the last reset; synchronises the recorded events.  reset != 0 clears. */
int nbody_timing_read(double *total_ms, int64_t *launches, int32_t reset);

/* Algorithmic flops per pair interaction counted from the kernel's own
 * instruction sequence (multiply-add = 2, rsqrt/rcp = 1, the Appendix
 * convention), for the given law, potential on/off and entry point. */
int32_t nbody_flops_per_pair(int32_t api, int32_t law_kind, int32_t with_potential);

/* Library version string. */
const char *nbody_version(void);

/* ---- issue-rate probes (measurement support for the roofline; not part of
 * the force path) ---- */

/* Device workspace bytes nbody_probe_issue_rates needs. */
size_t nbody_probe_workspace_bytes(void);

/* Measure, on the current device, the shader cycles a SIMD spends per wave64
 * instruction at eight waves per SIMD, each probe running independent chains
 * per lane (four untimed launches, then three timed ones of about a
 * millisecond, each taken at its own measured clock; the median is reported):
 *   out[0] v_fma_f32 with all operands in VGPRs (shared multiplier/addend)
 *   out[1] v_fma_f32 with one SGPR operand
 *   out[2] v_rsq_f32
 *   out[3] the shader clock in GHz while the out[0] probe runs (shader-cycle
 *          counter over the fixed-rate wall counter); out[4] that counter's
 *          rate in MHz
 *   out[5] one v_rsq_f32 with 13 independent FMAs interleaved: cycles per
 *          group of 14 (an rsq that overlapped the FMAs would make this close
 *          to 13 x out[0]; no overlap makes it 13 x out[0] + out[2] or more)
 *   out[6] v_fma_f32 whose multiplier and addend are distinct VGPRs that
 *          rotate over the chains
 *   out[7] v_mov_b32 with a DPP row rotation (a cross-lane move on the VALU)
 *   out[8] ds_bpermute_b32 (a cross-lane move through the LDS crossbar)
 * out: host double[n_out], n_out >= 9; ws: device workspace of
 * nbody_probe_workspace_bytes() bytes.  Synchronises `stream`. */
int nbody_probe_issue_rates(double *out, int32_t n_out, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
