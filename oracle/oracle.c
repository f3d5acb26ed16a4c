/*
 * FP64 CPU oracle for the all-pairs N-body force evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library; the two meet only at the seeded input arrays.
 *
 * Every function is the plain definition written out: a double loop over the
 * requested i and every j != i (Section 2, the naive all-pairs pseudo-code),
 * pair arithmetic in IEEE double (built with -ffp-contract=off, no fast-math),
 * and a Neumaier-compensated sum over j so that the reference itself is not
 * the dominant error when force terms cancel.  OpenMP runs over i only; the
 * j order is 0..N-1 for every i, so results do not depend on thread count.
 *
 * Readings of the paper used here, where it is silent or its printed form is
 * ambiguous:
 *   - displacement d_ij = r_j - r_i; gravity attracts (Eq. 1 with the
 *     Appendix listing's d = jpos - ipos and "+=");
 *   - the softening constant added to r^2 in the Appendix listing is eps^2,
 *     eps being the softening length passed in;
 *   - the softened potential phi_i = -G sum_j m_j / sqrt(r^2 + eps^2) whose
 *     negative gradient is Eq. 1;
 *   - LJC(linear) of Table 1 is read potential-consistently: pair energy
 *     u = k q_i q_j / (D r^2) + 4 e_ij [(s_ij/r)^12 - (s_ij/r)^6] with
 *     Lorentz-Berthelot combining s_ij = (s_i+s_j)/2, e_ij = sqrt(e_i e_j),
 *     and force F_i = -grad_i of the total energy.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- compensated summation (Neumaier's improvement of Kahan's method) ---- */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nval(const nsum *a) { return a->s + a->c; }

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    /* 0 restores the count OpenMP started with (OMP_NUM_THREADS or the
     * processor count), so that a request for one thread does not stick */
    static int initial = 0;
    if (initial == 0) initial = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : initial);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Number of threads the oracle's parallel loops will use after a call with
 * the given request (0 = OpenMP default). */
int oracle_threads(int nthreads) { return set_threads(nthreads); }

static inline int64_t row(const int64_t *ilist, int64_t k) { return ilist ? ilist[k] : k; }

/* Exclusion lists (Section 5: the LJC kernels read an exclusion list for each
 * particle).  Pair (i, j) is left out of particle i's sums when j appears in
 * eidx[eoff[i] .. eoff[i+1]).  eoff == NULL means no exclusions. */
static inline int excluded(const int64_t *eoff, const int64_t *eidx, int64_t i, int64_t j)
{
    if (!eoff) return 0;
    for (int64_t e = eoff[i]; e < eoff[i + 1]; ++e)
        if (eidx[e] == j) return 1;
    return 0;
}

/* ------------------------------------------------------------------------
 * Softened gravity, Eq. 1 (Section 3.3) and Table 1 row "Gravity (accel)".
 *   a_i   = G sum_{j != i, j0 <= j < j1} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}
 *   phi_i = -G sum_{same j} m_j / (|r_j - r_i|^2 + eps^2)^{1/2}
 * i runs over ilist[0..ni) (or 0..ni when ilist is NULL).  The j range
 * [j0, j1) exists so that the i-replication identity of Section 3.4
 * (partial sums over disjoint j ranges add up to the full sum) can be
 * checked.  acc is [ni][3]; phi is [ni] or NULL.
 * ---------------------------------------------------------------------- */
int oracle_gravity(const double *pos, const double *mass, int64_t n, double G, double eps,
                   const int64_t *ilist, int64_t ni, int64_t j0, int64_t j1,
                   double *acc, double *phi, int nthreads)
{
    if (n < 0 || ni < 0 || j0 < 0 || j1 > n || j0 > j1) return -1;
    set_threads(nthreads);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ni; ++k) {
        const int64_t i = row(ilist, k);
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
        for (int64_t j = j0; j < j1; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * j] - xi;
            const double dy = pos[3 * j + 1] - yi;
            const double dz = pos[3 * j + 2] - zi;
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double inv_s3 = 1.0 / (s2 * s);
            nadd(&ax, mass[j] * dx * inv_s3);
            nadd(&ay, mass[j] * dy * inv_s3);
            nadd(&az, mass[j] * dz * inv_s3);
            nadd(&ph, mass[j] / s);
        }
        acc[3 * k] = G * nval(&ax);
        acc[3 * k + 1] = G * nval(&ay);
        acc[3 * k + 2] = G * nval(&az);
        if (phi) phi[k] = -G * nval(&ph);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * LJ + Coulomb with a linear distance-dependent dielectric eps(r) = D r
 * (Table 1 row "LJC (linear)"; Section 2 on continuum-solvent models).
 *   u_ij = kc q_i q_j / (D r^2) + 4 e_ij [(s_ij/r)^12 - (s_ij/r)^6]
 *   F_i  = sum_{j != i} [ 2 kc q_i q_j / (D r^4)
 *                         + (24 e_ij / r^2) (2 (s_ij/r)^12 - (s_ij/r)^6) ] (r_i - r_j)
 *   U_i  = sum_{j != i} u_ij      (total potential energy = U_tot = 1/2 sum_i U_i)
 * params per atom: q (charge), sigma, epsilon.  force is [ni][3], energy
 * [ni] or NULL.
 * ---------------------------------------------------------------------- */
static int ljc_linear_impl(const double *pos, const double *q, const double *sigma,
                           const double *epsl, int64_t n, double kc, double D,
                           const int64_t *ilist, int64_t ni, int64_t j0, int64_t j1,
                           const int64_t *eoff, const int64_t *eidx,
                           double *force, double *energy, int nthreads)
{
    if (n < 0 || ni < 0 || j0 < 0 || j1 > n || j0 > j1) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ni; ++k) {
        const int64_t i = row(ilist, k);
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, en = {0, 0};
        for (int64_t j = j0; j < j1; ++j) {
            if (j == i || excluded(eoff, eidx, i, j)) continue;
            const double rx = xi - pos[3 * j];
            const double ry = yi - pos[3 * j + 1];
            const double rz = zi - pos[3 * j + 2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double sij = 0.5 * (sigma[i] + sigma[j]);
            const double eij = sqrt(epsl[i] * epsl[j]);
            const double sr2 = sij * sij / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double sr12 = sr6 * sr6;
            const double coul = kc * q[i] * q[j] / D;          /* u_C = coul / r^2 */
            const double W = 2.0 * coul / (r2 * r2) + 24.0 * eij / r2 * (2.0 * sr12 - sr6);
            nadd(&fx, W * rx);
            nadd(&fy, W * ry);
            nadd(&fz, W * rz);
            nadd(&en, coul / r2 + 4.0 * eij * (sr12 - sr6));
        }
        force[3 * k] = nval(&fx);
        force[3 * k + 1] = nval(&fy);
        force[3 * k + 2] = nval(&fz);
        if (energy) energy[k] = nval(&en);
    }
    return 0;
}

int oracle_ljc_linear(const double *pos, const double *q, const double *sigma,
                      const double *epsl, int64_t n, double kc, double D,
                      const int64_t *ilist, int64_t ni, int64_t j0, int64_t j1,
                      double *force, double *energy, int nthreads)
{
    return ljc_linear_impl(pos, q, sigma, epsl, n, kc, D, ilist, ni, j0, j1, NULL, NULL, force,
                           energy, nthreads);
}

/* ------------------------------------------------------------------------
 * LJ + Coulomb with a constant dielectric D (Table 1 row "LJC (constant)").
 *   u_ij = kc q_i q_j / (D r) + 4 e_ij [(s_ij/r)^12 - (s_ij/r)^6]
 *   F_i  = sum_{j != i} [ kc q_i q_j / (D r^3)
 *                         + (24 e_ij / r^2) (2 (s_ij/r)^12 - (s_ij/r)^6) ] (r_i - r_j)
 * (the Coulomb term is Table 1's q_i q_j r_ij / (eps r^3) with the constant kc / D).
 * ---------------------------------------------------------------------- */
static int ljc_constant_impl(const double *pos, const double *q, const double *sigma,
                             const double *epsl, int64_t n, double kc, double D,
                             const int64_t *ilist, int64_t ni, const int64_t *eoff,
                             const int64_t *eidx, double *force, double *energy, int nthreads)
{
    if (n < 0 || ni < 0) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ni; ++k) {
        const int64_t i = row(ilist, k);
        nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, en = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || excluded(eoff, eidx, i, j)) continue;
            const double rx = pos[3 * i] - pos[3 * j];
            const double ry = pos[3 * i + 1] - pos[3 * j + 1];
            const double rz = pos[3 * i + 2] - pos[3 * j + 2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double r = sqrt(r2);
            const double sij = 0.5 * (sigma[i] + sigma[j]);
            const double eij = sqrt(epsl[i] * epsl[j]);
            const double sr2 = sij * sij / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double sr12 = sr6 * sr6;
            const double coul = kc * q[i] * q[j] / D;          /* u_C = coul / r */
            const double W = coul / (r2 * r) + 24.0 * eij / r2 * (2.0 * sr12 - sr6);
            nadd(&fx, W * rx);
            nadd(&fy, W * ry);
            nadd(&fz, W * rz);
            nadd(&en, coul / r + 4.0 * eij * (sr12 - sr6));
        }
        force[3 * k] = nval(&fx);
        force[3 * k + 1] = nval(&fy);
        force[3 * k + 2] = nval(&fz);
        if (energy) energy[k] = nval(&en);
    }
    return 0;
}

int oracle_ljc_constant(const double *pos, const double *q, const double *sigma,
                        const double *epsl, int64_t n, double kc, double D,
                        const int64_t *ilist, int64_t ni, double *force, double *energy,
                        int nthreads)
{
    return ljc_constant_impl(pos, q, sigma, epsl, n, kc, D, ilist, ni, NULL, NULL, force, energy,
                             nthreads);
}

/* ------------------------------------------------------------------------
 * LJ + Coulomb with a distance-dependent dielectric zeta(r) (Table 1 row
 * "LJC (sigmoidal)").  The printed zeta(r) = exp(alpha r^3 + beta r^2 + gamma
 * + delta) is read as exp(alpha r^3 + beta r^2 + gamma r + delta) (the
 * constants are not given; they are inputs here), and the law is read
 * potential-consistently:
 *   u_ij = kc q_i q_j / (zeta(r) r) + 4 e_ij [(s_ij/r)^12 - (s_ij/r)^6]
 *   F_i  = sum_{j != i} [ kc q_i q_j (1 + r zeta'(r)/zeta(r)) / (zeta(r) r^3)
 *                         + (24 e_ij / r^2) (2 (s_ij/r)^12 - (s_ij/r)^6) ] (r_i - r_j)
 * with zeta'/zeta = 3 alpha r^2 + 2 beta r + gamma.
 * ---------------------------------------------------------------------- */
static int ljc_sigmoidal_impl(const double *pos, const double *q, const double *sigma,
                              const double *epsl, int64_t n, double kc, const double *zc,
                              const int64_t *ilist, int64_t ni, const int64_t *eoff,
                              const int64_t *eidx, double *force, double *energy, int nthreads)
{
    if (n < 0 || ni < 0 || !zc) return -1;
    set_threads(nthreads);
    const double al = zc[0], be = zc[1], ga = zc[2], de = zc[3];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ni; ++k) {
        const int64_t i = row(ilist, k);
        nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, en = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || excluded(eoff, eidx, i, j)) continue;
            const double rx = pos[3 * i] - pos[3 * j];
            const double ry = pos[3 * i + 1] - pos[3 * j + 1];
            const double rz = pos[3 * i + 2] - pos[3 * j + 2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double r = sqrt(r2);
            const double zeta = exp(al * r * r * r + be * r * r + ga * r + de);
            const double dlog = 3.0 * al * r * r + 2.0 * be * r + ga;      /* zeta' / zeta */
            const double sij = 0.5 * (sigma[i] + sigma[j]);
            const double eij = sqrt(epsl[i] * epsl[j]);
            const double sr2 = sij * sij / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double sr12 = sr6 * sr6;
            const double coul = kc * q[i] * q[j];
            const double W = coul * (1.0 + r * dlog) / (zeta * r2 * r) +
                             24.0 * eij / r2 * (2.0 * sr12 - sr6);
            nadd(&fx, W * rx);
            nadd(&fy, W * ry);
            nadd(&fz, W * rz);
            nadd(&en, coul / (zeta * r) + 4.0 * eij * (sr12 - sr6));
        }
        force[3 * k] = nval(&fx);
        force[3 * k + 1] = nval(&fy);
        force[3 * k + 2] = nval(&fz);
        if (energy) energy[k] = nval(&en);
    }
    return 0;
}

int oracle_ljc_sigmoidal(const double *pos, const double *q, const double *sigma,
                         const double *epsl, int64_t n, double kc, const double *zc,
                         const int64_t *ilist, int64_t ni, double *force, double *energy,
                         int nthreads)
{
    return ljc_sigmoidal_impl(pos, q, sigma, epsl, n, kc, zc, ilist, ni, NULL, NULL, force, energy,
                              nthreads);
}

/* Any of the three LJC laws (kind 1 linear, 2 constant, 3 sigmoidal; c1 is D
 * for the first two, zc the sigmoidal coefficients) with exclusion lists
 * eoff [n+1], eidx [eoff[n]] (pair (i, j) skipped when j is in i's list). */
int oracle_ljc_excl(int kind, const double *pos, const double *q, const double *sigma,
                    const double *epsl, int64_t n, double kc, double D, const double *zc,
                    const int64_t *eoff, const int64_t *eidx, double *force, double *energy,
                    int nthreads)
{
    if (!eoff || !eidx) return -1;
    switch (kind) {
    case 1: return ljc_linear_impl(pos, q, sigma, epsl, n, kc, D, NULL, n, 0, n, eoff, eidx, force,
                                   energy, nthreads);
    case 2: return ljc_constant_impl(pos, q, sigma, epsl, n, kc, D, NULL, n, eoff, eidx, force,
                                     energy, nthreads);
    case 3: return ljc_sigmoidal_impl(pos, q, sigma, epsl, n, kc, zc, NULL, n, eoff, eidx, force,
                                      energy, nthreads);
    default: return -1;
    }
}

/* Scale of a row's pair-energy sum: S_i = sum_{j != i, not excluded} |u_ij| for
 * the LJC laws above (kind 1 linear, 2 constant, 3 sigmoidal), with the same
 * u_ij as the energy sums (plain loop; every term is non-negative).  A rounding
 * error of the sum U_i is bounded by a small multiple of the unit roundoff
 * times S_i, while U_i itself can be a near-cancelling sum of Coulomb and
 * Lennard-Jones terms; eoff / eidx as in oracle_ljc_excl, or NULL. */
int oracle_ljc_energy_abs(int kind, const double *pos, const double *q, const double *sigma,
                          const double *epsl, int64_t n, double kc, double D, const double *zc,
                          const int64_t *eoff, const int64_t *eidx, double *out, int nthreads)
{
    if (n < 0 || kind < 1 || kind > 3 || (kind == 3 && !zc)) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || excluded(eoff, eidx, i, j)) continue;
            const double rx = pos[3 * i] - pos[3 * j];
            const double ry = pos[3 * i + 1] - pos[3 * j + 1];
            const double rz = pos[3 * i + 2] - pos[3 * j + 2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double r = sqrt(r2);
            const double sij = 0.5 * (sigma[i] + sigma[j]);
            const double eij = sqrt(epsl[i] * epsl[j]);
            const double sr2 = sij * sij / r2;
            const double sr6 = sr2 * sr2 * sr2;
            double uc;
            if (kind == 1) uc = kc * q[i] * q[j] / (D * r2);
            else if (kind == 2) uc = kc * q[i] * q[j] / (D * r);
            else uc = kc * q[i] * q[j] / (exp(zc[0] * r * r * r + zc[1] * r * r + zc[2] * r + zc[3]) * r);
            acc += fabs(uc + 4.0 * eij * (sr6 * sr6 - sr6));
        }
        out[i] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Time-step cycle (Section 1: force evaluation, then the update step, then
 * repeat).  The paper names no integrator; the reading is kick-drift-kick
 * leapfrog (velocity Verlet) in FP64 with the acceleration carried:
 *   v += dt/2 a(x);  x += dt v;  a = a(x);  v += dt/2 a.
 * law 0 = gravity (params = mass [n]; a is the acceleration of Eq. 1);
 * law 1 = LJC(linear), law 2 = LJC(constant) (c0 = kc, c1 = D; params = q,
 * sigma, eps as three [n] arrays packed one after another, i.e.
 * params[0..n), params[n..2n), params[2n..3n)); a = F * inv_mass.
 * acc holds a(t) on entry and a(t + nsteps dt) on exit.  pot (or NULL)
 * receives phi (gravity) or U_i (LJC) at the final positions.
 * ---------------------------------------------------------------------- */
static int eval_accel(int law, const double *pos, const double *params, const double *inv_mass,
                      int64_t n, double c0, double c1, double *acc, double *pot, int nthreads)
{
    if (law == 0)
        return oracle_gravity(pos, params, n, c0, c1, NULL, n, 0, n, acc, pot, nthreads);
    if (law == 1 || law == 2) {
        int rc = law == 1 ? oracle_ljc_linear(pos, params, params + n, params + 2 * n, n, c0, c1, NULL,
                                              n, 0, n, acc, pot, nthreads)
                          : oracle_ljc_constant(pos, params, params + n, params + 2 * n, n, c0, c1,
                                                NULL, n, acc, pot, nthreads);
        if (rc) return rc;
        for (int64_t i = 0; i < n; ++i) {
            const double w = inv_mass ? inv_mass[i] : 1.0;
            acc[3 * i] *= w;
            acc[3 * i + 1] *= w;
            acc[3 * i + 2] *= w;
        }
        return 0;
    }
    return -1;
}

int oracle_leapfrog(int law, double *pos, double *vel, double *acc, const double *params,
                    const double *inv_mass, int64_t n, double c0, double c1, double dt,
                    int32_t nsteps, double *pot, int nthreads)
{
    if (n < 0 || nsteps < 0) return -1;
    for (int32_t s = 0; s < nsteps; ++s) {
        for (int64_t e = 0; e < 3 * n; ++e) {
            vel[e] += 0.5 * dt * acc[e];
            pos[e] += dt * vel[e];
        }
        const int last = (s == nsteps - 1);
        int rc = eval_accel(law, pos, params, inv_mass, n, c0, c1, acc, last ? pot : NULL, nthreads);
        if (rc) return rc;
        for (int64_t e = 0; e < 3 * n; ++e) vel[e] += 0.5 * dt * acc[e];
    }
    if (nsteps == 0 && pot) {
        double *tmp = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        if (!tmp) return -2;
        int rc = eval_accel(law, pos, params, inv_mass, n, c0, c1, tmp, pot, nthreads);
        free(tmp);
        return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Adjoint of the gravity acceleration with respect to positions (the
 * Hessian-vector product of the potential).  Not in the paper; it is the
 * derivative of Eq. 1 written out.  With d = r_j - r_k, s^2 = |d|^2 + eps^2
 * and K(d) v = v / s^3 - 3 (d.v) d / s^5 (the Jacobian of d / s^3):
 *   dL/dr_k = G sum_{j != k} K(d) (m_k g_j - m_j g_k),     g_i = dL/da_i.
 * out is [ni][3].
 * ---------------------------------------------------------------------- */
int oracle_gravity_adjoint(const double *pos, const double *mass, int64_t n, double G, double eps,
                           const double *g, const int64_t *ilist, int64_t ni, double *out,
                           int nthreads)
{
    if (n < 0 || ni < 0) return -1;
    set_threads(nthreads);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t kk = 0; kk < ni; ++kk) {
        const int64_t k = row(ilist, kk);
        nsum ox = {0, 0}, oy = {0, 0}, oz = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            const double dx = pos[3 * j] - pos[3 * k];
            const double dy = pos[3 * j + 1] - pos[3 * k + 1];
            const double dz = pos[3 * j + 2] - pos[3 * k + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double inv_s3 = 1.0 / (s2 * s);
            const double inv_s5 = inv_s3 / s2;
            const double vx = mass[k] * g[3 * j] - mass[j] * g[3 * k];
            const double vy = mass[k] * g[3 * j + 1] - mass[j] * g[3 * k + 1];
            const double vz = mass[k] * g[3 * j + 2] - mass[j] * g[3 * k + 2];
            const double dv = dx * vx + dy * vy + dz * vz;
            nadd(&ox, vx * inv_s3 - 3.0 * dv * dx * inv_s5);
            nadd(&oy, vy * inv_s3 - 3.0 * dv * dy * inv_s5);
            nadd(&oz, vz * inv_s3 - 3.0 * dv * dz * inv_s5);
        }
        out[3 * kk] = G * nval(&ox);
        out[3 * kk + 1] = G * nval(&oy);
        out[3 * kk + 2] = G * nval(&oz);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Adjoint of the LJC(linear) force (derivative of the Table 1 law as read
 * above; not in the paper).  Write F_i = sum_j w(r_ij) d_ij with
 * d_ij = r_j - r_i and
 *   w = -[ C / r^4 + 24 e (2 s^12 / r^14 - s^6 / r^8) ],   C = 2 kc q_i q_j / D.
 * Its Jacobian in d is M(d) = w I + (w'/r) d d^T with
 *   w'/r = 4 C / r^6 + 24 e (28 s^12 / r^16 - 8 s^6 / r^10).
 * For g_i = dL/dF_i:
 *   dL/dr_k = sum_{j != k} M(d_kj) (g_j - g_k)
 *   dL/dp_k = sum_{j != k} (dw_kj/dp_k) d_kj . (g_k - g_j)   for p in {q, sigma, eps}
 * with dw/dq_k = -2 kc q_j / (D r^4),
 *      dw/dsigma_k = 1/2 * dw/ds_kj = -(12 e / (s r^2)) (24 (s/r)^12 - 6 (s/r)^6),
 *      dw/deps_k = (de_kj/deps_k) (w_LJ / e_kj),  de_kj/deps_k = eps_j / (2 e_kj),
 *      w_LJ = -24 e (2 s^12 / r^14 - s^6 / r^8).
 * Outputs are per atom ([ni][3] and [ni]); any output may be NULL.
 * ---------------------------------------------------------------------- */
static int ljc_adjoint_impl(const double *pos, const double *q, const double *sigma,
                            const double *epsl, int64_t n, double kc, double D, const double *g,
                            const int64_t *ilist, int64_t ni, const int64_t *eoff,
                            const int64_t *eidx, double *grad_pos, double *grad_q,
                            double *grad_sigma, double *grad_eps, int nthreads)
{
    if (n < 0 || ni < 0) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t kk = 0; kk < ni; ++kk) {
        const int64_t k = row(ilist, kk);
        nsum px = {0, 0}, py = {0, 0}, pz = {0, 0}, gq = {0, 0}, gs = {0, 0}, ge = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k || excluded(eoff, eidx, k, j)) continue;
            const double dx = pos[3 * j] - pos[3 * k];
            const double dy = pos[3 * j + 1] - pos[3 * k + 1];
            const double dz = pos[3 * j + 2] - pos[3 * k + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double sij = 0.5 * (sigma[k] + sigma[j]);
            const double eij = sqrt(epsl[k] * epsl[j]);
            const double sr2 = sij * sij / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double sr12 = sr6 * sr6;
            const double C = 2.0 * kc * q[k] * q[j] / D;
            const double wlj = -24.0 * eij / r2 * (2.0 * sr12 - sr6);
            const double w = -C / (r2 * r2) + wlj;
            const double wpr = 4.0 * C / (r2 * r2 * r2) + 24.0 * eij / (r2 * r2) * (28.0 * sr12 - 8.0 * sr6);
            /* position adjoint: M(d) (g_j - g_k) */
            const double ux = g[3 * j] - g[3 * k];
            const double uy = g[3 * j + 1] - g[3 * k + 1];
            const double uz = g[3 * j + 2] - g[3 * k + 2];
            const double du = dx * ux + dy * uy + dz * uz;
            nadd(&px, w * ux + wpr * du * dx);
            nadd(&py, w * uy + wpr * du * dy);
            nadd(&pz, w * uz + wpr * du * dz);
            /* parameter adjoints: (dw/dp_k) d . (g_k - g_j) = -(dw/dp_k) du */
            const double dw_dq = -2.0 * kc * q[j] / (D * r2 * r2);
            const double dw_ds = -(12.0 * eij / (sij * r2)) * (24.0 * sr12 - 6.0 * sr6);
            /* w_LJ / e_kj is finite for every e_kj; e_kj = sqrt(eps_k eps_j) does not
             * depend on eps_k when eps_j = 0, and its derivative is infinite when
             * eps_k = 0 < eps_j (the square root's derivative at 0). */
            const double wlj_per_e = -24.0 / r2 * (2.0 * sr12 - sr6);
            const double de_de = (epsl[j] == 0.0) ? 0.0 : epsl[j] / (2.0 * eij);
            const double dw_de = de_de * wlj_per_e;
            nadd(&gq, -dw_dq * du);
            nadd(&gs, -dw_ds * du);
            nadd(&ge, -dw_de * du);
        }
        if (grad_pos) {
            grad_pos[3 * kk] = nval(&px);
            grad_pos[3 * kk + 1] = nval(&py);
            grad_pos[3 * kk + 2] = nval(&pz);
        }
        if (grad_q) grad_q[kk] = nval(&gq);
        if (grad_sigma) grad_sigma[kk] = nval(&gs);
        if (grad_eps) grad_eps[kk] = nval(&ge);
    }
    return 0;
}

int oracle_ljc_adjoint(const double *pos, const double *q, const double *sigma, const double *epsl,
                       int64_t n, double kc, double D, const double *g, const int64_t *ilist,
                       int64_t ni, double *grad_pos, double *grad_q, double *grad_sigma,
                       double *grad_eps, int nthreads)
{
    return ljc_adjoint_impl(pos, q, sigma, epsl, n, kc, D, g, ilist, ni, NULL, NULL, grad_pos,
                            grad_q, grad_sigma, grad_eps, nthreads);
}

/* The LJC(linear) adjoint with exclusion lists.  It is the derivative of the
 * excluded forward when the lists are symmetric (j in E(i) exactly when i is
 * in E(j)), which bonded topologies are. */
int oracle_ljc_adjoint_excl(const double *pos, const double *q, const double *sigma,
                            const double *epsl, int64_t n, double kc, double D, const double *g,
                            const int64_t *eoff, const int64_t *eidx, double *grad_pos,
                            double *grad_q, double *grad_sigma, double *grad_eps, int nthreads)
{
    if (!eoff || !eidx) return -1;
    return ljc_adjoint_impl(pos, q, sigma, epsl, n, kc, D, g, NULL, n, eoff, eidx, grad_pos, grad_q,
                            grad_sigma, grad_eps, nthreads);
}

/* ------------------------------------------------------------------------
 * Softened gravity with its time derivative, Table 1 row "Gravity (accel &
 * jerk)"; Section 2 names this kernel (GAJ) for integration schemes that use
 * the derivative of the force.  With d = r_j - r_i, w = v_j - v_i and
 * s^2 = |d|^2 + eps^2:
 *   a_i    = G sum_{j != i} m_j d / s^3
 *   jerk_i = G sum_{j != i} m_j [ w / s^3 - 3 (d.w) d / s^5 ]
 *   phi_i  = -G sum_{j != i} m_j / s
 * (jerk_i is d a_i / dt along the motion: the derivative of d / s^3 with
 * d' = w and s' = (d.w) / s).  acc and jerk are [ni][3], phi [ni] or NULL.
 * ---------------------------------------------------------------------- */
int oracle_gravity_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                        double G, double eps, const int64_t *ilist, int64_t ni, double *acc,
                        double *jerk, double *phi, int nthreads)
{
    if (n < 0 || ni < 0) return -1;
    set_threads(nthreads);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ni; ++k) {
        const int64_t i = row(ilist, k);
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, jx = {0, 0}, jy = {0, 0}, jz = {0, 0},
             ph = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * j] - pos[3 * i];
            const double dy = pos[3 * j + 1] - pos[3 * i + 1];
            const double dz = pos[3 * j + 2] - pos[3 * i + 2];
            const double wx = vel[3 * j] - vel[3 * i];
            const double wy = vel[3 * j + 1] - vel[3 * i + 1];
            const double wz = vel[3 * j + 2] - vel[3 * i + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double inv_s3 = 1.0 / (s2 * s);
            const double inv_s5 = inv_s3 / s2;
            const double dw = dx * wx + dy * wy + dz * wz;
            nadd(&ax, mass[j] * dx * inv_s3);
            nadd(&ay, mass[j] * dy * inv_s3);
            nadd(&az, mass[j] * dz * inv_s3);
            nadd(&jx, mass[j] * (wx * inv_s3 - 3.0 * dw * dx * inv_s5));
            nadd(&jy, mass[j] * (wy * inv_s3 - 3.0 * dw * dy * inv_s5));
            nadd(&jz, mass[j] * (wz * inv_s3 - 3.0 * dw * dz * inv_s5));
            nadd(&ph, mass[j] / s);
        }
        acc[3 * k] = G * nval(&ax);
        acc[3 * k + 1] = G * nval(&ay);
        acc[3 * k + 2] = G * nval(&az);
        jerk[3 * k] = G * nval(&jx);
        jerk[3 * k + 1] = G * nval(&jy);
        jerk[3 * k + 2] = G * nval(&jz);
        if (phi) phi[k] = -G * nval(&ph);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Fourth-order Hermite predictor-corrector (Makino & Aarseth 1992), the
 * integrator that the acceleration-and-jerk kernel serves.  The paper names
 * no integrator; this scheme is the reading.  For one particle advanced by
 * h from (x0, v0, a0, j0), with a1, j1 evaluated at the predicted state:
 *   predict  xp = x0 + v0 h + a0 h^2/2 + j0 h^3/6,   vp = v0 + a0 h + j0 h^2/2
 *   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2      (second derivative of a at t0)
 *   a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3        (third derivative)
 *   correct  x1 = xp + a2 h^4/24 + a3 h^5/120,  v1 = vp + a2 h^3/6 + a3 h^4/24
 * ---------------------------------------------------------------------- */
static void hermite_predict(const double *x, const double *v, const double *a, const double *j,
                            double h, double *xp, double *vp)
{
    for (int c = 0; c < 3; ++c) {
        xp[c] = x[c] + h * (v[c] + h * (a[c] / 2.0 + h * j[c] / 6.0));
        vp[c] = v[c] + h * (a[c] + h * j[c] / 2.0);
    }
}

/* corrector; writes x1, v1 and the derivatives a2 (moved to t1: a2 + a3 h)
 * and a3 used by the time-step criterion */
static void hermite_correct(const double *xp, const double *vp, const double *a0, const double *j0,
                            const double *a1, const double *j1, double h, double *x1, double *v1,
                            double *a2_t1, double *a3_out)
{
    for (int c = 0; c < 3; ++c) {
        const double a2 = (-6.0 * (a0[c] - a1[c]) - h * (4.0 * j0[c] + 2.0 * j1[c])) / (h * h);
        const double a3 = (12.0 * (a0[c] - a1[c]) + 6.0 * h * (j0[c] + j1[c])) / (h * h * h);
        x1[c] = xp[c] + h * h * h * h * (a2 / 24.0 + h * a3 / 120.0);
        v1[c] = vp[c] + h * h * h * (a2 / 6.0 + h * a3 / 24.0);
        if (a2_t1) a2_t1[c] = a2 + a3 * h;
        if (a3_out) a3_out[c] = a3;
    }
}

/* Shared time step: nsteps steps of dt for all particles.  acc and jerk hold
 * a and jerk at the current state on entry and are replaced by the values at
 * the last predicted state on exit (the PEC scheme). */
int oracle_hermite(double *pos, double *vel, double *acc, double *jerk, const double *mass,
                   int64_t n, double G, double eps, double dt, int32_t nsteps, int nthreads)
{
    if (n < 0 || nsteps < 0 || !(dt > 0.0)) return -1;
    double *xp = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *vp = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *a1 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *j1 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!xp || !vp || !a1 || !j1) {
        free(xp), free(vp), free(a1), free(j1);
        return -2;
    }
    int rc = 0;
    for (int32_t s = 0; s < nsteps && rc == 0; ++s) {
        for (int64_t i = 0; i < n; ++i)
            hermite_predict(pos + 3 * i, vel + 3 * i, acc + 3 * i, jerk + 3 * i, dt, xp + 3 * i,
                            vp + 3 * i);
        rc = oracle_gravity_jerk(xp, vp, mass, n, G, eps, NULL, n, a1, j1, NULL, nthreads);
        for (int64_t i = 0; rc == 0 && i < n; ++i) {
            hermite_correct(xp + 3 * i, vp + 3 * i, acc + 3 * i, jerk + 3 * i, a1 + 3 * i,
                            j1 + 3 * i, dt, pos + 3 * i, vel + 3 * i, NULL, NULL);
            for (int c = 0; c < 3; ++c) {
                acc[3 * i + c] = a1[3 * i + c];
                jerk[3 * i + c] = j1[3 * i + c];
            }
        }
    }
    free(xp), free(vp), free(a1), free(j1);
    return rc;
}

/* ------------------------------------------------------------------------
 * Block (hierarchical) individual time steps for the Hermite scheme: the
 * setting in which Section 3.4 needs forces on a subset of the particles at
 * a time.  Every particle i carries its own time t_i and step dt_i, a power
 * of two fraction of dt_max (itself a power of two).  One block step:
 *   t = min_i (t_i + dt_i);  the active set is { i : t_i + dt_i == t }
 *   every particle is predicted to t from its own t_j (the predictor above)
 *   a and jerk of each active i are evaluated against all predicted j
 *   each active i is corrected with h = dt_i and gets t_i = t and a new step
 * New step (Aarseth's criterion, with a2' = a2 + a3 h the second derivative
 * at t):  dt* = sqrt( eta (|a1| |a2'| + |j1|^2) / (|j1| |a3| + |a2'|^2) ),
 * quantised to the largest dt_max / 2^k <= dt* that is at most twice the old
 * step and divides t.  Initial steps: dt* = eta_s |a| / |j|, quantised the
 * same way at t = 0.
 * ---------------------------------------------------------------------- */
static double norm3(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static double quantise_step(double dts, double dt_max, double t, double dt_old)
{
    double h = dt_max;
    int k = 0;
    while (h > dts && k < 60) {
        h *= 0.5;
        ++k;
    }
    if (dt_old > 0.0 && h > 2.0 * dt_old) h = 2.0 * dt_old;
    while (fmod(t, h) != 0.0 && k < 60) {
        h *= 0.5;
        ++k;
    }
    return h;
}

/* Initial step estimate eta_s |a| / |j| (dt_max when the jerk vanishes). */
static double initial_step(const double *a, const double *j, double eta_s, double dt_max)
{
    const double aj = norm3(j);
    return aj > 0.0 ? eta_s * norm3(a) / aj : dt_max;
}

/* Aarseth's criterion from a, its first three time derivatives at the end of
 * the step and eta:  sqrt( eta (|a| |a2| + |j|^2) / (|j| |a3| + |a2|^2) )
 * (dt_max when the denominator vanishes). */
static double aarseth_step(const double *a, const double *j, const double *a2, const double *a3,
                           double eta, double dt_max)
{
    const double na1 = norm3(a), nj1 = norm3(j);
    const double na2 = norm3(a2), na3 = norm3(a3);
    const double den = nj1 * na3 + na2 * na2;
    return den > 0.0 ? sqrt(eta * (na1 * na2 + nj1 * nj1) / den) : dt_max;
}

/* The three pieces of the step choice, exported so that tests can pin them on
 * hand-computed values; the block-step integrator below uses the same static
 * functions. */
double oracle_initial_step(const double *a, const double *j, double eta_s, double dt_max)
{
    return initial_step(a, j, eta_s, dt_max);
}

double oracle_aarseth_step(const double *a, const double *j, const double *a2, const double *a3,
                           double eta, double dt_max)
{
    return aarseth_step(a, j, a2, a3, eta, dt_max);
}

double oracle_quantise_step(double dts, double dt_max, double t, double dt_old)
{
    return quantise_step(dts, dt_max, t, dt_old);
}

int oracle_hermite_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                              double dt_max, double *t_i, double *dt_i)
{
    if (n < 0 || !(dt_max > 0.0)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const double dts = initial_step(acc + 3 * i, jerk + 3 * i, eta_s, dt_max);
        t_i[i] = 0.0;
        dt_i[i] = quantise_step(dts, dt_max, 0.0, 0.0);
    }
    return 0;
}

/* nblocks block steps.  pos, vel, acc, jerk, t_i, dt_i are per particle and
 * updated for the active particles of each block step; active[b] (or NULL)
 * receives the size of the active set of block step b and t_now the time
 * reached. */
int oracle_hermite_block(double *pos, double *vel, double *acc, double *jerk, double *t_i,
                         double *dt_i, const double *mass, int64_t n, double G, double eps,
                         double eta, double dt_max, int32_t nblocks, int64_t *active,
                         double *t_now, int nthreads)
{
    if (n <= 0 || nblocks < 0 || !(dt_max > 0.0)) return -1;
    const size_t sz = sizeof(double) * 3 * (size_t)n;
    double *xp = (double *)malloc(sz), *vp = (double *)malloc(sz);
    double *a1 = (double *)malloc(sz), *j1 = (double *)malloc(sz);
    int64_t *il = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!xp || !vp || !a1 || !j1 || !il) {
        free(xp), free(vp), free(a1), free(j1), free(il);
        return -2;
    }
    int rc = 0;
    double t = 0.0;
    for (int32_t b = 0; b < nblocks && rc == 0; ++b) {
        t = t_i[0] + dt_i[0];
        for (int64_t i = 1; i < n; ++i)
            if (t_i[i] + dt_i[i] < t) t = t_i[i] + dt_i[i];
        int64_t na = 0;
        for (int64_t i = 0; i < n; ++i)
            if (t_i[i] + dt_i[i] == t) il[na++] = i;
        if (active) active[b] = na;
        for (int64_t i = 0; i < n; ++i)
            hermite_predict(pos + 3 * i, vel + 3 * i, acc + 3 * i, jerk + 3 * i, t - t_i[i],
                            xp + 3 * i, vp + 3 * i);
        rc = oracle_gravity_jerk(xp, vp, mass, n, G, eps, il, na, a1, j1, NULL, nthreads);
        for (int64_t k = 0; rc == 0 && k < na; ++k) {
            const int64_t i = il[k];
            const double h = dt_i[i];
            double a2[3], a3[3];
            hermite_correct(xp + 3 * i, vp + 3 * i, acc + 3 * i, jerk + 3 * i, a1 + 3 * k,
                            j1 + 3 * k, h, pos + 3 * i, vel + 3 * i, a2, a3);
            for (int c = 0; c < 3; ++c) {
                acc[3 * i + c] = a1[3 * k + c];
                jerk[3 * i + c] = j1[3 * k + c];
            }
            const double dts = aarseth_step(a1 + 3 * k, j1 + 3 * k, a2, a3, eta, dt_max);
            t_i[i] = t;
            dt_i[i] = quantise_step(dts, dt_max, t, h);
        }
    }
    if (t_now) *t_now = t;
    free(xp), free(vp), free(a1), free(j1), free(il);
    return rc;
}
