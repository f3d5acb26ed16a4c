/*
 * Driver for the sanitizer build of the FP64 oracle (test infrastructure).
 *
 * Built together with oracle/oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it calls every exported oracle function on
 * small inputs with ragged shapes: no particles, one particle, a row subset,
 * a partial j range, empty and uneven exclusion lists, NULL optional
 * outputs.  Every output buffer is allocated at exactly the size the
 * function documents, so a write past its end is reported.  It also checks
 * that the results do not depend on the OpenMP thread count (the oracle's
 * j order is fixed) and that invalid sizes are refused with a nonzero code.
 * Prints "ok" and exits 0 when everything passed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_threads(int nthreads);
int oracle_gravity(const double *pos, const double *mass, int64_t n, double G, double eps,
                   const int64_t *ilist, int64_t ni, int64_t j0, int64_t j1, double *acc,
                   double *phi, int nthreads);
int oracle_ljc_linear(const double *pos, const double *q, const double *sigma, const double *epsl,
                      int64_t n, double kc, double D, const int64_t *ilist, int64_t ni, int64_t j0,
                      int64_t j1, double *force, double *energy, int nthreads);
int oracle_ljc_constant(const double *pos, const double *q, const double *sigma,
                        const double *epsl, int64_t n, double kc, double D, const int64_t *ilist,
                        int64_t ni, double *force, double *energy, int nthreads);
int oracle_ljc_sigmoidal(const double *pos, const double *q, const double *sigma,
                         const double *epsl, int64_t n, double kc, const double *zc,
                         const int64_t *ilist, int64_t ni, double *force, double *energy,
                         int nthreads);
int oracle_ljc_excl(int kind, const double *pos, const double *q, const double *sigma,
                    const double *epsl, int64_t n, double kc, double D, const double *zc,
                    const int64_t *eoff, const int64_t *eidx, double *force, double *energy,
                    int nthreads);
int oracle_leapfrog(int law, double *pos, double *vel, double *acc, const double *params,
                    const double *inv_mass, int64_t n, double c0, double c1, double dt,
                    int32_t nsteps, double *pot, int nthreads);
int oracle_gravity_adjoint(const double *pos, const double *mass, int64_t n, double G, double eps,
                           const double *g, const int64_t *ilist, int64_t ni, double *out,
                           int nthreads);
int oracle_ljc_adjoint(const double *pos, const double *q, const double *sigma, const double *epsl,
                       int64_t n, double kc, double D, const double *g, const int64_t *ilist,
                       int64_t ni, double *grad_pos, double *grad_q, double *grad_sigma,
                       double *grad_eps, int nthreads);
int oracle_ljc_adjoint_excl(const double *pos, const double *q, const double *sigma,
                            const double *epsl, int64_t n, double kc, double D, const double *g,
                            const int64_t *eoff, const int64_t *eidx, double *grad_pos,
                            double *grad_q, double *grad_sigma, double *grad_eps, int nthreads);
int oracle_gravity_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                        double G, double eps, const int64_t *ilist, int64_t ni, double *acc,
                        double *jerk, double *phi, int nthreads);
int oracle_hermite(double *pos, double *vel, double *acc, double *jerk, const double *mass,
                   int64_t n, double G, double eps, double dt, int32_t nsteps, int nthreads);
int oracle_hermite_block_init(const double *acc, const double *jerk, int64_t n, double eta_s,
                              double dt_max, double *t_i, double *dt_i);
int oracle_hermite_block(double *pos, double *vel, double *acc, double *jerk, double *t_i,
                         double *dt_i, const double *mass, int64_t n, double G, double eps,
                         double eta, double dt_max, int32_t nblocks, int64_t *active,
                         double *t_now, int nthreads);

static int failures = 0;

#define EXPECT(cond)                                                                 \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

/* xorshift64* values in [lo, hi) */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(double lo, double hi)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    const uint64_t r = rng_state * 0x2545f4914f6cdd1dull;
    return lo + (hi - lo) * (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

static double *dalloc(int64_t count)
{
    /* exact size; a zero count still yields a distinct, unreadable block */
    double *p = (double *)malloc(sizeof(double) * (size_t)(count > 0 ? count : 1));
    if (!p) abort();
    for (int64_t k = 0; k < count; ++k) p[k] = uniform(-1.0, 1.0);
    return p;
}

static int64_t *ialloc(int64_t count)
{
    int64_t *p = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    if (!p) abort();
    return p;
}

/* positions on a jittered lattice of spacing 1.2, so no two particles are
 * closer than about 0.6 and the LJC terms stay finite */
static double *lattice(int64_t n)
{
    double *p = dalloc(3 * n);
    int64_t side = 1;
    while (side * side * side < n) ++side;
    for (int64_t i = 0; i < n; ++i) {
        p[3 * i] = 1.2 * (double)(i % side) + uniform(-0.2, 0.2);
        p[3 * i + 1] = 1.2 * (double)((i / side) % side) + uniform(-0.2, 0.2);
        p[3 * i + 2] = 1.2 * (double)(i / (side * side)) + uniform(-0.2, 0.2);
    }
    return p;
}

static double *positive(int64_t n, double lo, double hi)
{
    double *p = dalloc(n);
    for (int64_t i = 0; i < n; ++i) p[i] = uniform(lo, hi);
    return p;
}

/* symmetric exclusion lists: i excludes i+1 and i+2 when i % 5 == 0 (and
 * the reverse entries), every other particle keeps an empty or short list */
static void exclusions(int64_t n, int64_t **eoff_out, int64_t **eidx_out)
{
    int64_t *cnt = ialloc(n), *eoff = ialloc(n + 1);
    for (int64_t i = 0; i < n; ++i) cnt[i] = 0;
    for (int64_t i = 0; i < n; i += 5)
        for (int64_t d = 1; d <= 2 && i + d < n; ++d) ++cnt[i], ++cnt[i + d];
    eoff[0] = 0;
    for (int64_t i = 0; i < n; ++i) eoff[i + 1] = eoff[i] + cnt[i];
    int64_t *eidx = ialloc(eoff[n]);
    for (int64_t i = 0; i < n; ++i) cnt[i] = eoff[i];
    for (int64_t i = 0; i < n; i += 5)
        for (int64_t d = 1; d <= 2 && i + d < n; ++d) {
            eidx[cnt[i]++] = i + d;
            eidx[cnt[i + d]++] = i;
        }
    free(cnt);
    *eoff_out = eoff;
    *eidx_out = eidx;
}

static int all_finite(const double *p, int64_t count)
{
    for (int64_t k = 0; k < count; ++k)
        if (!isfinite(p[k])) return 0;
    return 1;
}

static void run_forward(int64_t n)
{
    double *pos = lattice(n), *mass = positive(n, 0.5, 1.5);
    double *q = dalloc(n), *sg = positive(n, 0.3, 0.5), *ep = positive(n, 0.1, 0.4);
    const double zc[4] = {-0.01, 0.02, 0.3, -0.1};
    const int64_t ni = n > 3 ? n / 3 : n;
    int64_t *il = ialloc(ni);
    for (int64_t k = 0; k < ni; ++k) il[k] = (k * 7) % (n > 0 ? n : 1);

    double *acc = dalloc(3 * n), *phi = dalloc(n), *acc1 = dalloc(3 * n), *phi1 = dalloc(n);
    EXPECT(oracle_gravity(pos, mass, n, 1.0, 0.05, NULL, n, 0, n, acc, phi, 3) == 0);
    EXPECT(oracle_gravity(pos, mass, n, 1.0, 0.05, NULL, n, 0, n, acc1, phi1, 1) == 0);
    EXPECT(memcmp(acc, acc1, sizeof(double) * 3 * (size_t)n) == 0);
    EXPECT(memcmp(phi, phi1, sizeof(double) * (size_t)n) == 0);
    EXPECT(all_finite(acc, 3 * n) && all_finite(phi, n));
    free(acc1), free(phi1);

    double *accs = dalloc(3 * ni), *phis = dalloc(ni);
    EXPECT(oracle_gravity(pos, mass, n, 1.0, 0.05, il, ni, n / 4, n - n / 5, accs, phis, 2) == 0);
    EXPECT(oracle_gravity(pos, mass, n, 1.0, 0.0, il, ni, 0, n, accs, NULL, 2) == 0);

    double *f = dalloc(3 * ni), *e = dalloc(ni);
    EXPECT(oracle_ljc_linear(pos, q, sg, ep, n, 1.0, 4.0, il, ni, n > 0, n, f, e, 2) == 0);
    EXPECT(oracle_ljc_linear(pos, q, sg, ep, n, 1.0, 4.0, il, ni, 0, n, f, NULL, 2) == 0);
    EXPECT(oracle_ljc_constant(pos, q, sg, ep, n, 1.0, 4.0, il, ni, f, e, 2) == 0);
    EXPECT(oracle_ljc_sigmoidal(pos, q, sg, ep, n, 1.0, zc, il, ni, f, e, 2) == 0);
    EXPECT(oracle_ljc_sigmoidal(pos, q, sg, ep, n, 1.0, NULL, il, ni, f, e, 2) != 0);
    EXPECT(all_finite(f, 3 * ni) && all_finite(e, ni));

    int64_t *eoff, *eidx;
    exclusions(n, &eoff, &eidx);
    double *fn = dalloc(3 * n), *en = dalloc(n);
    for (int kind = 1; kind <= 3; ++kind)
        EXPECT(oracle_ljc_excl(kind, pos, q, sg, ep, n, 1.0, 4.0, zc, eoff, eidx, fn, en, 2) == 0);
    EXPECT(oracle_ljc_excl(4, pos, q, sg, ep, n, 1.0, 4.0, zc, eoff, eidx, fn, en, 2) != 0);
    EXPECT(oracle_ljc_excl(1, pos, q, sg, ep, n, 1.0, 4.0, zc, NULL, eidx, fn, en, 2) != 0);

    double *g = dalloc(3 * n), *gp = dalloc(3 * ni), *gq = dalloc(ni), *gs = dalloc(ni),
           *ge = dalloc(ni);
    EXPECT(oracle_gravity_adjoint(pos, mass, n, 1.0, 0.05, g, il, ni, gp, 2) == 0);
    EXPECT(oracle_ljc_adjoint(pos, q, sg, ep, n, 1.0, 4.0, g, il, ni, gp, gq, gs, ge, 2) == 0);
    EXPECT(oracle_ljc_adjoint(pos, q, sg, ep, n, 1.0, 4.0, g, il, ni, NULL, NULL, gs, NULL, 2) == 0);
    double *gpn = dalloc(3 * n), *gqn = dalloc(n), *gsn = dalloc(n), *gen = dalloc(n);
    EXPECT(oracle_ljc_adjoint_excl(pos, q, sg, ep, n, 1.0, 4.0, g, eoff, eidx, gpn, gqn, gsn, gen,
                                   2) == 0);
    EXPECT(all_finite(gpn, 3 * n) && all_finite(gen, n));

    double *vel = dalloc(3 * n), *jk = dalloc(3 * ni);
    EXPECT(oracle_gravity_jerk(pos, vel, mass, n, 1.0, 0.05, il, ni, accs, jk, phis, 2) == 0);
    EXPECT(oracle_gravity_jerk(pos, vel, mass, n, 1.0, 0.05, NULL, 0, accs, jk, NULL, 2) == 0);

    free(pos), free(mass), free(q), free(sg), free(ep), free(il), free(acc), free(phi);
    free(accs), free(phis), free(f), free(e), free(eoff), free(eidx), free(fn), free(en);
    free(g), free(gp), free(gq), free(gs), free(ge), free(gpn), free(gqn), free(gsn), free(gen);
    free(vel), free(jk);
}

static void run_integrators(int64_t n)
{
    double *pos = lattice(n), *vel = dalloc(3 * n), *acc = dalloc(3 * n), *pot = dalloc(n);
    double *mass = positive(n, 0.5, 1.5), *im = positive(n, 0.5, 2.0);
    double *par = dalloc(3 * n); /* q | sigma | eps blocks */
    for (int64_t i = 0; i < n; ++i) {
        par[n + i] = uniform(0.3, 0.5);
        par[2 * n + i] = uniform(0.1, 0.4);
    }
    EXPECT(oracle_gravity(pos, mass, n, 1.0, 0.05, NULL, n, 0, n, acc, NULL, 2) == 0);
    EXPECT(oracle_leapfrog(0, pos, vel, acc, mass, NULL, n, 1.0, 0.05, 1e-3, 3, pot, 2) == 0);
    EXPECT(oracle_leapfrog(1, pos, vel, acc, par, im, n, 1.0, 4.0, 1e-4, 2, pot, 2) == 0);
    EXPECT(oracle_leapfrog(2, pos, vel, acc, par, NULL, n, 1.0, 4.0, 1e-4, 2, NULL, 2) == 0);
    EXPECT(oracle_leapfrog(5, pos, vel, acc, par, NULL, n, 1.0, 4.0, 1e-4, 1, NULL, 2) != 0);
    EXPECT(all_finite(pos, 3 * n) && all_finite(vel, 3 * n));

    double *jk = dalloc(3 * n);
    EXPECT(oracle_gravity_jerk(pos, vel, mass, n, 1.0, 0.05, NULL, n, acc, jk, NULL, 2) == 0);
    EXPECT(oracle_hermite(pos, vel, acc, jk, mass, n, 1.0, 0.05, 1e-3, 2, 2) == 0);
    EXPECT(oracle_hermite(pos, vel, acc, jk, mass, n, 1.0, 0.05, 0.0, 2, 2) != 0);

    double *ti = dalloc(n), *dti = dalloc(n), t_now = -1.0;
    const int32_t nb = 6;
    int64_t *active = ialloc(nb);
    EXPECT(oracle_hermite_block_init(acc, jk, n, 0.01, 1.0 / 64.0, ti, dti) == 0);
    if (n > 0) {
        EXPECT(oracle_hermite_block(pos, vel, acc, jk, ti, dti, mass, n, 1.0, 0.05, 0.02,
                                    1.0 / 64.0, nb, active, &t_now, 2) == 0);
        EXPECT(t_now > 0.0 && t_now <= nb / 64.0);
        for (int32_t b = 0; b < nb; ++b) EXPECT(active[b] >= 1 && active[b] <= n);
    } else {
        EXPECT(oracle_hermite_block(pos, vel, acc, jk, ti, dti, mass, n, 1.0, 0.05, 0.02,
                                    1.0 / 64.0, nb, active, &t_now, 2) != 0);
    }
    EXPECT(all_finite(pos, 3 * n) && all_finite(vel, 3 * n));

    free(pos), free(vel), free(acc), free(pot), free(mass), free(im), free(par), free(jk);
    free(ti), free(dti), free(active);
}

int main(void)
{
    const int64_t sizes[] = {0, 1, 2, 37, 130};
    for (size_t s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s) {
        run_forward(sizes[s]);
        run_integrators(sizes[s]);
    }
    /* negative sizes are refused before any access */
    double dummy[3] = {0, 0, 0};
    EXPECT(oracle_gravity(dummy, dummy, -1, 1.0, 0.0, NULL, 0, 0, 0, dummy, NULL, 1) != 0);
    EXPECT(oracle_leapfrog(0, dummy, dummy, dummy, dummy, NULL, -1, 1.0, 0.0, 1e-3, 1, NULL, 1) != 0);
    EXPECT(oracle_gravity_jerk(dummy, dummy, dummy, 1, 1.0, 0.0, NULL, -1, dummy, dummy, NULL, 1) != 0);
    oracle_threads(0);
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
