/*
 * c_abi_driver.c -- drives libhfgpe through include/hfgpe.h alone: plain C,
 * HIP runtime calls for device memory, no Python and no torch.  Each case
 * checks the library against a closed form of the linear problem
 * (sigma = 0, eps = 0), where the exact rule of Lemma 2 propagates the
 * harmonic oscillator exactly, or against a conserved quantity:
 *
 *   1. coherent state, 1-D, mu = omega = 1, x0 = 1: after time T the packet
 *      is the ground state moved to x0 cos T with momentum -x0 sin T and
 *      phase x0^2 sin(2T)/4 - T/2 (c128);
 *   2. 2-D anisotropic ground state: stationary, phase exp(-i T (wx + wy)/2)
 *      (c128);
 *   3. ragged batch (N = 64, 256, 1024, with sigma != 0) in c64: the
 *      splitting conserves each instance's norm; hfgpe_norm against the
 *      initial norm;
 *   4. error paths: a non-power-of-two grid, a null state, a null plan.
 *
 * Prints one line per case and exits 0 when every check holds.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hfgpe.h"

static const double kPi = 3.14159265358979323846;
static int failures = 0;

#define CHECK(cond, ...)                               \
    do {                                               \
        if (!(cond)) {                                 \
            printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            printf(__VA_ARGS__);                       \
            printf("\n");                              \
            ++failures;                                \
        }                                              \
    } while (0)

static void params_linear(hfgpe_params *p, double mu, const double *w, int nd)
{
    memset(p, 0, sizeof(*p));
    p->mu = mu;
    for (int j = 0; j < 3; ++j) {
        p->omega[j].v0 = (j < nd) ? w[j] : 1.0;
        p->omega[j].kind = HFGPE_TF_SIN;
        p->v[j].c0 = 1.0;
    }
}

static void grid_1d(hfgpe_grid *g, int n, double lo, double hi)
{
    memset(g, 0, sizeof(*g));
    g->ndim = 1;
    g->n[0] = n;
    g->n[1] = g->n[2] = 1;
    g->lo[0] = lo;
    g->hi[0] = hi;
    g->hi[1] = g->hi[2] = 1.0;
}

static int scheme_of(const char *name, hfgpe_ho_rule rule, hfgpe_scheme *s, double *a, double *b)
{
    int m = 0;
    int rc = hfgpe_scheme_preset(name, &m, a, b);
    if (rc != HFGPE_OK) return rc;
    s->m = m;
    s->a = a;
    s->b = b;
    s->ho_rule = rule;
    s->ho_substeps = 0;
    return HFGPE_OK;
}

/* relative L2 distance of two interleaved complex arrays */
static double rel_l2(const double *u, const double *v, long n)
{
    double num = 0.0, den = 0.0;
    for (long i = 0; i < 2 * n; ++i) {
        num += (u[i] - v[i]) * (u[i] - v[i]);
        den += v[i] * v[i];
    }
    return sqrt(num / den);
}

static int case_coherent(void)
{
    const int n = 256;
    const double lo = -10.0, hi = 10.0, x0 = 1.0, dt = 0.01;
    const long nsteps = 1000;
    hfgpe_grid g;
    hfgpe_params p;
    double w[1] = {1.0}, a[16], b[17];
    hfgpe_scheme s;
    grid_1d(&g, n, lo, hi);
    params_linear(&p, 1.0, w, 1);
    CHECK(scheme_of("leapfrog", HFGPE_HO_EXACT_CONST, &s, a, b) == HFGPE_OK, "leapfrog preset");
    hfgpe_plan *plan = NULL;
    int rc = hfgpe_plan_create(&plan, 1, &g, &p, &s, HFGPE_C128, dt, NULL, NULL);
    CHECK(rc == HFGPE_OK, "plan_create: %s", hfgpe_status_string(rc));
    if (rc != HFGPE_OK) return 1;
    int64_t off[2];
    CHECK(hfgpe_instance_offsets(plan, off) == HFGPE_OK && off[0] == 0 && off[1] == n, "offsets");

    double *h = (double *)malloc(sizeof(double) * 2 * n);
    double *ex = (double *)malloc(sizeof(double) * 2 * n);
    const double dx = (hi - lo) / n, T = dt * (double)nsteps;
    const double c = pow(kPi, -0.25);
    for (int i = 0; i < n; ++i) {
        double x = lo + i * dx;
        h[2 * i] = c * exp(-(x - x0) * (x - x0) / 2.0);
        h[2 * i + 1] = 0.0;
        double y = x - x0 * cos(T);
        double amp = c * exp(-y * y / 2.0);
        double ph = -x * x0 * sin(T) + x0 * x0 * sin(2.0 * T) / 4.0 - T / 2.0;
        ex[2 * i] = amp * cos(ph);
        ex[2 * i + 1] = amp * sin(ph);
    }
    void *d = NULL;
    CHECK(hipMalloc(&d, sizeof(double) * 2 * n) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(d, h, sizeof(double) * 2 * n, hipMemcpyHostToDevice) == hipSuccess, "copy in");
    rc = hfgpe_evolve(plan, d, 0.0, nsteps);
    CHECK(rc == HFGPE_OK, "evolve: %s", hfgpe_status_string(rc));
    double nrm = 0.0;
    CHECK(hfgpe_norm(plan, d, &nrm) == HFGPE_OK, "norm");
    CHECK(hipMemcpy(h, d, sizeof(double) * 2 * n, hipMemcpyDeviceToHost) == hipSuccess, "copy out");
    CHECK(hfgpe_device_status(plan) == HFGPE_OK, "device status");
    double e = rel_l2(h, ex, n);
    printf("case 1 coherent state 1-D c128, %ld steps: rel L2 vs closed form %.3e, norm %.15f\n", nsteps, e, nrm);
    CHECK(e < 1e-12, "coherent state off the closed form: %.3e", e);
    CHECK(fabs(nrm - 1.0) < 1e-12, "norm %.17g", nrm);
    hipFree(d);
    free(h);
    free(ex);
    hfgpe_plan_destroy(plan);
    return 0;
}

static int case_ground_2d(void)
{
    const int n = 64;
    const double L = 8.0, dt = 0.05;
    const long nsteps = 40;
    const double w[2] = {1.0, 1.7};
    hfgpe_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = 2;
    g.n[0] = g.n[1] = n;
    g.n[2] = 1;
    g.lo[0] = g.lo[1] = -L;
    g.hi[0] = g.hi[1] = L;
    g.hi[2] = 1.0;
    hfgpe_params p;
    params_linear(&p, 1.0, w, 2);
    double a[16], b[17];
    hfgpe_scheme s;
    CHECK(scheme_of("ni5_84", HFGPE_HO_EXACT_CONST, &s, a, b) == HFGPE_OK, "ni5_84 preset");
    hfgpe_plan *plan = NULL;
    int rc = hfgpe_plan_create(&plan, 1, &g, &p, &s, HFGPE_C128, dt, NULL, NULL);
    CHECK(rc == HFGPE_OK, "plan_create 2-D: %s", hfgpe_status_string(rc));
    if (rc != HFGPE_OK) return 1;
    const long np = (long)n * n;
    double *h = (double *)malloc(sizeof(double) * 2 * np);
    double *ex = (double *)malloc(sizeof(double) * 2 * np);
    const double dx = 2.0 * L / n, T = dt * (double)nsteps;
    const double E = 0.5 * (w[0] + w[1]);
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix < n; ++ix) {
            double x = -L + ix * dx, y = -L + iy * dx;
            double v = pow(w[0] * w[1], 0.25) / sqrt(kPi) * exp(-(w[0] * x * x + w[1] * y * y) / 2.0);
            long k = (long)iy * n + ix;  /* x fastest */
            h[2 * k] = v;
            h[2 * k + 1] = 0.0;
            ex[2 * k] = v * cos(E * T);
            ex[2 * k + 1] = -v * sin(E * T);
        }
    void *d = NULL;
    CHECK(hipMalloc(&d, sizeof(double) * 2 * np) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(d, h, sizeof(double) * 2 * np, hipMemcpyHostToDevice) == hipSuccess, "copy in");
    rc = hfgpe_evolve(plan, d, 0.0, nsteps);
    CHECK(rc == HFGPE_OK, "evolve 2-D: %s", hfgpe_status_string(rc));
    double en[4] = {0.0, 0.0, 0.0, 0.0};  /* total, kinetic, potential, interaction */
    CHECK(hfgpe_energy(plan, d, T, en) == HFGPE_OK, "energy");
    CHECK(hipMemcpy(h, d, sizeof(double) * 2 * np, hipMemcpyDeviceToHost) == hipSuccess, "copy out");
    double e = rel_l2(h, ex, np);
    double etot = en[0];
    printf("case 2 ground state 2-D c128, NI5 + exact, %ld steps: rel L2 vs closed form %.3e, energy %.15f (exact %.15f)\n",
           nsteps, e, etot, E);
    CHECK(e < 1e-12, "ground state moved: %.3e", e);
    CHECK(fabs(etot - E) < 1e-10, "energy %.17g vs %.17g", etot, E);
    hipFree(d);
    free(h);
    free(ex);
    hfgpe_plan_destroy(plan);
    return 0;
}

static int case_ragged_c64(void)
{
    const int sizes[3] = {64, 256, 1024};
    hfgpe_grid g[3];
    hfgpe_params p[3];
    const double w[1] = {1.0};
    for (int k = 0; k < 3; ++k) {
        const double half = sizes[k] / 64.0 + 6.0;
        grid_1d(&g[k], sizes[k], -half, half);
        params_linear(&p[k], 1.0, w, 1);
        p[k].omega[0].amp = 0.3;  /* omega(t) = 1 + 0.3 sin(2t): the CF4 rule */
        p[k].omega[0].freq = 2.0;
        p[k].sigma.v0 = 5.0 * (k + 1);
        p[k].sigma.kind = HFGPE_TF_SIN;
    }
    double a[16], b[17];
    hfgpe_scheme s;
    CHECK(scheme_of("srkn6_4", HFGPE_HO_CF4, &s, a, b) == HFGPE_OK, "srkn6_4 preset");
    hfgpe_plan *plan = NULL;
    int rc = hfgpe_plan_create(&plan, 3, g, p, &s, HFGPE_C64, 1e-3, NULL, NULL);
    CHECK(rc == HFGPE_OK, "plan_create ragged: %s", hfgpe_status_string(rc));
    if (rc != HFGPE_OK) return 1;
    int64_t off[4];
    CHECK(hfgpe_instance_offsets(plan, off) == HFGPE_OK, "offsets");
    CHECK(off[3] == 64 + 256 + 1024, "total %lld", (long long)off[3]);
    float *h = (float *)malloc(sizeof(float) * 2 * off[3]);
    double n0[3];
    for (int k = 0; k < 3; ++k) {
        const double dx = (g[k].hi[0] - g[k].lo[0]) / sizes[k];
        n0[k] = 0.0;
        for (int i = 0; i < sizes[k]; ++i) {
            double x = g[k].lo[0] + i * dx;
            float re = (float)exp(-(x - 0.5) * (x - 0.5) / 2.0), im = (float)(0.1 * x * re);
            h[2 * (off[k] + i)] = re;
            h[2 * (off[k] + i) + 1] = im;
            n0[k] += ((double)re * re + (double)im * im) * dx;
        }
    }
    void *d = NULL;
    CHECK(hipMalloc(&d, sizeof(float) * 2 * off[3]) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(d, h, sizeof(float) * 2 * off[3], hipMemcpyHostToDevice) == hipSuccess, "copy in");
    rc = hfgpe_evolve(plan, d, 0.0, 500);
    CHECK(rc == HFGPE_OK, "evolve ragged: %s", hfgpe_status_string(rc));
    double nrm[3];
    CHECK(hfgpe_norm(plan, d, nrm) == HFGPE_OK, "norm");
    double worst = 0.0;
    for (int k = 0; k < 3; ++k) worst = fmax(worst, fabs(nrm[k] - n0[k]) / n0[k]);
    printf("case 3 ragged batch c64 (N = 64, 256, 1024), SRKN6 + CF4, sigma > 0, 500 steps: worst relative norm change %.3e\n",
           worst);
    CHECK(worst < 1e-5, "norm not conserved: %.3e", worst);
    hipFree(d);
    free(h);
    hfgpe_plan_destroy(plan);
    return 0;
}

static int case_errors(void)
{
    hfgpe_grid g;
    hfgpe_params p;
    const double w[1] = {1.0};
    double a[16], b[17];
    hfgpe_scheme s;
    grid_1d(&g, 48, -5.0, 5.0);
    params_linear(&p, 1.0, w, 1);
    scheme_of("leapfrog", HFGPE_HO_CF4, &s, a, b);
    hfgpe_plan *plan = (hfgpe_plan *)&g;  /* must be reset to NULL on error */
    int rc = hfgpe_plan_create(&plan, 1, &g, &p, &s, HFGPE_C128, 1e-3, NULL, NULL);
    CHECK(rc == HFGPE_E_UNSUPPORTED_SHAPE && plan == NULL, "N = 48 accepted (rc %d)", rc);
    grid_1d(&g, 64, -5.0, 5.0);
    rc = hfgpe_plan_create(&plan, 1, &g, &p, &s, HFGPE_C128, 1e-3, NULL, NULL);
    CHECK(rc == HFGPE_OK, "plan_create: %s", hfgpe_status_string(rc));
    if (rc == HFGPE_OK) {
        CHECK(hfgpe_evolve(plan, NULL, 0.0, 1) == HFGPE_E_INVALID_ARG, "null state accepted");
        CHECK(hfgpe_evolve(plan, NULL, 0.0, 0) == HFGPE_OK, "zero steps is a no-op");
        hfgpe_plan_destroy(plan);
    }
    CHECK(hfgpe_evolve(NULL, NULL, 0.0, 1) == HFGPE_E_INVALID_ARG, "null plan accepted");
    CHECK(hfgpe_plan_destroy(NULL) == HFGPE_OK, "destroy(NULL)");
    CHECK(strlen(hfgpe_status_string(HFGPE_E_SINGULAR)) > 0, "status string");
    int ma = -1, mi = -1;
    CHECK(hfgpe_version(&ma, &mi) == HFGPE_OK && ma == HFGPE_VERSION_MAJOR && mi == HFGPE_VERSION_MINOR,
          "version");
    printf("case 4 error paths: done\n");
    return 0;
}

int main(void)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        printf("no HIP device\n");
        return 2;
    }
    case_coherent();
    case_ground_2d();
    case_ragged_c64();
    case_errors();
    printf("%s: %d failed check(s)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
