/*
 * hfgpe_oracle.c -- plain, slow FP64 CPU oracle for the Hermite-Fourier
 * split-step integrator of
 *   P. Bader and S. Blanes, "Fourier methods for the perturbed harmonic
 *   oscillator in linear and nonlinear Schroedinger equations" (arXiv:1007.3470).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes (each function cites the passage it follows):
 *   - the periodic equidistant grid x_i = a + i (b-a)/N (Sec. 1, Eq. GP1ODE);
 *   - its own iterative radix-2 FFT, twiddles evaluated directly with cos/sin
 *     (the discrete Fourier transform of Sec. 2.1, Eq. GP1ODE_T);
 *   - the harmonic-oscillator stage coefficients by the "2x2 route": the
 *     classical (Heisenberg) matrix S of the stage propagator is built first
 *     (exact constant-frequency flow, the two-exponential commutator-free
 *     product of Eq. CommutatorFree, the exponential of the sixth-order
 *     Magnus generator of Sec. 4.2, or the fundamental matrix of the stage
 *     integrated as a product of q such Magnus steps over sub-intervals of
 *     length tau/q -- Eq. HO(t)sol states that the exact HO flow for any
 *     omega(t) is of this 2x2 form) and then factored as
 *     S = K(f) D(g) K(e), i.e. g = S12, e = (1-S11)/g, f = (1-S22)/g, which is
 *     the content of Lemma 2 and Theorems 1-2 (Sec. 2.2);
 *   - the Fourier split (i) of Sec. 2.1 as the comparison method: exact
 *     drift D(a_i h/mu) and a B flow that carries the harmonic potential;
 *   - one time step as Table "algorithm" of Sec. 2 with the HO split (ii):
 *     the B flow (Lemma 1, frozen time) and the A flow = K(f) D(g) K(e),
 *     applied one after the other WITHOUT merging adjacent x-phases (the
 *     GPU library merges them; the unmerged order is the cross-check);
 *   - a coupled trap (non-diagonal W, Sec. 1's general x^T M x): the stage
 *     flow is a 2d x 2d symplectic matrix, built per normal mode of the
 *     (averaged) W and factored as K(F) D(G) K(E) with symmetric d x d
 *     matrices, G = S12, E = G^-1 (I - S11), F = (I - S22) G^-1; chirps and
 *     drift are then full quadratic forms x^T C x / 2 and k^T G k / 2;
 *   - norm and energy observables (Sec. 1).
 *
 * Conventions (readings where the paper is silent):
 *   forward DFT  u^_q = sum_n u_n exp(-2 pi i q n / N)   (unnormalised)
 *   inverse DFT  u_n  = (1/N) sum_q u^_q exp(+2 pi i q n / N)
 *   k_q = 2 pi / L * (q < N/2 ? q : q - N)
 *   K(c): u(x) <- exp(-i c x^2/2) u(x);  D(g): u^(k) <- exp(-i g k^2/2) u^(k)
 *   B_w(tau): u <- exp(-i h w (eps V_I(x) + sigma(tau) |u|^2)) u
 *
 * Parameter block (doubles, ORC_NPAR per instance):
 *   [0]            mu
 *   [1+4j..4+4j]   v0, amp, freq, phase of omega_j(t), in the form [36+j]
 *   [13..16]       v0, amp, freq, phase of sigma(t), in the form [39]
 *   [17]           eps
 *   [18+6j..23+6j] V_I factor of axis j: c0, c2, c4, gs, k, phi
 *                  v_j(x) = (c0 + c2 x^2 + c4 x^4) * (gs > 0 ? exp(-x^2/gs) : 1)
 *                           * cos(k x + phi);   V_I = prod_j v_j(x_j)
 *                  (evolve and energy also take eps V_I as an explicit array
 *                  over the grid, which replaces this factor form)
 *   [40..42]       W_xy, W_xz, W_yz: off-diagonal entries of the
 *                  squared-frequency matrix W(t) of a coupled trap
 *                  V_HO = (mu/2) x^T W(t) x, W_jj = omega_j(t)^2 (the general
 *                  quadratic potential x^T M(t) x of Sec. 1 with M = mu W / 2),
 *                  each times its modulation [47+4k..50+4k]
 *   [43..46]       modulation of the perturbation: eps V_I(x, t) =
 *                  m(t) eps V_I(x) (Sec. 1 lets V_I depend on t)
 *   [47..58]       modulations of W_xy, W_xz, W_yz
 *                  a modulation is (amp, freq, phase, form):
 *                  form 0: m(t) = 1 + amp sin(freq t + phase)
 *                  form 2: m(t) = 1 + amp t sech^2(freq (t - phase))
 *                  (all zero: m = 1)
 *   [36+j], [39]   form of omega_j(t), sigma(t):
 *                  0: v(t)   = v0 (1 + amp sin(freq t + phase))
 *                  1: v(t)^2 = v0 (1 + amp sin(freq t + phase))  (the modulated
 *                     squared frequency of the first example of Sec. 4.2)
 *                  2: v(t)   = v0 (1 + amp t sech^2(freq (t - phase)))  (the
 *                     short pulse of the second example of Sec. 4.2)
 *
 * Threads: evolve and energy take a thread count.  The loops they split
 * (pencils of an axis transform, grid points of a pointwise flow) compute
 * every element exactly as one thread would, so the result is bitwise the
 * same for any count; reductions (norm, energy sums) stay sequential.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -fPIC -shared -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NPAR 59
#define ORC_PI 3.14159265358979323846

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ESINGULAR = -2, ORC_EFREQ = -3, ORC_ENOMEM = -4 };
enum { ORC_HO_EXACT_CONST = 0, ORC_HO_CF4 = 1, ORC_HO_MAGNUS6 = 2, ORC_FSPLIT = 3, ORC_HO_FUNDAMENTAL = 4 };

/* ------------------------------------------------------------------------ */
/* Parameter access                                                          */
/* ------------------------------------------------------------------------ */

static double par_mu(const double *p) { return p[0]; }

/* A time-dependent coefficient in one of the three forms listed above;
 * returns v(t) for forms 0 and 2 and v(t)^2 for form 1. */
static double tform(const double *c, int form, double t)
{
    if (form == 2) {
        double sech = 1.0 / cosh(c[2] * (t - c[3]));
        return c[0] * (1.0 + c[1] * t * sech * sech);
    }
    return c[0] * (1.0 + c[1] * sin(c[2] * t + c[3]));
}

/* A modulation factor m(t) (parameter block layout above). */
static double tmod(const double *c, double t)
{
    if ((int)c[3] == 2) {
        double sech = 1.0 / cosh(c[1] * (t - c[2]));
        return 1.0 + c[0] * t * sech * sech;
    }
    return 1.0 + c[0] * sin(c[1] * t + c[2]);
}

/* omega_j(t)^2 of the trap, Eq. GP1b with a time-dependent frequency. */
static double par_omega_sq(const double *p, int j, double t)
{
    int form = (int)p[36 + j];
    double v = tform(p + 1 + 4 * j, form, t);
    return form == 1 ? v : v * v;
}

/* sigma(t) of the mean-field term, Sec. 1 (forms 0 and 2). */
static double par_sigma(const double *p, double t)
{
    return tform(p + 13, (int)p[39], t);
}

static double par_eps(const double *p) { return p[17]; }

/* Time factor of eps V_I at time t. */
static double par_vmod(const double *p, double t) { return tmod(p + 43, t); }

/* Off-diagonal W_ij(t) of the coupled trap (i != j, axes < 3). */
static double par_wcross(const double *p, int i, int j, double t)
{
    if (i > j) { int tt = i; i = j; j = tt; }
    int k = (i == 0) ? (j == 1 ? 0 : 1) : 2;
    return p[40 + k] * tmod(p + 47 + 4 * k, t);
}

static int par_coupled(const double *p, int ndim)
{
    return ndim >= 2 && (p[40] != 0.0 || (ndim == 3 && (p[41] != 0.0 || p[42] != 0.0)));
}

/* W(t), d x d, row-major. */
static void par_wmat(const double *p, int d, double t, double *W)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            W[i * d + j] = (i == j) ? par_omega_sq(p, i, t) : par_wcross(p, i, j, t);
}

/* One separable factor of the perturbing potential V_I. */
static double vfactor(const double *p, int j, double x)
{
    const double *v = p + 18 + 6 * j;
    double poly = v[0] + v[1] * x * x + v[2] * x * x * x * x;
    double gauss = (v[3] > 0.0) ? exp(-x * x / v[3]) : 1.0;
    return poly * gauss * cos(v[4] * x + v[5]);
}

/* ------------------------------------------------------------------------ */
/* FFT: iterative radix-2, bit reversal first, twiddles by direct cos/sin.  */
/* ------------------------------------------------------------------------ */

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

/* Twiddle table tw[q] = exp(-2 pi i q / n), q < n/2, each entry evaluated
 * directly (no recurrences). */
static double *make_twiddles(int n)
{
    int half = n / 2 > 0 ? n / 2 : 1;
    double *tw = (double *)malloc(sizeof(double) * 2 * half);
    if (!tw) return NULL;
    for (int q = 0; q < half; ++q) {
        double ang = -2.0 * ORC_PI * (double)q / (double)n;
        tw[2 * q] = cos(ang);
        tw[2 * q + 1] = sin(ang);
    }
    return tw;
}

/* In-place FFT of a contiguous complex vector z (interleaved re, im).
 * sign = -1 forward (unnormalised), +1 inverse (scaled by 1/n). */
static void fft_contig(int n, double *z, int sign, const double *tw)
{
    if (n <= 1) return;
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = z[2 * i], ti = z[2 * i + 1];
            z[2 * i] = z[2 * j];
            z[2 * i + 1] = z[2 * j + 1];
            z[2 * j] = tr;
            z[2 * j + 1] = ti;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int s = 0; s < n; s += len) {
            for (int q = 0; q < half; ++q) {
                double wr = tw[2 * q * step];
                double wi = tw[2 * q * step + 1];
                if (sign > 0) wi = -wi;
                double *u = z + 2 * (s + q);
                double *v = z + 2 * (s + q + half);
                double vr = v[0] * wr - v[1] * wi;
                double vi = v[0] * wi + v[1] * wr;
                v[0] = u[0] - vr;
                v[1] = u[1] - vi;
                u[0] = u[0] + vr;
                u[1] = u[1] + vi;
            }
        }
    }
    if (sign > 0) {
        double inv = 1.0 / (double)n;
        for (int i = 0; i < 2 * n; ++i) z[i] *= inv;
    }
}

/* FFT along one axis of a row-major d-D array (x fastest).  n[0] is the x
 * extent, n[1] y, n[2] z.  Each pencil is copied out, transformed, copied
 * back; the pencils are shared out over nt threads. */
static int fft_axis(const int n[3], int axis, double *z, int sign, int nt)
{
    int len = n[axis];
    if (len <= 1) return ORC_OK;
    long stride = 1;
    for (int j = 0; j < axis; ++j) stride *= n[j];
    long total = (long)n[0] * n[1] * n[2];
    long npencil = total / len;
    double *tw = make_twiddles(len);
    if (!tw) return ORC_ENOMEM;
    int rc = ORC_OK;
#pragma omp parallel num_threads(nt) if (nt > 1)
    {
        double *buf = (double *)malloc(sizeof(double) * 2 * len);
        if (!buf) {
#pragma omp atomic write
            rc = ORC_ENOMEM;
        }
#pragma omp for schedule(static)
        for (long pidx = 0; pidx < npencil; ++pidx) {
            if (!buf) continue;
            /* pencil start: split pidx into (outer, inner) around the axis */
            long inner = pidx % stride, outer = pidx / stride;
            long base = outer * stride * len + inner;
            for (int i = 0; i < len; ++i) {
                buf[2 * i] = z[2 * (base + i * stride)];
                buf[2 * i + 1] = z[2 * (base + i * stride) + 1];
            }
            fft_contig(len, buf, sign, tw);
            for (int i = 0; i < len; ++i) {
                z[2 * (base + i * stride)] = buf[2 * i];
                z[2 * (base + i * stride) + 1] = buf[2 * i + 1];
            }
        }
        free(buf);
    }
    free(tw);
    return rc;
}

/* d-D FFT = 1-D FFT along every axis. */
static int fftn_nt(int ndim, const int *n_in, double *z, int sign, int nt)
{
    int n[3] = {1, 1, 1};
    if (ndim < 1 || ndim > 3) return ORC_EINVAL;
    for (int j = 0; j < ndim; ++j) {
        if (!is_pow2(n_in[j])) return ORC_EINVAL;
        n[j] = n_in[j];
    }
    for (int j = 0; j < ndim; ++j) {
        int rc = fft_axis(n, j, z, sign, nt);
        if (rc) return rc;
    }
    return ORC_OK;
}

int orc_fftn(int ndim, const int *n_in, double *z, int sign)
{
    return fftn_nt(ndim, n_in, z, sign, 1);
}

/* ------------------------------------------------------------------------ */
/* 2x2 route for the harmonic-oscillator stage coefficients                 */
/* ------------------------------------------------------------------------ */

/* The 2x2 matrices of this section are held in "deviation form"
 * X = S - I, so that 1 - S11 and 1 - S22, which the factorisation divides by
 * S12, come out without the cancellation 1 - cos(w tau) would suffer for
 * small steps.  cos(x) - 1 is evaluated as -2 sin^2(x/2). */
static double cosm1(double x)
{
    double s = sin(0.5 * x);
    return -2.0 * s * s;
}

/* Product in deviation form: (I + A)(I + B) = I + A + B + A B. */
static void dev_mul(const double A[4], const double B[4], double C[4])
{
    double c0 = A[0] + B[0] + (A[0] * B[0] + A[1] * B[2]);
    double c1 = A[1] + B[1] + (A[0] * B[1] + A[1] * B[3]);
    double c2 = A[2] + B[2] + (A[2] * B[0] + A[3] * B[2]);
    double c3 = A[3] + B[3] + (A[2] * B[1] + A[3] * B[3]);
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}

/* Classical flow over time tau of H = p^2/(2 mu) + mu q x^2 / 2 (q = omega^2
 * held fixed), acting on (x, p): x' = p/mu, p' = -mu q x.  This is the exact
 * HO evolution matrix of Lemma 2's proof, generalised to mu.  Deviation form. */
static int ho_flow(double q, double mu, double tau, double X[4])
{
    if (!(q > 0.0)) return ORC_EFREQ;
    double w = sqrt(q);
    double cm = cosm1(w * tau), s = sin(w * tau);
    X[0] = cm;
    X[1] = s / (mu * w);
    X[2] = -mu * w * s;
    X[3] = cm;
    return ORC_OK;
}

/* Fourth-order commutator-free approximation, Eq. CommutatorFree: the
 * product of two constant-frequency half-step flows with Gauss-averaged
 * squared frequencies.  The right factor (weighted toward the earlier node)
 * acts first, so S = M(omega_L^2) M(omega_R^2). */
static int ho_cf4(const double *p, int axis, double t0, double tau, double X[4])
{
    double c1 = 0.5 - sqrt(3.0) / 6.0, c2 = 0.5 + sqrt(3.0) / 6.0;
    double al = 0.5 - 1.0 / sqrt(3.0), be = 1.0 - al;
    double q1 = par_omega_sq(p, axis, t0 + c1 * tau);
    double q2 = par_omega_sq(p, axis, t0 + c2 * tau);
    double qL = al * q1 + be * q2;
    double qR = be * q1 + al * q2;
    double ML[4], MR[4];
    int rc = ho_flow(qL, par_mu(p), 0.5 * tau, ML);
    if (rc) return rc;
    rc = ho_flow(qR, par_mu(p), 0.5 * tau, MR);
    if (rc) return rc;
    dev_mul(ML, MR, X);
    return ORC_OK;
}

/* Sixth-order Magnus approximation of Sec. 4.2: exponent
 * -i (tau/2)(alpha x^2 + beta (xp+px) + gamma p^2) with the three-node Gauss
 * rule on the stage interval [t0, t0+tau]; the omega_i of the printed
 * formulas are read as squared frequencies at the nodes.  The formulas are
 * for mu = 1; other mu go through the canonical scaling X = sqrt(mu) x,
 * P = p / sqrt(mu).  Deviation form. */
static int ho_magnus6(const double *p, int axis, double t0, double tau, double X[4])
{
    double c1 = 0.5 - sqrt(15.0) / 10.0, c2 = 0.5, c3 = 0.5 + sqrt(15.0) / 10.0;
    double w1 = par_omega_sq(p, axis, t0 + c1 * tau);
    double w2 = par_omega_sq(p, axis, t0 + c2 * tau);
    double w3 = par_omega_sq(p, axis, t0 + c3 * tau);
    double tt = tau * tau;
    double alpha = (5.0 * w1 + 8.0 * w2 + 5.0 * w3) / 18.0
                 + tt / 486.0 * (17.0 / 4.0 * (w1 * w1 + w3 * w3) + 8.0 * w2 * w2
                                 + w1 * w2 + w2 * w3 - 37.0 / 2.0 * w1 * w3);
    double beta = tau * sqrt(5.0 / 3.0) * (w3 - w1)
                * (1.0 / 12.0 + tt / 3240.0 * (5.0 * w1 + 8.0 * w2 + 5.0 * w3));
    double gamma = 1.0 + tt / 54.0 * (w1 - 2.0 * w2 + w3);
    /* Classical generator of H = (alpha x^2 + 2 beta x p + gamma p^2)/2:
     * x' = beta x + gamma p, p' = -alpha x - beta p.  Its square is
     * -(alpha gamma - beta^2) I, so exp(tau G) = cos(eta tau) I + sin(eta tau)/eta G. */
    double eta2 = alpha * gamma - beta * beta;
    if (!(eta2 > 0.0)) return ORC_EFREQ;
    double eta = sqrt(eta2);
    double cm = cosm1(eta * tau), s = sin(eta * tau) / eta;
    /* back to the physical frame: x = X / sqrt(mu), p = sqrt(mu) P */
    double mu = par_mu(p);
    X[0] = cm + s * beta;
    X[1] = s * gamma / mu;
    X[2] = -s * alpha * mu;
    X[3] = cm - s * beta;
    return ORC_OK;
}

/* Fundamental matrix of the stage, x' = p/mu, p' = -mu omega(t)^2 x over
 * [t0, t0 + tau], integrated numerically: the flow over consecutive
 * sub-intervals of length tau/q composes (later sub-intervals act last), and
 * each sub-interval's flow is taken from the sixth-order Magnus rule above.
 * Deviation form. */
static int ho_fundamental(const double *p, int axis, double t0, double tau, int q, double X[4])
{
    if (q < 1) return ORC_EINVAL;
    double h = tau / (double)q;
    X[0] = X[1] = X[2] = X[3] = 0.0;
    for (int k = 0; k < q; ++k) {
        double A[4], Y[4];
        int rc = ho_magnus6(p, axis, t0 + (double)k * h, h, A);
        if (rc) return rc;
        dev_mul(A, X, Y);
        memcpy(X, Y, sizeof(Y));
    }
    return ORC_OK;
}

/* Stage matrix (deviation form) for one axis over [t0, t0 + tau]; q is the
 * sub-step count of the fundamental-matrix rule. */
static int ho_stage_matrix(int rule, int q, const double *p, int axis, double t0, double tau,
                           double S[4])
{
    switch (rule) {
    case ORC_HO_EXACT_CONST:
        return ho_flow(par_omega_sq(p, axis, t0), par_mu(p), tau, S);
    case ORC_HO_CF4:
        return ho_cf4(p, axis, t0, tau, S);
    case ORC_HO_MAGNUS6:
        return ho_magnus6(p, axis, t0, tau, S);
    case ORC_HO_FUNDAMENTAL:
        return ho_fundamental(p, axis, t0, tau, q, S);
    default:
        return ORC_EINVAL;
    }
}

/* Factor a symplectic 2x2 matrix S = I + X as K(f) D(g) K(e) (rightmost
 * first), with K(c) = [[1,0],[-c,1]] and D(g) = [[1,g],[0,1]]:
 * K(f) D(g) K(e) = [[1 - g e, g], [-f - e + f g e, 1 - f g]], hence
 * g = S12, e = (1 - S11)/g, f = (1 - S22)/g. */
static int factor_kdk(const double X[4], double *f, double *g, double *e)
{
    double gg = X[1];
    if (!(fabs(gg) > 1e-300) || !isfinite(gg)) return ORC_ESINGULAR;
    *g = gg;
    *e = -X[0] / gg;
    *f = -X[3] / gg;
    return ORC_OK;
}

/* Public: the 2x2 stage matrix S (not the deviation) for tests. */
int orc_stage_matrix(int rule, int q, const double *par, int axis, double t0, double tau, double *S)
{
    int rc = ho_stage_matrix(rule, q, par, axis, t0, tau, S);
    if (rc) return rc;
    S[0] += 1.0;
    S[3] += 1.0;
    return ORC_OK;
}

/* Public: (f, g, e) of every stage and axis of the step starting at tn.
 * out[(i*ndim + j)*3 + {0,1,2}] = f, g, e of stage i, axis j. */
int orc_stage_coeffs(int ndim, const double *par, int m, const double *a, int rule, int q,
                     double dt, double tn, double *out)
{
    if (rule == ORC_FSPLIT) return ORC_EINVAL;
    double tau = tn;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < ndim; ++j) {
            double X[4];
            int rc = ho_stage_matrix(rule, q, par, j, tau, a[i] * dt, X);
            if (rc) return rc;
            rc = factor_kdk(X, &out[(i * ndim + j) * 3 + 0], &out[(i * ndim + j) * 3 + 1],
                            &out[(i * ndim + j) * 3 + 2]);
            if (rc) return rc;
        }
        tau = tau + a[i] * dt;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Coupled trap: 2d x 2d stage matrices (d <= 3)                            */
/* ------------------------------------------------------------------------ */

/* Symmetric eigen-decomposition W = Q diag(lam) Q^T by cyclic Jacobi
 * rotations (d <= 3); Q holds the eigenvectors as columns. */
static void sym_eig(int d, const double *Win, double *lam, double *Q)
{
    double A[9];
    memcpy(A, Win, sizeof(double) * d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Q[i * d + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = i + 1; j < d; ++j) off += A[i * d + j] * A[i * d + j];
        if (off < 1e-300) break;
        for (int pq = 0; pq < d; ++pq)
            for (int qq = pq + 1; qq < d; ++qq) {
                double apq = A[pq * d + qq];
                if (apq == 0.0) continue;
                double theta = (A[qq * d + qq] - A[pq * d + pq]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < d; ++k) { /* A <- J^T A J */
                    double akp = A[k * d + pq], akq = A[k * d + qq];
                    A[k * d + pq] = c * akp - sn * akq;
                    A[k * d + qq] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {
                    double apk = A[pq * d + k], aqk = A[qq * d + k];
                    A[pq * d + k] = c * apk - sn * aqk;
                    A[qq * d + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < d; ++k) {
                    double qkp = Q[k * d + pq], qkq = Q[k * d + qq];
                    Q[k * d + pq] = c * qkp - sn * qkq;
                    Q[k * d + qq] = sn * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < d; ++i) lam[i] = A[i * d + i];
}

static void mat_mul(int d, const double *A, const double *B, double *C)
{
    double T[9];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double acc = 0.0;
            for (int k = 0; k < d; ++k) acc += A[i * d + k] * B[k * d + j];
            T[i * d + j] = acc;
        }
    memcpy(C, T, sizeof(double) * d * d);
}

/* Inverse by Gauss-Jordan elimination with partial pivoting. */
static int mat_inv(int d, const double *Ain, double *X)
{
    double A[9];
    memcpy(A, Ain, sizeof(double) * d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) X[i * d + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (fabs(A[r * d + c]) > fabs(A[piv * d + c])) piv = r;
        if (!(fabs(A[piv * d + c]) > 1e-300)) return ORC_ESINGULAR;
        for (int k = 0; k < d; ++k) {
            double t = A[c * d + k]; A[c * d + k] = A[piv * d + k]; A[piv * d + k] = t;
            t = X[c * d + k]; X[c * d + k] = X[piv * d + k]; X[piv * d + k] = t;
        }
        double inv = 1.0 / A[c * d + c];
        for (int k = 0; k < d; ++k) { A[c * d + k] *= inv; X[c * d + k] *= inv; }
        for (int r = 0; r < d; ++r) {
            if (r == c) continue;
            double f = A[r * d + c];
            for (int k = 0; k < d; ++k) { A[r * d + k] -= f * A[c * d + k]; X[r * d + k] -= f * X[c * d + k]; }
        }
    }
    return ORC_OK;
}

/* A 2d x 2d matrix in deviation form, as four d x d blocks: S = I + X. */
typedef struct { double b[4][9]; } blk_t;

/* Flow over tau of H = p^2/(2 mu) + (mu/2) x^T W x, W constant and positive
 * definite: per normal mode (W = Q diag(w_k^2) Q^T) the constant-frequency
 * flow of Lemma 2's proof, rotated back.  Deviation form. */
static int ho_flow_full(int d, const double *W, double mu, double tau, blk_t *X)
{
    double lam[3], Q[9];
    sym_eig(d, W, lam, Q);
    double cm[3], s1[3], s2[3];
    for (int k = 0; k < d; ++k) {
        if (!(lam[k] > 0.0)) return ORC_EFREQ;
        double w = sqrt(lam[k]);
        cm[k] = cosm1(w * tau);
        s1[k] = sin(w * tau) / (mu * w);
        s2[k] = -mu * w * sin(w * tau);
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double a = 0, b = 0, c = 0;
            for (int k = 0; k < d; ++k) {
                double qq = Q[i * d + k] * Q[j * d + k];
                a += qq * cm[k];
                b += qq * s1[k];
                c += qq * s2[k];
            }
            X->b[0][i * d + j] = a;
            X->b[1][i * d + j] = b;
            X->b[2][i * d + j] = c;
            X->b[3][i * d + j] = a;
        }
    return ORC_OK;
}

/* (I + A)(I + B) = I + A + B + A B, blockwise. */
static void blk_mul(int d, const blk_t *A, const blk_t *B, blk_t *C)
{
    blk_t T;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double P1[9], P2[9];
            mat_mul(d, A->b[r * 2 + 0], B->b[0 * 2 + c], P1);
            mat_mul(d, A->b[r * 2 + 1], B->b[1 * 2 + c], P2);
            for (int k = 0; k < d * d; ++k)
                T.b[r * 2 + c][k] = A->b[r * 2 + c][k] + B->b[r * 2 + c][k] + (P1[k] + P2[k]);
        }
    *C = T;
}

/* Stage matrix of the coupled trap over [t0, t0 + tau]: the exact flow for a
 * constant W (rule exact_const), or the commutator-free product of
 * Eq. CommutatorFree with W averaged at the two Gauss nodes (rule cf4; the
 * factor weighted to the earlier node acts first). */
static int ho_stage_full(int rule, const double *p, int d, double t0, double tau, blk_t *X)
{
    double mu = par_mu(p);
    if (rule == ORC_HO_EXACT_CONST) {
        double W[9];
        par_wmat(p, d, t0, W);
        return ho_flow_full(d, W, mu, tau, X);
    }
    if (rule == ORC_HO_CF4) {
        double c1 = 0.5 - sqrt(3.0) / 6.0, c2 = 0.5 + sqrt(3.0) / 6.0;
        double al = 0.5 - 1.0 / sqrt(3.0), be = 1.0 - al;
        double W1[9], W2[9], WL[9], WR[9];
        par_wmat(p, d, t0 + c1 * tau, W1);
        par_wmat(p, d, t0 + c2 * tau, W2);
        for (int k = 0; k < d * d; ++k) {
            WL[k] = al * W1[k] + be * W2[k];
            WR[k] = be * W1[k] + al * W2[k];
        }
        blk_t L, R;
        int rc = ho_flow_full(d, WL, mu, 0.5 * tau, &L);
        if (rc) return rc;
        rc = ho_flow_full(d, WR, mu, 0.5 * tau, &R);
        if (rc) return rc;
        blk_mul(d, &L, &R, X);
        return ORC_OK;
    }
    return ORC_EINVAL;  /* other rules are written for a diagonal W */
}

/* S = I + X = K(F) D(G) K(E) with K(C) = [[I, 0], [-C, I]], D(G) = [[I, G], [0, I]]:
 * G = S12, E = -G^-1 X11, F = -X22 G^-1. */
static int factor_kdk_full(int d, const blk_t *X, double *F, double *Gm, double *E)
{
    double Gi[9] = {0};
    memcpy(Gm, X->b[1], sizeof(double) * d * d);
    int rc = mat_inv(d, Gm, Gi);
    if (rc) return rc;
    mat_mul(d, Gi, X->b[0], E);
    mat_mul(d, X->b[3], Gi, F);
    for (int k = 0; k < d * d; ++k) { E[k] = -E[k]; F[k] = -F[k]; }
    return ORC_OK;
}

/* The K(F) D(G) K(E) factors (symmetric d x d) that make up one stage of the
 * coupled trap, in the order they act.  For d >= 2 the triple K(F) D(G) K(E)
 * spans only flows whose S12 block is symmetric; the flow of a constant W is
 * one of them (per normal mode it is Lemma 2), but the commutator-free
 * product of two different W is in general not.  So the exact rule gives one
 * factor triple, and the commutator-free rule gives its two exponentials as
 * two triples: the flow of W_R over tau/2, then that of W_L over tau/2. */
static int coupled_factors(int rule, const double *p, int d, double t0, double tau, double *F,
                           double *Gm, double *E, int *nf)
{
    double mu = par_mu(p);
    blk_t X;
    if (rule == ORC_HO_EXACT_CONST) {
        double W[9];
        par_wmat(p, d, t0, W);
        int rc = ho_flow_full(d, W, mu, tau, &X);
        if (rc) return rc;
        *nf = 1;
        return factor_kdk_full(d, &X, F, Gm, E);
    }
    if (rule == ORC_HO_CF4) {
        double c1 = 0.5 - sqrt(3.0) / 6.0, c2 = 0.5 + sqrt(3.0) / 6.0;
        double al = 0.5 - 1.0 / sqrt(3.0), be = 1.0 - al;
        double W1[9], W2[9], WL[9], WR[9];
        par_wmat(p, d, t0 + c1 * tau, W1);
        par_wmat(p, d, t0 + c2 * tau, W2);
        for (int k = 0; k < d * d; ++k) {
            WL[k] = al * W1[k] + be * W2[k];
            WR[k] = be * W1[k] + al * W2[k];
        }
        const double *Ws[2] = {WR, WL};
        for (int h = 0; h < 2; ++h) {
            int rc = ho_flow_full(d, Ws[h], mu, 0.5 * tau, &X);
            if (rc) return rc;
            rc = factor_kdk_full(d, &X, F + 9 * h, Gm + 9 * h, E + 9 * h);
            if (rc) return rc;
        }
        *nf = 2;
        return ORC_OK;
    }
    return ORC_EINVAL;
}

/* Public (tests): the 2d x 2d stage matrix S of the coupled trap, row-major. */
int orc_stage_matrix_full(int rule, const double *par, int d, double t0, double tau, double *S)
{
    blk_t X;
    if (d < 2 || d > 3) return ORC_EINVAL;
    int rc = ho_stage_full(rule, par, d, t0, tau, &X);
    if (rc) return rc;
    int n = 2 * d;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            int br = r / d, bc = c / d;
            S[r * n + c] = X.b[br * 2 + bc][(r % d) * d + (c % d)] + (r == c ? 1.0 : 0.0);
        }
    return ORC_OK;
}

/* Public (tests): F, G, E (each d x d, row-major) of every factor triple of
 * the step starting at tn for the coupled trap, in the order they act (one
 * per stage for exact_const, two per stage for cf4):
 * out[(f*3 + {0,1,2}) * d*d + ...]; *nout = number of triples. */
int orc_stage_coeffs_full(int d, const double *par, int m, const double *a, int rule, double dt,
                          double tn, double *out, int *nout)
{
    double tau = tn;
    int k = 0;
    for (int i = 0; i < m; ++i) {
        double F[18], Gm[18], E[18];
        int nf = 0;
        int rc = coupled_factors(rule, par, d, tau, a[i] * dt, F, Gm, E, &nf);
        if (rc) return rc;
        for (int h = 0; h < nf; ++h, ++k) {
            memcpy(out + (k * 3 + 0) * d * d, F + 9 * h, sizeof(double) * d * d);
            memcpy(out + (k * 3 + 1) * d * d, Gm + 9 * h, sizeof(double) * d * d);
            memcpy(out + (k * 3 + 2) * d * d, E + 9 * h, sizeof(double) * d * d);
        }
        tau = tau + a[i] * dt;
    }
    *nout = k;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pointwise flows and the time step                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ndim;
    int n[3];
    double lo[3], dx[3];
    long total;
    const double *par;
    double *vi;   /* eps * V_I at every grid point */
    double *x2h;  /* per-axis x_j^2 / 2 tables, concatenated */
    double *k2h;  /* per-axis k_j^2 / 2 tables, concatenated */
    int nt;       /* threads for the pencil and point loops */
} grid_t;

static long axis_index(const grid_t *G, long idx, int axis)
{
    long s = 1;
    for (int j = 0; j < axis; ++j) s *= G->n[j];
    return (idx / s) % G->n[axis];
}

/* vi_in: eps V_I at every point (row-major, x fastest), or NULL for the
 * separable factor form of the parameter block. */
static int grid_init(grid_t *G, int ndim, const int *n, const double *lo, const double *hi,
                     const double *par, const double *vi_in, int nt)
{
    memset(G, 0, sizeof(*G));
    if (ndim < 1 || ndim > 3 || nt < 1) return ORC_EINVAL;
    G->ndim = ndim;
    G->nt = nt;
    G->par = par;
    G->total = 1;
    int off = 0;
    for (int j = 0; j < 3; ++j) {
        G->n[j] = (j < ndim) ? n[j] : 1;
        if (!is_pow2(G->n[j])) return ORC_EINVAL;
        G->lo[j] = (j < ndim) ? lo[j] : 0.0;
        G->dx[j] = (j < ndim) ? (hi[j] - lo[j]) / (double)G->n[j] : 1.0;
        G->total *= G->n[j];
        off += G->n[j];
    }
    G->vi = (double *)malloc(sizeof(double) * G->total);
    G->x2h = (double *)malloc(sizeof(double) * off);
    G->k2h = (double *)malloc(sizeof(double) * off);
    if (!G->vi || !G->x2h || !G->k2h) return ORC_ENOMEM;
    off = 0;
    for (int j = 0; j < 3; ++j) {
        double L = G->dx[j] * G->n[j];
        for (int i = 0; i < G->n[j]; ++i) {
            double x = (j < ndim) ? G->lo[j] + i * G->dx[j] : 0.0;
            int q = (2 * i < G->n[j]) ? i : i - G->n[j];
            double k = (j < ndim) ? 2.0 * ORC_PI / L * q : 0.0;
            G->x2h[off + i] = 0.5 * x * x;
            G->k2h[off + i] = 0.5 * k * k;
        }
        off += G->n[j];
    }
    double eps = par_eps(par);
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double v = 1.0;
        for (int j = 0; j < ndim; ++j) {
            long i = axis_index(G, idx, j);
            v *= vfactor(par, j, G->lo[j] + i * G->dx[j]);
        }
        G->vi[idx] = vi_in ? vi_in[idx] : eps * v;
    }
    return ORC_OK;
}

static void grid_free(grid_t *G)
{
    free(G->vi);
    free(G->x2h);
    free(G->k2h);
}

static const double *axis_table(const grid_t *G, const double *tab, int axis)
{
    int off = 0;
    for (int j = 0; j < axis; ++j) off += G->n[j];
    return tab + off;
}

static void mul_phase(double *z, double theta)
{
    /* z <- exp(-i theta) z */
    double c = cos(theta), s = sin(theta);
    double re = z[0] * c + z[1] * s;
    double im = z[1] * c - z[0] * s;
    z[0] = re;
    z[1] = im;
}

/* B flow frozen at time tau with weight w (Lemma 1; Table "algorithm"):
 * u <- exp(-i dt w (eps V_I(x, tau) + sigma(tau) |u|^2)) u. */
static void apply_B(const grid_t *G, double *u, double dt, double w, double tau)
{
    if (w == 0.0) return;
    double sig = par_sigma(G->par, tau), vm = par_vmod(G->par, tau);
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double a2 = u[2 * idx] * u[2 * idx] + u[2 * idx + 1] * u[2 * idx + 1];
        mul_phase(u + 2 * idx, dt * w * (vm * G->vi[idx] + sig * a2));
    }
}

/* Kick K(c): u <- exp(-i sum_j c_j x_j^2 / 2) u. */
static void apply_K(const grid_t *G, double *u, const double *c)
{
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double th = 0.0;
        for (int j = 0; j < G->ndim; ++j)
            th += c[j] * axis_table(G, G->x2h, j)[axis_index(G, idx, j)];
        mul_phase(u + 2 * idx, th);
    }
}

/* Drift D(g): d-D FFT, multiply by exp(-i sum_j g_j k_j^2/2), inverse FFT
 * (Eq. GP1ODE_T and its solution). */
static int apply_D(const grid_t *G, double *u, const double *g)
{
    int rc = fftn_nt(G->ndim, G->n, u, -1, G->nt);
    if (rc) return rc;
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double th = 0.0;
        for (int j = 0; j < G->ndim; ++j)
            th += g[j] * axis_table(G, G->k2h, j)[axis_index(G, idx, j)];
        mul_phase(u + 2 * idx, th);
    }
    return fftn_nt(G->ndim, G->n, u, +1, G->nt);
}

/* Coordinates (or wavenumbers) of grid point idx along every axis. */
static void point_coords(const grid_t *G, long idx, double *x, double *k)
{
    for (int j = 0; j < G->ndim; ++j) {
        long i = axis_index(G, idx, j);
        if (x) x[j] = G->lo[j] + i * G->dx[j];
        if (k) {
            double L = G->dx[j] * G->n[j];
            long q = (2 * i < G->n[j]) ? i : i - G->n[j];
            k[j] = 2.0 * ORC_PI / L * (double)q;
        }
    }
}

static double quad_form(int d, const double *C, const double *v)
{
    double acc = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) acc += C[i * d + j] * v[i] * v[j];
    return 0.5 * acc;
}

/* Chirp with a symmetric matrix: u <- exp(-i x^T C x / 2) u. */
static void apply_K_full(const grid_t *G, double *u, const double *C)
{
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double x[3];
        point_coords(G, idx, x, NULL);
        mul_phase(u + 2 * idx, quad_form(G->ndim, C, x));
    }
}

/* Drift with a symmetric matrix: FFT, u^ <- exp(-i k^T G k / 2) u^, inverse FFT. */
static int apply_D_full(const grid_t *G, double *u, const double *Gm)
{
    int rc = fftn_nt(G->ndim, G->n, u, -1, G->nt);
    if (rc) return rc;
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double k[3];
        point_coords(G, idx, NULL, k);
        mul_phase(u + 2 * idx, quad_form(G->ndim, Gm, k));
    }
    return fftn_nt(G->ndim, G->n, u, +1, G->nt);
}

/* B flow of the Fourier split (Eq. FourierSplit) frozen at tau: the harmonic
 * potential joins the pointwise phase,
 * u <- exp(-i dt w (sum_j mu omega_j(tau)^2 x_j^2/2 + eps V_I + sigma |u|^2)) u. */
static void apply_B_fsplit(const grid_t *G, double *u, double dt, double w, double tau)
{
    if (w == 0.0) return;
    double sig = par_sigma(G->par, tau), mu = par_mu(G->par), vm = par_vmod(G->par, tau);
    double q[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < G->ndim; ++j) {
        q[j] = mu * par_omega_sq(G->par, j, tau);
    }
#pragma omp parallel for schedule(static) num_threads(G->nt) if (G->nt > 1)
    for (long idx = 0; idx < G->total; ++idx) {
        double harm = 0.0;
        for (int j = 0; j < G->ndim; ++j)
            harm += q[j] * axis_table(G, G->x2h, j)[axis_index(G, idx, j)];
        if (par_coupled(G->par, G->ndim)) {  /* off-diagonal part of (mu/2) x^T W x */
            double x[3];
            point_coords(G, idx, x, NULL);
            for (int i = 0; i < G->ndim; ++i)
                for (int j = i + 1; j < G->ndim; ++j) harm += mu * par_wcross(G->par, i, j, tau) * x[i] * x[j];
        }
        double a2 = u[2 * idx] * u[2 * idx] + u[2 * idx + 1] * u[2 * idx + 1];
        mul_phase(u + 2 * idx, dt * w * (harm + vm * G->vi[idx] + sig * a2));
    }
}

/* One step of the Fourier split: A = p^2/(2 mu) is the exact drift D(a_i dt / mu),
 * B carries the harmonic potential (Eq. FourierSplit with Table "algorithm"). */
static int step_fsplit(const grid_t *G, double *u, int m, const double *a, const double *b, double dt,
                       double tn)
{
    double tau = tn;
    apply_B_fsplit(G, u, dt, b[0], tau);
    for (int i = 0; i < m; ++i) {
        double g[3];
        for (int j = 0; j < G->ndim; ++j) g[j] = a[i] * dt / par_mu(G->par);
        int rc = apply_D(G, u, g);
        if (rc) return rc;
        tau = tau + a[i] * dt;
        apply_B_fsplit(G, u, dt, b[i + 1], tau);
    }
    return ORC_OK;
}

/* One step t_n -> t_n + dt of the composition (Eq. prod-gen, Table
 * "algorithm"), with each A flow replaced by its K(f) D(g) K(e) factorisation.
 * b holds m+1 weights (BAB form; b[0] = 0 gives an ABA-type scheme). */
static int step_once(const grid_t *G, double *u, int m, const double *a, const double *b,
                     int rule, int q, double dt, double tn)
{
    if (rule == ORC_FSPLIT) return step_fsplit(G, u, m, a, b, dt, tn);
    double tau = tn;
    apply_B(G, u, dt, b[0], tau);
    if (par_coupled(G->par, G->ndim)) {  /* coupled trap: matrix chirps and drift */
        const int d = G->ndim;
        for (int i = 0; i < m; ++i) {
            double F[18], Gm[18], E[18];
            int nf = 0;
            int rc = coupled_factors(rule, G->par, d, tau, a[i] * dt, F, Gm, E, &nf);
            if (rc) return rc;
            for (int h = 0; h < nf; ++h) {
                apply_K_full(G, u, E + 9 * h);
                rc = apply_D_full(G, u, Gm + 9 * h);
                if (rc) return rc;
                apply_K_full(G, u, F + 9 * h);
            }
            tau = tau + a[i] * dt;
            apply_B(G, u, dt, b[i + 1], tau);
        }
        return ORC_OK;
    }
    for (int i = 0; i < m; ++i) {
        double f[3], g[3], e[3];
        for (int j = 0; j < G->ndim; ++j) {
            double X[4];
            int rc = ho_stage_matrix(rule, q, G->par, j, tau, a[i] * dt, X);
            if (rc) return rc;
            rc = factor_kdk(X, &f[j], &g[j], &e[j]);
            if (rc) return rc;
        }
        apply_K(G, u, e);
        int rc = apply_D(G, u, g);
        if (rc) return rc;
        apply_K(G, u, f);
        tau = tau + a[i] * dt;
        apply_B(G, u, dt, b[i + 1], tau);
    }
    return ORC_OK;
}

/* Public: evolve one instance nsteps steps from t0 on nthreads threads.  psi
 * is interleaved complex (re, im) in row-major order with x fastest. */
int orc_evolve(int ndim, const int *n, const double *lo, const double *hi, const double *par,
               int m, const double *a, const double *b, int rule, int q, double dt, double t0,
               long nsteps, const double *vi, double *psi, int nthreads)
{
    if (m < 1 || nsteps < 0) return ORC_EINVAL;
    grid_t G;
    int rc = grid_init(&G, ndim, n, lo, hi, par, vi, nthreads);
    if (rc) { grid_free(&G); return rc; }
    for (long s = 0; s < nsteps && rc == ORC_OK; ++s)
        rc = step_once(&G, psi, m, a, b, rule, q, dt, t0 + (double)s * dt);
    grid_free(&G);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Observables                                                               */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } ksum_t;
static void ksum_add(ksum_t *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double ksum_val(const ksum_t *k) { return k->s + k->c; }

/* Discrete L2 norm squared: h^d sum |u|^2 (the preserved norm of Sec. 1). */
int orc_norm(int ndim, const int *n, const double *lo, const double *hi, const double *psi,
             double *out)
{
    double cell = 1.0;
    long total = 1;
    for (int j = 0; j < ndim; ++j) {
        if (!is_pow2(n[j])) return ORC_EINVAL;
        cell *= (hi[j] - lo[j]) / (double)n[j];
        total *= n[j];
    }
    ksum_t acc = {0.0, 0.0};
    for (long idx = 0; idx < total; ++idx)
        ksum_add(&acc, psi[2 * idx] * psi[2 * idx] + psi[2 * idx + 1] * psi[2 * idx + 1]);
    *out = cell * ksum_val(&acc);
    return ORC_OK;
}

/* Energy of the GPE (Sec. 1):
 *   E = h^d [ (1/Ntot) sum_k |k|^2/(2 mu) |u^_k|^2
 *             + sum_x (V(x,t) |u|^2 + sigma(t)/2 |u|^4) ],
 *   V = sum_j mu omega_j(t)^2 x_j^2 / 2 + eps V_I(x).
 * out[0..3] = total, kinetic, potential, interaction. */
int orc_energy(int ndim, const int *n, const double *lo, const double *hi, const double *par,
               double t, const double *vi, const double *psi, double *out, int nthreads)
{
    grid_t G;
    int rc = grid_init(&G, ndim, n, lo, hi, par, vi, nthreads);
    if (rc) { grid_free(&G); return rc; }
    double cell = 1.0;
    for (int j = 0; j < ndim; ++j) cell *= G.dx[j];
    double *uh = (double *)malloc(sizeof(double) * 2 * G.total);
    if (!uh) { grid_free(&G); return ORC_ENOMEM; }
    memcpy(uh, psi, sizeof(double) * 2 * G.total);
    rc = fftn_nt(ndim, G.n, uh, -1, G.nt);
    if (rc) { free(uh); grid_free(&G); return rc; }
    double mu = par_mu(par), sig = par_sigma(par, t), vm = par_vmod(par, t);
    ksum_t kin = {0, 0}, pot = {0, 0}, inter = {0, 0};
    for (long idx = 0; idx < G.total; ++idx) {
        double k2h = 0.0, vh = 0.0;
        for (int j = 0; j < ndim; ++j) {
            long i = axis_index(&G, idx, j);
            k2h += axis_table(&G, G.k2h, j)[i];
            vh += mu * par_omega_sq(par, j, t) * axis_table(&G, G.x2h, j)[i];
        }
        if (par_coupled(par, ndim)) {  /* off-diagonal part of (mu/2) x^T W x */
            double x[3];
            point_coords(&G, idx, x, NULL);
            for (int i = 0; i < ndim; ++i)
                for (int j = i + 1; j < ndim; ++j) vh += mu * par_wcross(par, i, j, t) * x[i] * x[j];
        }
        double a2h = uh[2 * idx] * uh[2 * idx] + uh[2 * idx + 1] * uh[2 * idx + 1];
        ksum_add(&kin, k2h / mu * a2h);
        double a2 = psi[2 * idx] * psi[2 * idx] + psi[2 * idx + 1] * psi[2 * idx + 1];
        ksum_add(&pot, (vh + vm * G.vi[idx]) * a2);
        ksum_add(&inter, 0.5 * sig * a2 * a2);
    }
    out[1] = cell * ksum_val(&kin) / (double)G.total;
    out[2] = cell * ksum_val(&pot);
    out[3] = cell * ksum_val(&inter);
    out[0] = out[1] + out[2] + out[3];
    free(uh);
    grid_free(&G);
    return ORC_OK;
}

int orc_npar(void) { return ORC_NPAR; }

/* Public (tests): apply the drift D(g) alone to one instance. */
int orc_drift(int ndim, const int *n, const double *lo, const double *hi, const double *g,
              double *psi)
{
    double par[ORC_NPAR];
    memset(par, 0, sizeof(par));
    par[0] = 1.0;
    for (int j = 0; j < 3; ++j) par[18 + 6 * j] = 1.0;
    grid_t G;
    int rc = grid_init(&G, ndim, n, lo, hi, par, NULL, 1);
    if (rc == ORC_OK) rc = apply_D(&G, psi, g);
    grid_free(&G);
    return rc;
}
