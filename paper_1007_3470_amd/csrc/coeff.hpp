// coeff.hpp -- stage coefficients (f, g, e) of the harmonic-oscillator part
// by the closed forms of Lemma 2 and Theorems 1-2, or by the numerically
// integrated fundamental matrix, in FP64, usable on the host
// (hfgpe_stage_coeffs, plan validation) and in the coefficient kernel.
//
// A stage over [t0, t0 + tau] propagates H0(t) = p^2/(2 mu) + mu omega(t)^2 x^2/2
// as K(f) D(g) K(e) (e acts first):
//   K(c) u = exp(-i c x^2/2) u,   D(g) u^ = exp(-i g k^2/2) u^.
// The closed forms are written for mu = 1; a general mu follows from the
// canonical scaling X = sqrt(mu) x, P = p/sqrt(mu): f -> mu f, e -> mu e,
// g -> g / mu.  Every 1 - cos(y) is evaluated as 2 sin^2(y/2) so small steps
// keep full relative accuracy in f and e.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "layout.hpp"

namespace hfgpe {

struct Fge {
    double f, g, e;
    int status;  // 0 or an HFGPE_E_* code
};

// the modulated quantity before the kind's final square root
__host__ __device__ inline double tf_inner(const TFunc &m, double t)
{
    if (m.kind == 2) {
        const double c = cosh(m.freq * (t - m.phase));
        return m.v0 * (1.0 + m.amp * t / (c * c));
    }
    return m.v0 * (1.0 + m.amp * sin(m.freq * t + m.phase));
}

// v(t)
__host__ __device__ inline double tf_value(const TFunc &m, double t)
{
    const double v = tf_inner(m, t);
    return m.kind == 1 ? sqrt(v) : v;
}

// v(t)^2 (for kind 1 without the round trip through the square root)
__host__ __device__ inline double tf_square(const TFunc &m, double t)
{
    const double v = tf_inner(m, t);
    return m.kind == 1 ? v : v * v;
}

// 1 - cos(y)
__host__ __device__ inline double versin(double y)
{
    double s = sin(0.5 * y);
    return 2.0 * s * s;
}

// Lemma 2 (generalised to mu): f = e = mu w tan(w tau / 2), g = sin(w tau)/(mu w),
// valid for |w tau| < pi.
__host__ __device__ inline Fge fge_exact(double mu, double w, double tau)
{
    Fge r{0.0, 0.0, 0.0, 0};
    if (!(w > 0.0)) { r.status = -4; return r; }
    if (!(fabs(w * tau) < M_PI)) { r.status = -3; return r; }
    r.g = sin(w * tau) / (mu * w);
    r.f = mu * w * tan(0.5 * w * tau);
    r.e = r.f;
    return r;
}

// Eq. CommutatorFree (fourth order) with Gauss-Legendre nodes on the stage
// interval, decomposed by Theorem 2.  The factor with omega_R acts first.
__host__ __device__ inline Fge fge_cf4(double mu, const TFunc &om, double t0, double tau)
{
    Fge r{0.0, 0.0, 0.0, 0};
    const double r3 = 1.7320508075688772;  // sqrt(3)
    const double c1 = 0.5 - r3 / 6.0, c2 = 0.5 + r3 / 6.0;
    const double al = 0.5 - 1.0 / r3, be = 1.0 - al;
    double q1 = tf_square(om, t0 + c1 * tau), q2 = tf_square(om, t0 + c2 * tau);
    double qL = al * q1 + be * q2;
    double qR = be * q1 + al * q2;
    if (!(qL > 0.0) || !(qR > 0.0)) { r.status = -4; return r; }
    double wL = sqrt(qL), wR = sqrt(qR);
    double yL = 0.5 * wL * tau, yR = 0.5 * wR * tau;
    double cL = cos(yL), sL = sin(yL), cR = cos(yR), sR = sin(yR);
    double g = sL * cR / wL + cL * sR / wR;
    if (!(g * tau > 0.0)) { r.status = -3; return r; }
    // 1 - cL cR = (1 - cL) + cL (1 - cR)
    double one_m = versin(yL) + cL * versin(yR);
    r.g = g / mu;
    r.f = mu * (one_m + wL / wR * sL * sR) / g;
    r.e = mu * (one_m + wR / wL * sL * sR) / g;
    return r;
}

// Generator of the sixth-order Magnus approximation of Sec. 4.2 on
// [t0, t0 + tau] for mu = 1 (three Gauss nodes on the interval; the printed
// omega_i are squared frequencies): the exponent is
// -i tau/2 (alpha x^2 + beta (xp + px) + gamma p^2).
struct Magnus6 {
    double alpha, beta, gamma;
};

__host__ __device__ inline Magnus6 magnus6_generator(const TFunc &om, double t0, double tau)
{
    const double r15 = 3.872983346207417;  // sqrt(15)
    double w1 = tf_square(om, t0 + (0.5 - r15 / 10.0) * tau);
    double w2 = tf_square(om, t0 + 0.5 * tau);
    double w3 = tf_square(om, t0 + (0.5 + r15 / 10.0) * tau);
    double tt = tau * tau;
    Magnus6 r;
    r.alpha = (5.0 * w1 + 8.0 * w2 + 5.0 * w3) / 18.0 +
              tt / 486.0 * (4.25 * (w1 * w1 + w3 * w3) + 8.0 * w2 * w2 + w1 * w2 + w2 * w3 - 18.5 * w1 * w3);
    r.beta = tau * 1.2909944487358056 /* sqrt(5/3) */ * (w3 - w1) *
             (1.0 / 12.0 + tt / 3240.0 * (5.0 * w1 + 8.0 * w2 + 5.0 * w3));
    r.gamma = 1.0 + tt / 54.0 * (w1 - 2.0 * w2 + w3);
    return r;
}

// Sixth-order Magnus rule decomposed by Theorem 1.
__host__ __device__ inline Fge fge_magnus6(double mu, const TFunc &om, double t0, double tau)
{
    Fge r{0.0, 0.0, 0.0, 0};
    const Magnus6 M = magnus6_generator(om, t0, tau);
    double eta2 = M.alpha * M.gamma - M.beta * M.beta;
    if (!(eta2 > 0.0)) { r.status = -4; return r; }
    double eta = sqrt(eta2);
    double y = eta * tau;
    if (!(fabs(y) < M_PI)) { r.status = -3; return r; }
    double sn = sin(y);
    double g = M.gamma / eta * sn;
    if (!(g * tau > 0.0)) { r.status = -3; return r; }
    double vs = versin(y), bs = M.beta / eta * sn;
    r.g = g / mu;
    r.f = mu * (vs + bs) / g;
    r.e = mu * (vs - bs) / g;
    return r;
}

// Fundamental-matrix rule: the classical flow of the stage (x' = p, p' = -omega^2(t) x
// for mu = 1) as the product of q sixth-order Magnus sub-steps of length tau/q, later
// sub-steps on the left.  Each factor is exp(s G) with G = [[beta, gamma], [-alpha, -beta]],
// G^2 = -eta^2 I, i.e. cos(eta s) I + sin(eta s)/eta G.  Matrices are carried as their
// deviation from I so 1 - S11 and 1 - S22 keep full relative accuracy; the factorisation
// S = K(f) D(g) K(e) gives g = S12, e = (1 - S11)/S12, f = (1 - S22)/S12, then the
// canonical scaling to mu.
__host__ __device__ inline Fge fge_fundamental(double mu, const TFunc &om, double t0, double tau, int q)
{
    Fge r{0.0, 0.0, 0.0, 0};
    const double s = tau / (double)q;
    double X00 = 0.0, X01 = 0.0, X10 = 0.0, X11 = 0.0;  // accumulated S - I
    for (int k = 0; k < q; ++k) {
        const Magnus6 M = magnus6_generator(om, t0 + (double)k * s, s);
        double eta2 = M.alpha * M.gamma - M.beta * M.beta;
        if (!(eta2 > 0.0)) { r.status = -4; return r; }
        double eta = sqrt(eta2);
        double y = eta * s;
        if (!(fabs(y) < M_PI)) { r.status = -3; return r; }
        double sn = sin(y) / eta, cm = -versin(y);
        // deviation of this sub-step's factor
        double A00 = cm + sn * M.beta, A01 = sn * M.gamma, A10 = -sn * M.alpha, A11 = cm - sn * M.beta;
        // (I + A)(I + X) = I + A + X + A X
        double n00 = A00 + X00 + (A00 * X00 + A01 * X10);
        double n01 = A01 + X01 + (A00 * X01 + A01 * X11);
        double n10 = A10 + X10 + (A10 * X00 + A11 * X10);
        double n11 = A11 + X11 + (A10 * X01 + A11 * X11);
        X00 = n00; X01 = n01; X10 = n10; X11 = n11;
    }
    (void)X10;
    const double g = X01;
    if (!(g * tau > 0.0) || !isfinite(g)) { r.status = -3; return r; }
    r.g = g / mu;
    r.e = -mu * X00 / g;
    r.f = -mu * X11 / g;
    return r;
}

// Fourier split (Eq. FourierSplit): the A flow is the free drift over tau, no
// chirps; the harmonic potential is carried by the B phase (see kern_coeff).
__host__ __device__ inline Fge fge_fsplit(double mu, double tau)
{
    Fge r{0.0, tau / mu, 0.0, 0};
    return r;
}

__host__ __device__ inline Fge fge_stage(int rule, double mu, const TFunc &om, double t0, double tau,
                                         int substeps)
{
    switch (rule) {
    case 0: return fge_exact(mu, tf_value(om, t0), tau);
    case 1: return fge_cf4(mu, om, t0, tau);
    case 2: return fge_magnus6(mu, om, t0, tau);
    case 3: return fge_fsplit(mu, tau);
    case 4: return fge_fundamental(mu, om, t0, tau, substeps);
    default: { Fge r{0.0, 0.0, 0.0, -1}; return r; }
    }
}

}  // namespace hfgpe
