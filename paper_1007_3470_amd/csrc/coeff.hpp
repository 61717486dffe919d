// coeff.hpp -- stage coefficients (f, g, e) of the harmonic-oscillator part
// by the closed forms of Lemma 2 and Theorems 1-2, in FP64, usable on the
// host (hfgpe_stage_coeffs, plan validation) and in the coefficient kernel.
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

__host__ __device__ inline double sinmod(const SinMod &m, double t)
{
    return m.v0 * (1.0 + m.amp * sin(m.freq * t + m.phase));
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
__host__ __device__ inline Fge fge_cf4(double mu, const SinMod &om, double t0, double tau)
{
    Fge r{0.0, 0.0, 0.0, 0};
    const double r3 = 1.7320508075688772;  // sqrt(3)
    const double c1 = 0.5 - r3 / 6.0, c2 = 0.5 + r3 / 6.0;
    const double al = 0.5 - 1.0 / r3, be = 1.0 - al;
    double w1 = sinmod(om, t0 + c1 * tau), w2 = sinmod(om, t0 + c2 * tau);
    double qL = al * w1 * w1 + be * w2 * w2;
    double qR = be * w1 * w1 + al * w2 * w2;
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

// Sixth-order Magnus approximation of Sec. 4.2 (three Gauss nodes on the stage
// interval; the printed omega_i are squared frequencies), exponent
// -i tau/2 (alpha x^2 + beta (xp + px) + gamma p^2), decomposed by Theorem 1.
__host__ __device__ inline Fge fge_magnus6(double mu, const SinMod &om, double t0, double tau)
{
    Fge r{0.0, 0.0, 0.0, 0};
    const double r15 = 3.872983346207417;  // sqrt(15)
    double a1 = sinmod(om, t0 + (0.5 - r15 / 10.0) * tau);
    double a2 = sinmod(om, t0 + 0.5 * tau);
    double a3 = sinmod(om, t0 + (0.5 + r15 / 10.0) * tau);
    double w1 = a1 * a1, w2 = a2 * a2, w3 = a3 * a3;
    double tt = tau * tau;
    double alpha = (5.0 * w1 + 8.0 * w2 + 5.0 * w3) / 18.0 +
                   tt / 486.0 * (4.25 * (w1 * w1 + w3 * w3) + 8.0 * w2 * w2 + w1 * w2 + w2 * w3 - 18.5 * w1 * w3);
    double beta = tau * 1.2909944487358056 /* sqrt(5/3) */ * (w3 - w1) *
                  (1.0 / 12.0 + tt / 3240.0 * (5.0 * w1 + 8.0 * w2 + 5.0 * w3));
    double gamma = 1.0 + tt / 54.0 * (w1 - 2.0 * w2 + w3);
    double eta2 = alpha * gamma - beta * beta;
    if (!(eta2 > 0.0)) { r.status = -4; return r; }
    double eta = sqrt(eta2);
    double y = eta * tau;
    if (!(fabs(y) < M_PI)) { r.status = -3; return r; }
    double sn = sin(y);
    double g = gamma / eta * sn;
    if (!(g * tau > 0.0)) { r.status = -3; return r; }
    double vs = versin(y), bs = beta / eta * sn;
    r.g = g / mu;
    r.f = mu * (vs + bs) / g;
    r.e = mu * (vs - bs) / g;
    return r;
}

// Fourier split (Eq. FourierSplit): the A flow is the free drift over tau, no
// chirps; the harmonic potential is carried by the B phase (see kern_coeff).
__host__ __device__ inline Fge fge_fsplit(double mu, double tau)
{
    Fge r{0.0, tau / mu, 0.0, 0};
    return r;
}

__host__ __device__ inline Fge fge_stage(int rule, double mu, const SinMod &om, double t0, double tau)
{
    switch (rule) {
    case 0: return fge_exact(mu, om.v0, tau);
    case 1: return fge_cf4(mu, om, t0, tau);
    case 2: return fge_magnus6(mu, om, t0, tau);
    case 3: return fge_fsplit(mu, tau);
    default: { Fge r{0.0, 0.0, 0.0, -1}; return r; }
    }
}

}  // namespace hfgpe
