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
    // a constant form: v0 exactly, as v0 (1 + 0 * ...) would give, without the
    // transcendental
    if (m.amp == 0.0) return m.v0;
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

// The rules below take omega(t) as any type with tf_square(om, t) and
// tf_value(om, t) found by argument-dependent lookup: the instance's TFunc
// forms on the device, or a caller's host function of t.

// Eq. CommutatorFree (fourth order) with Gauss-Legendre nodes on the stage
// interval, decomposed by Theorem 2.  The factor with omega_R acts first.
template <class Om>
__host__ __device__ inline Fge fge_cf4(double mu, const Om &om, double t0, double tau)
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
    double cL, sL, cR, sR;
    sincos(yL, &sL, &cL);
    sincos(yR, &sR, &cR);
    double g = sL * cR / wL + cL * sR / wR;
    if (!(g * tau > 0.0)) { r.status = -3; return r; }
    // 1 - cL cR = (1 - cL) + cL (1 - cR), with 1 - cos y = sin^2 y / (1 + cos y):
    // no cancellation while 1 + cos y stays away from 0, which holds for the
    // half-stage angles |y| < pi/2 of every stage the plan's validation accepts
    double one_m = sL * sL / (1.0 + cL) + cL * (sR * sR / (1.0 + cR));
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

template <class Om>
__host__ __device__ inline Magnus6 magnus6_generator(const Om &om, double t0, double tau)
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
template <class Om>
__host__ __device__ inline Fge fge_magnus6(double mu, const Om &om, double t0, double tau)
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
template <class Om>
__host__ __device__ inline Fge fge_fundamental(double mu, const Om &om, double t0, double tau, int q)
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

// The rule as a compile-time constant (the coefficient kernel is instantiated
// per rule, so no other rule's code shares its register allocation).
template <int RULE, class Om>
__host__ __device__ inline Fge fge_stage_t(double mu, const Om &om, double t0, double tau, int substeps)
{
    if constexpr (RULE == 0) return fge_exact(mu, tf_value(om, t0), tau);
    if constexpr (RULE == 1) return fge_cf4(mu, om, t0, tau);
    if constexpr (RULE == 2) return fge_magnus6(mu, om, t0, tau);
    if constexpr (RULE == 3) return fge_fsplit(mu, tau);
    if constexpr (RULE == 4) return fge_fundamental(mu, om, t0, tau, substeps);
    Fge r{0.0, 0.0, 0.0, -1};
    return r;
}

template <class Om>
__host__ __device__ inline Fge fge_stage(int rule, double mu, const Om &om, double t0, double tau, int substeps)
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

// ---------------------------------------------------------------------------
// Coupled trap: H0 = p^2/(2 mu) + (mu/2) x^T W x with a symmetric d x d W
// (d <= 3, row-major).  For a constant W the flow is, per normal mode w_k of
// W = Q diag(w_k^2) Q^T, the flow of Lemma 2, so it factors as K(F) D(G) K(E)
// with F = E = Q diag(mu w_k tan(w_k tau/2)) Q^T and G = Q diag(sin(w_k tau)/(mu w_k)) Q^T.
// ---------------------------------------------------------------------------

// cyclic Jacobi eigen-decomposition of a symmetric d x d matrix (A is overwritten)
__host__ __device__ inline void jacobi_eig(int d, double *A, double *lam, double *Q)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Q[i * d + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < d; ++i) {
            diag += A[i * d + i] * A[i * d + i];
            for (int j = i + 1; j < d; ++j) off += A[i * d + j] * A[i * d + j];
        }
        if (!(off > 1e-34 * diag)) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                const double apq = A[p * d + q];
                if (apq == 0.0) continue;
                const double th = (A[q * d + q] - A[p * d + p]) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < d; ++k) {
                    const double akp = A[k * d + p], akq = A[k * d + q];
                    A[k * d + p] = c * akp - sn * akq;
                    A[k * d + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {
                    const double apk = A[p * d + k], aqk = A[q * d + k];
                    A[p * d + k] = c * apk - sn * aqk;
                    A[q * d + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < d; ++k) {
                    const double qkp = Q[k * d + p], qkq = Q[k * d + q];
                    Q[k * d + p] = c * qkp - sn * qkq;
                    Q[k * d + q] = sn * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < d; ++i) lam[i] = A[i * d + i];
}

// F (= E) and G of the exact constant-W flow over tau; 0, -3 (|w tau| >= pi for
// some mode) or -4 (W not positive definite)
__host__ __device__ inline int coupled_exact(int d, const double *W, double mu, double tau, double *F, double *G)
{
    double A[9], lam[3], Q[9], f[3], g[3];
    for (int k = 0; k < d * d; ++k) A[k] = W[k];
    jacobi_eig(d, A, lam, Q);
    for (int k = 0; k < d; ++k) {
        if (!(lam[k] > 0.0)) return -4;
        const double w = sqrt(lam[k]);
        if (!(fabs(w * tau) < M_PI)) return -3;
        f[k] = mu * w * tan(0.5 * w * tau);
        g[k] = sin(w * tau) / (mu * w);
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double a = 0.0, b = 0.0;
            for (int k = 0; k < d; ++k) {
                const double qq = Q[i * d + k] * Q[j * d + k];
                a += qq * f[k];
                b += qq * g[k];
            }
            F[i * d + j] = a;
            G[i * d + j] = b;
        }
    return 0;
}

// W(t) of instance I (d x d)
__host__ __device__ inline void coupled_wmat(const InstDev &I, int d, double t, double *W)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            if (i == j) {
                W[i * d + j] = tf_square(I.om[i], t);
            } else {
                const int a = i < j ? i : j, b = i < j ? j : i;
                const int k = a + b - 1;  // (0,1) -> 0, (0,2) -> 1, (1,2) -> 2
                W[i * d + j] = I.wx[k] * tf_value(I.wxm[k], t);
            }
        }
}

// Factor triple number k of the step starting at tn for a coupled trap, as it
// acts: exact (rule 0) one triple per stage; the commutator-free rule (1) two
// triples per stage, the flow of W_R over half the stage then that of W_L (the
// product of the two leaves the K(F) D(G) K(E) family for d >= 2); the Fourier
// split (3) the free drift G = a_i dt / mu I with no chirps.  E = F except for
// the Fourier split (both zero).  Returns 0 or a status code.
__host__ __device__ inline int coupled_triple(const InstDev &I, const SchemeDev &S, double dt, double tn, int k,
                                              double *F, double *G)
{
    const int d = I.ndim;
    const int i = (S.rule == 1) ? (k >> 1) : k;
    const double t0 = tn + dt * S.cum[i];
    const double len = dt * S.a[i];
    if (S.rule == 3) {
        for (int a = 0; a < d * d; ++a) { F[a] = 0.0; G[a] = 0.0; }
        for (int a = 0; a < d; ++a) G[a * d + a] = len / I.mu;
        return 0;
    }
    double W[9];
    if (S.rule == 0) {
        coupled_wmat(I, d, t0, W);
        return coupled_exact(d, W, I.mu, len, F, G);
    }
    if (S.rule == 1) {
        const double r3 = 1.7320508075688772;
        const double c1 = 0.5 - r3 / 6.0, c2 = 0.5 + r3 / 6.0;
        const double al = 0.5 - 1.0 / r3, be = 1.0 - al;
        double W1[9], W2[9];
        coupled_wmat(I, d, t0 + c1 * len, W1);
        coupled_wmat(I, d, t0 + c2 * len, W2);
        const bool right = (k & 1) == 0;  // W_R acts first
        for (int a = 0; a < d * d; ++a) W[a] = right ? (be * W1[a] + al * W2[a]) : (al * W1[a] + be * W2[a]);
        return coupled_exact(d, W, I.mu, 0.5 * len, F, G);
    }
    return -1;
}

// effective stages per step of a coupled plan
__host__ __device__ inline int coupled_stages(const SchemeDev &S) { return S.rule == 1 ? 2 * S.m : S.m; }

}  // namespace hfgpe
