// coeff_step.hpp -- the merged per-stage records of one time step of one
// instance (separable trap), shared by the coefficient kernel, which writes
// them to a record table in HBM, and the resident 1-D step kernel, which
// evaluates them in LDS for blocks of steps.
//
// For step n the stages run over [tau_i, tau_i + a_i dt] with
// tau_i = t_n + dt (a_0 + ... + a_{i-1}) (time frozen in B as in Table
// "algorithm").  Record i holds the stage's drift coefficient g_i and the
// x-space phase applied after it, in which adjacent chirps and B flows are
// merged (Eq. leapfrogHF, Eq. prod-genHarmOsc):
//   inside a step:          chi = f_i + e_{i+1},  w = dt b_{i+1} at tau_{i+1}
//   across a step boundary: chi = f_{m-1} + e'_0, w = dt (b_m + b_0) at t_{n+1}
//   after the last step:    chi = f_{m-1},        w = dt b_m at t_{n+1}
// and s = w sigma(tau).  Under the Fourier split (no chirps) chi is instead
// w mu omega_j(tau)^2, the harmonic potential of the B flow.  The opening
// phase of an evolve call (chi = e_0(t_0), w = dt b_0 at t_0) is the record
// `open`.  w finally takes the time factor m(tau) of eps V_I.
#pragma once
#include <hip/hip_runtime.h>

#include "coeff.hpp"
#include "layout.hpp"

namespace hfgpe {

template <int RULE, int ND>
struct StepCoeffs {
    const InstDev &I;
    const SchemeDev &S;
    double dt, tn, tn1;
    bool last;   // step n is the evolve call's last
    Fge cur[ND];  // (f, g, e) of the stage being merged; stage 0 after first()
    int status = 0;

    __device__ __forceinline__ StepCoeffs(const InstDev &I_, const SchemeDev &S_, double t0, double dt_, int64_t n,
                                          int64_t nsteps_total)
        : I(I_), S(S_), dt(dt_), tn(t0 + (double)n * dt_), tn1(t0 + (double)(n + 1) * dt_),
          last(n == nsteps_total - 1)
    {
    }

    __device__ __forceinline__ void keep(const Fge &q) { status = status ? status : q.status; }

    // stage 0 of step n
    __device__ __forceinline__ void first()
    {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            cur[j] = fge_stage_t<RULE>(I.mu, I.om[j], tn, dt * S.a[0], S.substeps);
            keep(cur[j]);
        }
    }

    // the opening record of an evolve call (step n = 0); after first()
    __device__ __forceinline__ Rec opening() const
    {
        Rec o;
#pragma unroll
        for (int j = 0; j < 3; ++j) { o.g[j] = 0.0; o.chi[j] = 0.0; }
#pragma unroll
        for (int j = 0; j < ND; ++j) o.chi[j] = cur[j].e;
        o.w = dt * S.b[0];
        o.s = o.w * tf_value(I.sig, tn);
        if constexpr (RULE == 3) {
#pragma unroll
            for (int j = 0; j < ND; ++j) o.chi[j] += o.w * I.mu * tf_square(I.om[j], tn);
        }
        o.w *= tf_value(I.vmod, tn);  // eps V_I(x, t) = m(t) eps V_I(x)
        return o;
    }

    // Records 0 .. m-1 of step n, after first(), each passed to emit(i, rec).
    // e_next: the ND values e of stage 0 of step n + 1 when the caller has
    // them (the same values this function would evaluate), else null.
    template <class Emit>
    __device__ __forceinline__ void records(const double *e_next, Emit &&emit)
    {
        const int m = S.m;
        for (int i = 0; i < m; ++i) {
            Rec r;
            double fprev[ND];
#pragma unroll
            for (int j = 0; j < 3; ++j) { r.g[j] = 0.0; r.chi[j] = 0.0; }
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                r.g[j] = cur[j].g;
                fprev[j] = cur[j].f;
            }
            double tau_next;
            if (i < m - 1) {
                tau_next = tn + dt * S.cum[i + 1];
#pragma unroll
                for (int j = 0; j < ND; ++j) {
                    cur[j] = fge_stage_t<RULE>(I.mu, I.om[j], tau_next, dt * S.a[i + 1], S.substeps);
                    keep(cur[j]);
                    r.chi[j] = fprev[j] + cur[j].e;
                }
                r.w = dt * S.b[i + 1];
            } else if (!last) {
                tau_next = tn1;
#pragma unroll
                for (int j = 0; j < ND; ++j) {
                    double en;
                    if (e_next) {
                        en = e_next[j];
                    } else {
                        const Fge q = fge_stage_t<RULE>(I.mu, I.om[j], tn1, dt * S.a[0], S.substeps);
                        keep(q);
                        en = q.e;
                    }
                    r.chi[j] = fprev[j] + en;
                }
                r.w = dt * (S.b[m] + S.b[0]);
            } else {
                tau_next = tn1;
#pragma unroll
                for (int j = 0; j < ND; ++j) r.chi[j] = fprev[j];
                r.w = dt * S.b[m];
            }
            r.s = r.w * tf_value(I.sig, tau_next);
            if constexpr (RULE == 3) {  // Fourier split: the harmonic potential is part of B
#pragma unroll
                for (int j = 0; j < ND; ++j) r.chi[j] += r.w * I.mu * tf_square(I.om[j], tau_next);
            }
            r.w *= tf_value(I.vmod, tau_next);
            bool finite = isfinite(r.w) && isfinite(r.s);
#pragma unroll
            for (int j = 0; j < 3; ++j) finite = finite && isfinite(r.g[j]) && isfinite(r.chi[j]);
            if (!finite && !status) status = -7;
            emit(i, r);
        }
    }
};

__device__ __forceinline__ void raise_err(int *err, int code)
{
    if (code != 0) atomicCAS(err, 0, code);
}

}  // namespace hfgpe
