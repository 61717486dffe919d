// kern_coeff.hip -- per (instance, step) stage-coefficient kernels: the
// merged records of every step of a chunk (coeff_step.hpp; separable traps)
// written to the plan's record table, and the coupled-trap records.
#include <hip/hip_runtime.h>

#include "coeff_step.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace hfgpe {

// One instantiation per (HO rule, dimension): the stage loop over axes
// unrolls and the per-axis coefficients stay in registers.  Consecutive
// threads take consecutive steps of an instance, so the first-stage
// coefficients of step n + 1, which the merge at the end of step n needs, are
// taken from the neighbouring thread through LDS (the same values it would
// compute) instead of being evaluated twice.
constexpr int kCoeffThreads = 128;

template <int RULE, int ND>
__global__ __launch_bounds__(kCoeffThreads) void coeff_kernel(const InstDev *__restrict__ insts, int n_inst,
                                                              const SchemeDev *__restrict__ sch,
                                                              Rec *__restrict__ rec, Rec *__restrict__ rec_open,
                                                              double t0, double dt, int64_t step0, int k_steps,
                                                              int64_t nsteps_total, int *err)
{
    __shared__ double first_e[ND][kCoeffThreads];  // e of stage 0 of each thread's step
    const int64_t total = (int64_t)n_inst * k_steps;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = idx < total;
    const int inst = active ? (int)(idx / k_steps) : 0;
    const int s = active ? (int)(idx % k_steps) : 0;
    const int64_t n = step0 + s;
    StepCoeffs<RULE, ND> sc(insts[inst], *sch, t0, dt, n, nsteps_total);
    if (active) sc.first();
#pragma unroll
    for (int j = 0; j < ND; ++j) first_e[j][threadIdx.x] = active ? sc.cur[j].e : 0.0;
    __syncthreads();
    // the neighbour holds step n + 1 of the same instance
    const bool have_next = threadIdx.x + 1 < blockDim.x && idx + 1 < total && s + 1 < k_steps;
    if (!active) return;
    if (n == 0) rec_open[inst] = sc.opening();
    double e_next[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) e_next[j] = have_next ? first_e[j][threadIdx.x + 1] : 0.0;
    Rec *out = rec + ((size_t)inst * k_steps + s) * sch->m;
    sc.records(have_next ? e_next : nullptr, [&](int i, const Rec &r) { out[i] = r; });
    raise_err(err, sc.status);
}

// Coupled trap (non-diagonal W, d >= 2): one record per effective stage (two
// per stage for the commutator-free rule, see coupled_triple), the diagonal of
// G and of the merged chirp matrix in Rec, the off-diagonal entries in RecX.
// Merging as above with matrices: chi = F_k + E_{k+1}; between the two halves
// of a commutator-free stage no B acts (w = 0).  Under the Fourier split the
// chirp is w mu W(tau), the whole harmonic potential of the B flow.
__device__ __forceinline__ void store_mats(int d, const double *G, const double *C, Rec &r, RecX &x)
{
    for (int j = 0; j < 3; ++j) {
        r.g[j] = (j < d) ? G[j * d + j] : 0.0;
        r.chi[j] = (j < d) ? C[j * d + j] : 0.0;
    }
    x.gx[0] = G[1];  // (0,1)
    x.chix[0] = C[1];
    x.gx[1] = (d > 2) ? G[2] : 0.0;  // (0,2)
    x.chix[1] = (d > 2) ? C[2] : 0.0;
    x.gx[2] = (d > 2) ? G[5] : 0.0;  // (1,2)
    x.chix[2] = (d > 2) ? C[5] : 0.0;
}

__global__ void coeff_coupled_kernel(const InstDev *__restrict__ insts, int n_inst,
                                     const SchemeDev *__restrict__ sch, Rec *__restrict__ rec,
                                     Rec *__restrict__ rec_open, RecX *__restrict__ recx,
                                     RecX *__restrict__ recx_open, double t0, double dt, int64_t step0,
                                     int k_steps, int64_t nsteps_total, int *err)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_inst * k_steps) return;
    const int inst = (int)(idx / k_steps);
    const int s = (int)(idx % k_steps);
    const InstDev &I = insts[inst];
    const SchemeDev &S = *sch;
    const int d = I.ndim, m = S.m, me = coupled_stages(S);
    const bool fsplit = S.rule == 3;
    const int64_t n = step0 + s;
    const double tn = t0 + (double)n * dt;
    const double tn1 = t0 + (double)(n + 1) * dt;
    const bool last = (n == nsteps_total - 1);

    // chirp of weight w of the Fourier split's B flow at time t: w mu W(t)
    auto add_harm = [&](double *C, double w, double t) {
        if (!fsplit) return;
        double W[9];
        coupled_wmat(I, d, t, W);
        for (int a = 0; a < d * d; ++a) C[a] += w * I.mu * W[a];
    };

    double F[9], G[9], Fn[9], Gn[9];
    int st = coupled_triple(I, S, dt, tn, 0, F, G);
    raise_err(err, st);
    if (n == 0) {
        Rec o;
        RecX ox;
        double C[9], Z[9];
        for (int a = 0; a < d * d; ++a) { C[a] = F[a]; Z[a] = 0.0; }  // E_0 = F_0
        o.w = dt * S.b[0];
        add_harm(C, o.w, tn);
        o.s = o.w * tf_value(I.sig, tn);
        o.w *= tf_value(I.vmod, tn);
        store_mats(d, Z, C, o, ox);
        rec_open[inst] = o;
        recx_open[inst] = ox;
    }
    Rec *out = rec + ((size_t)inst * k_steps + s) * me;
    RecX *outx = recx + ((size_t)inst * k_steps + s) * me;
    for (int k = 0; k < me; ++k) {
        Rec r;
        RecX x;
        double C[9];
        double w, tau_next;
        const int i = (S.rule == 1) ? (k >> 1) : k;
        const bool half = (S.rule == 1) && ((k & 1) == 0);  // first half of a commutator-free stage
        if (k < me - 1) {
            st = coupled_triple(I, S, dt, tn, k + 1, Fn, Gn);
            raise_err(err, st);
            for (int a = 0; a < d * d; ++a) C[a] = F[a] + Fn[a];  // E_{k+1} = F_{k+1}
            w = half ? 0.0 : dt * S.b[i + 1];
            tau_next = tn + dt * S.cum[i + 1];
        } else if (!last) {
            st = coupled_triple(I, S, dt, tn1, 0, Fn, Gn);
            raise_err(err, st);
            for (int a = 0; a < d * d; ++a) C[a] = F[a] + Fn[a];
            w = dt * (S.b[m] + S.b[0]);
            tau_next = tn1;
        } else {
            for (int a = 0; a < d * d; ++a) C[a] = F[a];
            w = dt * S.b[m];
            tau_next = tn1;
        }
        if (!half) add_harm(C, w, tau_next);
        r.w = half ? 0.0 : w * tf_value(I.vmod, tau_next);
        r.s = half ? 0.0 : w * tf_value(I.sig, tau_next);
        store_mats(d, G, C, r, x);
        bool finite = isfinite(r.w) && isfinite(r.s);
        for (int j = 0; j < 3; ++j)
            finite = finite && isfinite(r.g[j]) && isfinite(r.chi[j]) && isfinite(x.gx[j]) && isfinite(x.chix[j]);
        if (!finite) raise_err(err, -7);
        out[k] = r;
        outx[k] = x;
        for (int a = 0; a < d * d; ++a) { F[a] = Fn[a]; G[a] = Gn[a]; }
    }
}

template <int RULE, int ND>
static hipError_t launch_coeff_t(const LaunchCoeff &L, unsigned grid, int bs)
{
    hipLaunchKernelGGL((coeff_kernel<RULE, ND>), dim3(grid), dim3(bs), 0, L.stream, L.insts, L.n_inst, L.scheme,
                       L.rec, L.rec_open, L.t0, L.dt, L.step0, L.k_steps, L.nsteps_total, L.err);
    return hipGetLastError();
}

template <int RULE>
static hipError_t launch_coeff_nd(const LaunchCoeff &L, unsigned grid, int bs)
{
    switch (L.ndim) {
    case 1: return launch_coeff_t<RULE, 1>(L, grid, bs);
    case 2: return launch_coeff_t<RULE, 2>(L, grid, bs);
    case 3: return launch_coeff_t<RULE, 3>(L, grid, bs);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_coeff_rule(const LaunchCoeff &L, unsigned grid, int bs)
{
    switch (L.rule) {
    case 0: return launch_coeff_nd<0>(L, grid, bs);
    case 1: return launch_coeff_nd<1>(L, grid, bs);
    case 2: return launch_coeff_nd<2>(L, grid, bs);
    case 3: return launch_coeff_nd<3>(L, grid, bs);
    case 4: return launch_coeff_nd<4>(L, grid, bs);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_coeff(const LaunchCoeff &L)
{
    int64_t total = (int64_t)L.n_inst * L.k_steps;
    if (total <= 0) return hipSuccess;
    const int bs = kCoeffThreads;
    int64_t grid = (total + bs - 1) / bs;
    if (L.recx) {
        hipLaunchKernelGGL(coeff_coupled_kernel, dim3((unsigned)grid), dim3(bs), 0, L.stream, L.insts, L.n_inst,
                           L.scheme, L.rec, L.rec_open, L.recx, L.recx_open, L.t0, L.dt, L.step0, L.k_steps,
                           L.nsteps_total, L.err);
        return hipGetLastError();
    }
    return launch_coeff_rule(L, (unsigned)grid, bs);
}

}  // namespace hfgpe
