// kern_1d.hip -- resident 1-D Hermite-Fourier step kernel for gfx950.
//
// One workgroup of 256 threads owns `count` same-size instances for K time
// steps (K up to a whole evolve call): the state is loaded from HBM once, kept
// in FP64 registers, advanced K steps and stored once.  Per stage (Sec. 3,
// Eq. leapfrogHF / prod-genHarmOsc):
//   forward FFT  ->  drift D(g) = exp(-i g k^2/2) (and 1/N)  ->  inverse FFT
//   ->  merged x-space phase exp(-i (chi x^2/2 + w eps V_I + s |u|^2))
// The FFT is a Stockham auto-sort FFT split over the T = N/P threads of an
// instance: every pass is a radix-P butterfly on P registers (the first pass
// may use a smaller radix), with an LDS exchange between passes.  Thread t
// holds the points {t + c T, c = 0..P-1} both before the first pass and after
// the last one, so the drift, the x-phase and the step boundary need no data
// movement.  Twiddles of passes 1.. are computed once per launch (sincospi of
// exact dyadic angles) and stay in registers; phases use the FP64 cis_neg.
// Storage: Store = float2 (c64) or double2 (c128) in HBM; Xch = the LDS
// exchange type (FP64 for both).  Arithmetic is FP64 throughout.
#include <hip/hip_runtime.h>

#include "devmath.hpp"
#include "fft_lds.hpp"
#include "hf1d_fixed.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace hfgpe {

template <typename Store, typename Xch, int P, int MAXS>
__global__ __launch_bounds__(kThreads1D, (P <= 8 ? 2 : 1)) void hf1d_kernel(const Item1D *__restrict__ items,
                                                          const int *__restrict__ perm,
                                                          const InstDev *__restrict__ insts,
                                                          const Rec *__restrict__ rec,
                                                          const Rec *__restrict__ rec_open,
                                                          const double2 *__restrict__ cistab,
                                                          const void *__restrict__ vi, int vi_f32,
                                                          Store *__restrict__ psi, int m, int K,
                                                          int rec_steps, int step_base,
                                                          int apply_opening)
{
    constexpr int LOGP = Log2<P>::value;
    constexpr int LDS_ELEMS = kThreads1D * P + ((kThreads1D * P) >> kPadShift);
    __shared__ Xch lds[LDS_ELEMS];
    __shared__ CisTable ctab;
    __shared__ double vel[kThreads1D * P];  // eps V_I at every point of the group
    load_cis_table(&ctab, cistab);

    const Item1D it = items[blockIdx.x];
    const int logn = it.logn;
    const int N = 1 << logn;
    const int logT = logn - LOGP;
    const int T = 1 << logT;
    const int tid = threadIdx.x;
    const int slot = tid >> logT;
    const int tl = tid & (T - 1);
    const bool active = slot < it.count;
    const int inst_id = perm[it.first + (active ? slot : 0)];
    const InstDev &I = insts[inst_id];

    Fft1D<Xch, P, MAXS> fft;
    fft.init(logn, tl, lds + slot * (N + (N >> kPadShift)));

    double2 u[P];
    const double lo = I.lo[0], dx = I.dx[0], eps = I.eps;
    const VFac vf = I.vf[0];
    Store *base = psi + I.offset;
    double *ve = vel + slot * N;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int i = tl + c * T;
        double x = lo + (double)i * dx;
        ve[i] = vi ? vi_at(vi, vi_f32, I.offset + i) : eps * vfactor(vf, x);
        u[c] = active ? to_d2(base[i]) : make_double2(0.0, 0.0);
    }
    __syncthreads();  // cis table in LDS

    auto xphase = [&](const Rec &r) {
        const double chi = r.chi[0], w = r.w, s = r.s;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            double x = lo + (double)(tl + c * T) * dx;
            double a2 = fma(u[c].x, u[c].x, u[c].y * u[c].y);
            double th = fma(chi, 0.5 * x * x, fma(w, ve[tl + c * T], s * a2));
            u[c] = cmul(u[c], cis_neg_tab(th, ctab));
        }
    };

    const double invN = 1.0 / (double)N;
    const double ks = I.kscale[0];
    if (apply_opening) xphase(rec_open[inst_id]);
    const Rec *rp = rec + ((size_t)inst_id * (size_t)rec_steps + (size_t)step_base) * (size_t)m;
    for (int step = 0; step < K; ++step) {
        for (int st = 0; st < m; ++st) {
            const Rec r = rp[step * m + st];
            fft.template run<-1>(u);
            const double g = r.g[0];
#pragma unroll
            for (int c = 0; c < P; ++c) {
                int q = tl + c * T;
                int sq = q - ((2 * q >= N) ? N : 0);
                double k = ks * (double)sq;
                double2 f = cis_neg_tab(g * (0.5 * k * k), ctab);
                u[c] = cmul(u[c], make_double2(f.x * invN, f.y * invN));
            }
            fft.template run<+1>(u);
            xphase(r);
        }
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < P; ++c) base[tl + c * T] = from_d2<Store>(u[c]);
    }
}

// Kinetic energy of 1-D instances: sum_k k^2 |u^_k|^2 / (2 mu N), forward FFT
// in LDS with FP64 exchange, per-thread compensated sums combined in a fixed
// order by the first thread of each instance slot.
template <typename Store, int P, int MAXS>
__global__ __launch_bounds__(kThreads1D) void kin1d_kernel(const Item1D *__restrict__ items,
                                                           const int *__restrict__ perm,
                                                           const InstDev *__restrict__ insts,
                                                           const Store *__restrict__ psi,
                                                           double *__restrict__ kin)
{
    constexpr int LOGP = Log2<P>::value;
    constexpr int LDS_ELEMS = kThreads1D * P + ((kThreads1D * P) >> kPadShift);
    __shared__ double2 lds[LDS_ELEMS];
    __shared__ double part[2][kThreads1D];

    const Item1D it = items[blockIdx.x];
    const int logn = it.logn;
    const int N = 1 << logn;
    const int logT = logn - LOGP;
    const int T = 1 << logT;
    const int tid = threadIdx.x;
    const int slot = tid >> logT;
    const int tl = tid & (T - 1);
    const bool active = slot < it.count;
    const int inst_id = perm[it.first + (active ? slot : 0)];
    const InstDev &I = insts[inst_id];

    Fft1D<double2, P, MAXS> fft;
    fft.init(logn, tl, lds + slot * (N + (N >> kPadShift)));
    double2 u[P];
    const Store *base = psi + I.offset;
#pragma unroll
    for (int c = 0; c < P; ++c) u[c] = active ? to_d2(base[tl + c * T]) : make_double2(0.0, 0.0);
    fft.template run<-1>(u);
    double s = 0.0, cc = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int q = tl + c * T;
        int sq = q - ((2 * q >= N) ? N : 0);
        double k = I.kscale[0] * (double)sq;
        double v = k * k * fma(u[c].x, u[c].x, u[c].y * u[c].y);
        double t = s + v;
        cc += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
        s = t;
    }
    part[0][tid] = s;
    part[1][tid] = cc;
    __syncthreads();
    if (active && tl == 0) {
        double a = 0.0, ac = 0.0;
        for (int i = 0; i < T; ++i) {
            double v = part[0][tid + i] + part[1][tid + i];
            double t = a + v;
            ac += (fabs(a) >= fabs(v)) ? ((a - t) + v) : ((v - t) + a);
            a = t;
        }
        kin[inst_id] = (a + ac) / (2.0 * I.mu * (double)N);
    }
}

template <typename Store, int P, int MAXS>
static hipError_t launch_kin_p(const LaunchKin1D &L)
{
    hipLaunchKernelGGL((kin1d_kernel<Store, P, MAXS>), dim3(L.n_items), dim3(kThreads1D), 0, L.stream,
                       L.items, L.perm, L.insts, (const Store *)L.psi, L.kin);
    return hipGetLastError();
}

template <typename Store>
static hipError_t launch_kin_store(const LaunchKin1D &L)
{
    switch (L.P) {
    case 1: return launch_kin_p<Store, 1, 1>(L);
    case 2: return launch_kin_p<Store, 2, 1>(L);
    case 4: return launch_kin_p<Store, 4, 1>(L);
    case 8: return launch_kin_p<Store, 8, 4>(L);
    case 16: return launch_kin_p<Store, 16, 3>(L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kinetic_1d(const LaunchKin1D &L)
{
    if (L.n_items <= 0) return hipSuccess;
    if (L.c64) return launch_kin_store<float2>(L);
    return launch_kin_store<double2>(L);
}

template <typename Store, typename Xch, int P, int MAXS>
static hipError_t launch_p(const Launch1D &L)
{
    hipLaunchKernelGGL((hf1d_kernel<Store, Xch, P, MAXS>), dim3(L.n_items), dim3(kThreads1D), 0, L.stream,
                       L.items, L.perm, L.insts, L.rec, L.rec_open, L.cistab, L.vi, L.vi_f32, (Store *)L.psi, L.m, L.K,
                       L.rec_steps, L.step_base, L.apply_opening);
    return hipGetLastError();
}

template <typename Store, typename Xch>
static hipError_t launch_store(const Launch1D &L)
{
    if (L.fixed) {
        if (L.P != 8) return hipErrorInvalidValue;
        if (L.coef_rule >= 0) return launch_hf1d_fused(L);  // kern_1d_fused.hip
        return launch_hf1d_fixed<Store, -1>(L);
    }
    if (L.coef_rule >= 0) return hipErrorInvalidValue;  // in-kernel records: fixed shapes only
    switch (L.P) {
    case 1: return launch_p<Store, Xch, 1, 1>(L);
    case 2: return launch_p<Store, Xch, 2, 1>(L);
    case 4: return launch_p<Store, Xch, 4, 1>(L);
    case 8: return launch_p<Store, Xch, 8, 4>(L);
    case 16: return launch_p<Store, Xch, 16, 3>(L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hf1d(const Launch1D &L)
{
    if (L.n_items <= 0) return hipSuccess;
    // The LDS exchange is FP64 for both storage types: rounding the exchanged
    // values to FP32 costs conversions on every pass and, over thousands of
    // steps of a strongly nonlinear instance, pushes the c64 error past 5e-5.
    if (L.c64) return launch_store<float2, double2>(L);
    return launch_store<double2, double2>(L);
}

bool fixed_shape_1d(int n) { return n >= 64 && n <= 2048; }

int points_per_thread_1d(int n)
{
    if (n <= 1) return 1;
    if (n <= 4) return n;
    if (n <= 2048) return 8;
    if (n == 4096) return 16;
    return 0;
}

}  // namespace hfgpe
