// hf1d_fixed.hpp -- the resident 1-D step kernel for 64 <= N <= 2048 with the
// FFT shape fixed at compile time (FftFix8, 8 points per thread): one body per
// grid size, selected per workgroup, so LDS addresses and index arithmetic
// are constants.  Per stage (Sec. 3, Eq. leapfrogHF / prod-genHarmOsc):
//   forward FFT  ->  drift D(g) = exp(-i g k^2/2) (and 1/N)  ->  inverse FFT
//   ->  merged x-space phase exp(-i (chi x^2/2 + w eps V_I + s |u|^2))
// The stage records come either from the plan's record table in HBM (RULE <
// 0; written by the coefficient kernel or from a host callback) or are
// evaluated inside the kernel (RULE = the plan's HO rule): the workgroup
// evaluates the records of a block of steps of its instances into LDS, one
// step per thread, with the same arithmetic as the coefficient kernel
// (coeff_step.hpp), then advances its instances through the block.
#pragma once
#include <hip/hip_runtime.h>

#include "coeff_step.hpp"
#include "devmath.hpp"
#include "fft_lds.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace hfgpe {

// FFT exchange buffer of a workgroup: 256 threads x 8 points, one padding
// element in 8.  Two of them with records from the table: the passes
// alternate between the two, which takes one barrier per pass instead of two
// (two workgroups per CU still fit the 160 KB of LDS: 72 KB of buffers and the
// 6 KB phase table each).  One with in-kernel records, whose 17 KB of record
// blocks would otherwise leave room for one workgroup per CU.
constexpr int kLds1D = kThreads1D * 8 + ((kThreads1D * 8) >> kPadShift);
template <int RULE>
constexpr int nbuf_1d() { return RULE < 0 ? 2 : 1; }

// the part of a stage record a 1-D step uses
struct Rec1 {
    double g, chi, w, s;
};
// records of one in-kernel block: a block covers kRecLds1D / (count m) steps
constexpr int kRecLds1D = 512;

struct Coef1D {
    const SchemeDev *sch;
    double t0, dt;
    int64_t step0;         // global index of the chunk's first step
    int64_t nsteps_total;  // steps of the evolve call
    int *err;
};

// The records of the chunk's steps s0 + s (s < kb) of the group's `count`
// instances into crec[(j kb + s) m + i], one step per thread, and the opening
// record of instance slot j into copen[j] when global step 0 is among them.
// Kept out of line: the step loop's register allocation does not see this
// code.
template <int RULE>
__device__ __noinline__ void eval_records_1d(int first, int count, const int *__restrict__ perm,
                                             const InstDev *__restrict__ insts, const SchemeDev &S,
                                             const Coef1D &ci, int s0, int kb, Rec1 *crec, Rec1 *copen)
{
    const int m = S.m;
    for (int task = threadIdx.x; task < count * kb; task += kThreads1D) {
        const int j = task / kb, s = task - j * kb;
        const int64_t n = ci.step0 + s0 + s;
        StepCoeffs<RULE, 1> sc(insts[perm[first + j]], S, ci.t0, ci.dt, n, ci.nsteps_total);
        sc.first();
        if (n == 0) {
            const Rec o = sc.opening();
            copen[j] = Rec1{0.0, o.chi[0], o.w, o.s};
        }
        Rec1 *dst = crec + (j * kb + s) * m;
        sc.records(nullptr, [&](int i, const Rec &r) { dst[i] = Rec1{r.g[0], r.chi[0], r.w, r.s}; });
        raise_err(ci.err, sc.status);
    }
}

template <typename Store, int LOGN, int RULE>
__device__ __forceinline__ void hf1d_fixed_body(const Item1D &it, const int *__restrict__ perm,
                                                const InstDev *__restrict__ insts, const Rec *__restrict__ rec,
                                                const Rec *__restrict__ rec_open, const CisTable &ctab,
                                                const void *__restrict__ vi, int vi_f32, double2 *lds,
                                                Rec1 *crec, Rec1 *copen, const SchemeDev &S, const Coef1D &ci,
                                                Store *__restrict__ psi, int m,
                                                int K, int rec_steps, int step_base, int apply_opening)
{
    using F = FftFix8<LOGN, double2, nbuf_1d<RULE>(), kLds1D>;
    constexpr int P = 8, N = F::N, T = F::T;
    const int tid = threadIdx.x;
    const int slot = tid >> F::LOGT;
    const int tl = tid & (T - 1);
    const bool active = slot < it.count;
    const int rslot = active ? slot : 0;
    const int inst_id = perm[it.first + rslot];
    const InstDev &I = insts[inst_id];

    F fft;
    fft.init(tl, slot, lds);

    double2 u[P];
    const double lo = I.lo[0], dx = I.dx[0], eps = I.eps;
    const VFac vf = I.vf[0];
    Store *base = psi + I.offset;
    double ve[P];  // eps V_I at the thread's points, in registers
#pragma unroll
    for (int c = 0; c < P; ++c) {
        const int i = tl + c * T;
        const double x = lo + (double)i * dx;
        ve[c] = vi ? vi_at(vi, vi_f32, I.offset + i) : eps * vfactor(vf, x);
        u[c] = active ? to_d2(base[i]) : make_double2(0.0, 0.0);
    }
    __syncthreads();  // cis table in LDS

    auto xphase = [&](double chi, double w, double s) {
        double th[P];
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const double x = lo + (double)(tl + c * T) * dx;
            const double a2 = fma(u[c].x, u[c].x, u[c].y * u[c].y);
            th[c] = fma(chi, 0.5 * x * x, fma(w, ve[c], s * a2));
        }
        cis_apply_batch<P>(u, th, ctab);
    };

    constexpr double invN = 1.0 / (double)N;
    const double ks = I.kscale[0];
    // Drift D(g) and 1/N at the thread's points q = tl + c'T, c' = 0..3 and
    // -4..-1 (the upper half of the points are the negative wavenumbers):
    // the angle al (tl + c'T)^2, al = g ks^2/2, is quadratic in c', so three
    // table evaluations -- at c' = 0, its first difference towards c' = 1
    // and the second difference 2 al T^2 -- give the eight factors by
    // products, stepping outwards from c' = 0 in both directions.
    const double tl2 = (double)(tl * tl), dfwd = (double)(2 * tl * T + T * T);
    constexpr double d2 = 2.0 * (double)T * (double)T;
    auto drift = [&](double g) {
        const double al = g * (0.5 * ks * ks);
        const double ang[3] = {al * tl2, al * dfwd, al * d2};
        double2 f[3];
        cis_batch<3>(ang, f, ctab);
        const double2 f0 = make_double2(f[0].x * invN, f[0].y * invN);
        const double2 Q = f[2];
        double2 D = f[1];         // angle step c' -> c' + 1 at c' = 0
        double2 E = cmulc(Q, D);  // angle step c' -> c' - 1 at c' = 0: al (T^2 - 2 tl T)
        double2 fp = f0, fm = f0;
        u[0] = cmul(u[0], f0);
#pragma unroll
        for (int c = 1; c < P / 2; ++c) {
            fp = cmul(fp, D);
            u[c] = cmul(u[c], fp);
            if (c + 1 < P / 2) D = cmul(D, Q);
        }
#pragma unroll
        for (int c = P - 1; c >= P / 2; --c) {
            fm = cmul(fm, E);
            u[c] = cmul(u[c], fm);
            if (c > P / 2) E = cmul(E, Q);
        }
    };
    // the forward transform starts in exchange buffer 0, the inverse in the
    // buffer the forward's last pass did not read, and the next stage's
    // forward in buffer 0 again (the park area of the in-kernel records)
    constexpr int kInvStart = F::next_start(0);
    static_assert(F::next_start(kInvStart) == 0, "exchange buffers");
    auto stage = [&](double g, double chi, double w, double s) {
        fft.template run<-1, 0>(u);
        drift(g);
        fft.template run<+1, kInvStart>(u);
        xphase(chi, w, s);
    };

    if constexpr (RULE < 0) {
        if (apply_opening) {
            const Rec &o = rec_open[inst_id];
            xphase(o.chi[0], o.w, o.s);
        }
        const Rec *rp = rec + ((size_t)inst_id * (size_t)rec_steps + (size_t)step_base) * (size_t)m;
        for (int step = 0; step < K; ++step) {
            for (int st = 0; st < m; ++st) {
                const Rec r = rp[step * m + st];
                stage(r.g[0], r.chi[0], r.w, r.s);
            }
        }
    } else {
        const int B = kRecLds1D / (it.count * m);  // >= 1: count <= 32, m <= 16
        // the state is parked in the FFT exchange buffer (free between steps)
        // while the records are evaluated, so the registers of the state are
        // free for that code
        double2 *park = lds + slot * F::ROW + tl;
        for (int b0 = 0; b0 < K; b0 += B) {
            const int kb = min(B, K - b0);
#pragma unroll
            for (int c = 0; c < P; ++c) park[c * F::TP] = u[c];
            __syncthreads();  // the previous block's records are consumed
            eval_records_1d<RULE>(it.first, it.count, perm, insts, S, ci, step_base + b0, kb, crec, copen);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = park[c * F::TP];
            __syncthreads();  // every parked value is read before a first pass overwrites the buffer
            if (b0 == 0 && apply_opening) {
                const Rec1 o = copen[rslot];
                xphase(o.chi, o.w, o.s);
            }
            const Rec1 *rp = crec + rslot * kb * m;
            for (int step = 0; step < kb; ++step) {
                for (int st = 0; st < m; ++st) {
                    const Rec1 r = rp[step * m + st];
                    stage(r.g, r.chi, r.w, r.s);
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < P; ++c) base[tl + c * T] = from_d2<Store>(u[c]);
    }
}

template <typename Store, int RULE>
__global__ __launch_bounds__(kThreads1D, 2) void hf1d_fixed_kernel(const Item1D *__restrict__ items,
                                                                const int *__restrict__ perm,
                                                                const InstDev *__restrict__ insts,
                                                                const Rec *__restrict__ rec,
                                                                const Rec *__restrict__ rec_open,
                                                                const double2 *__restrict__ cistab,
                                                                const void *__restrict__ vi, int vi_f32,
                                                                Coef1D ci, Store *__restrict__ psi, int m, int K,
                                                                int rec_steps, int step_base, int apply_opening)
{
    constexpr int NREC = (RULE < 0) ? 1 : kRecLds1D;
    constexpr int NOPEN = (RULE < 0) ? 1 : kThreads1D / 8;
    __shared__ double2 lds[nbuf_1d<RULE>() * kLds1D];
    __shared__ CisTable ctab;
    __shared__ Rec1 crec[NREC];
    __shared__ Rec1 copen[NOPEN];
    // the scheme in LDS: the record phases read it after a barrier each time
    // instead of keeping its values in registers across the steps
    __shared__ SchemeDev sch[(RULE < 0) ? 1 : 1];
    if constexpr (RULE >= 0) {
        constexpr int W = (int)(sizeof(SchemeDev) / sizeof(int));
        static_assert(sizeof(SchemeDev) % sizeof(int) == 0, "scheme copy");
        for (int i = threadIdx.x; i < W; i += kThreads1D)
            reinterpret_cast<int *>(sch)[i] = reinterpret_cast<const int *>(ci.sch)[i];
    }
    load_cis_table(&ctab, cistab);
    const Item1D it = items[blockIdx.x];
#define HFGPE_1D_BODY(LG)                                                                                         \
    hf1d_fixed_body<Store, LG, RULE>(it, perm, insts, rec, rec_open, ctab, vi, vi_f32, lds, crec, copen, sch[0], ci, \
                                     psi, m, K, rec_steps, step_base, apply_opening)
    switch (it.logn) {
    case 6: HFGPE_1D_BODY(6); break;
    case 7: HFGPE_1D_BODY(7); break;
    case 8: HFGPE_1D_BODY(8); break;
    case 9: HFGPE_1D_BODY(9); break;
    case 10: HFGPE_1D_BODY(10); break;
    case 11: HFGPE_1D_BODY(11); break;
    default: break;  // the launcher sends only 64 <= N <= 2048 here
    }
#undef HFGPE_1D_BODY
}

template <typename Store, int RULE>
hipError_t launch_hf1d_fixed(const Launch1D &L)
{
    const Coef1D ci{L.scheme, L.t0, L.dt, L.step0, L.nsteps_total, L.err};
    hipLaunchKernelGGL((hf1d_fixed_kernel<Store, RULE>), dim3(L.n_items), dim3(kThreads1D), 0, L.stream, L.items,
                       L.perm, L.insts, L.rec, L.rec_open, L.cistab, L.vi, L.vi_f32, ci, (Store *)L.psi, L.m, L.K,
                       L.rec_steps, L.step_base, L.apply_opening);
    return hipGetLastError();
}

}  // namespace hfgpe
