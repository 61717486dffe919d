// kern_nd.hip -- 2-D / 3-D Hermite-Fourier axis passes for gfx950: launch
// dispatch, the runtime-shaped pass instances and the kinetic-energy kernel.
// The pass kernel itself and the d-D design are in nd_pass.hpp; passes along
// axes of 128 .. 1024 points (other than the opening pass of an evolve call)
// run the fixed-shape instances of kern_nd_fix.hip (separable) and
// kern_nd_fix_coupled.hip (coupled-trap kinds).
#include <hip/hip_runtime.h>

#include "nd_pass.hpp"

namespace hfgpe {

// Kinetic-energy partial sums along one axis: for every pencil along `axis`,
// sum_k k_j^2 |FFT_j(u)|^2 / N_j; block b of instance k writes part[k*nblk + b].
template <typename Store, int P, int MAXS>
__global__ __launch_bounds__(kThreadsND) void kin_nd_kernel(const InstDev *__restrict__ insts, int nblk,
                                                            const Store *__restrict__ psi, NdShape sh, int axis,
                                                            double *__restrict__ part)
{
    constexpr int LOGP = Log2<P>::value;
    constexpr int LDS_ELEMS = kThreadsND * P + ((kThreadsND * P) >> kPadShift);
    __shared__ double2 lds[LDS_ELEMS];
    __shared__ double red[2][kThreadsND];
    const int inst = blockIdx.x / nblk, blk = blockIdx.x % nblk;
    const InstDev &I = insts[inst];
    const int lnj = sh.logn[axis], nj = 1 << lnj;
    const int logT = lnj - LOGP, T = 1 << logT;
    const int ltot = sh.logn[0] + sh.logn[1] + sh.logn[2];
    const int64_t npencil = (int64_t)1 << (ltot - lnj);
    int lG = 8 - logT;
    if ((int64_t)1 << lG > npencil) lG = ltot - lnj;
    const int G = 1 << lG;
    const int tid = threadIdx.x;
    const int slot = tid >> logT, tl = tid & (T - 1);
    const bool active = slot < G;
    int lstride = 0;
    for (int j = 0; j < axis; ++j) lstride += sh.logn[j];
    Fft1D<double2, P, MAXS> fft;
    fft.init(lnj, tl, lds + slot * (nj + (nj >> kPadShift)));
    double s = 0.0, cc = 0.0;
    const Store *u0 = psi + I.offset;
    for (int64_t g = blk; g < (npencil >> lG); g += nblk) {
        const int64_t p = (g << lG) + slot;  // pencil index: (outer, inner) flattened
        const int64_t inner = p & (((int64_t)1 << lstride) - 1), outer = p >> lstride;
        const int64_t base = outer * ((int64_t)nj << lstride) + inner;
        double2 u[P];
#pragma unroll
        for (int c = 0; c < P; ++c)
            u[c] = active ? to_d2(u0[base + ((int64_t)(tl + c * T) << lstride)]) : make_double2(0.0, 0.0);
        fft.template run<-1>(u);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            int q = tl + c * T;
            int sq = q - ((2 * q >= nj) ? nj : 0);
            double k = I.kscale[axis] * (double)sq;
            double v = k * k * fma(u[c].x, u[c].x, u[c].y * u[c].y) / (double)nj;
            double t = s + v;
            cc += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
            s = t;
        }
        __syncthreads();
    }
    red[0][tid] = s;
    red[1][tid] = cc;
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, ac = 0.0;
        for (int i = 0; i < kThreadsND; ++i) {
            double v = red[0][i] + red[1][i];
            double t = a + v;
            ac += (fabs(a) >= fabs(v)) ? ((a - t) + v) : ((v - t) + a);
            a = t;
        }
        part[(int64_t)inst * nblk + blk] = a + ac;
    }
}

// log2 of the pencils per group of an axis pass: tpb/T pencils, limited by the
// pencils available (x) or by the contiguous run of x positions (strided axes).
int nd_group_log(const int *n, int axis, int tpb)
{
    int logn[3], ltot = 0, lstride = 0;
    for (int j = 0; j < 3; ++j) {
        logn[j] = 0;
        while ((1 << logn[j]) < n[j]) ++logn[j];
        ltot += logn[j];
        if (j < axis) lstride += logn[j];
    }
    int P = points_per_thread_nd(n[axis]);
    int lp = 0;
    while ((1 << lp) < P) ++lp;
    int logT = logn[axis] - lp;
    int ltpb = 0;
    while ((1 << ltpb) < tpb) ++ltpb;
    int lG = ltpb - logT;
    if (axis == 0) {
        if (lG > ltot - logn[axis]) lG = ltot - logn[axis];
    } else if (lG > lstride) {
        lG = lstride;
    }
    return lG;
}

// Threads per workgroup of an axis pass.  A c64 strided axis whose 256-thread
// group holds fewer than 8 pencils moves rows of under 64 bytes per access;
// there a 512-thread group doubles the row length.  At 64 bytes and above the
// two co-resident 256-thread groups (one loading while the other computes) are
// faster than one 512-thread group with 128-byte rows.
int nd_threads(const int *n, int axis, int c64)
{
    if (axis == 0 || !c64 || points_per_thread_nd(n[axis]) != 8) return kThreadsND;
    const int lg256 = nd_group_log(n, axis, kThreadsND);
    return (lg256 < 3 && nd_group_log(n, axis, 512) > lg256) ? 512 : kThreadsND;
}

template <typename Store, int P, int MAXS, int MODE>
static hipError_t launch_pass_mode(const LaunchND &L)
{
    switch (L.kind) {
    case kPassSep:
        if constexpr (P == 8 && sizeof(Store) == 8) {
            if (nd_pass_threads(L) == 512) return launch_pass_tpb<Store, P, MAXS, MODE, 512, kPassSep, 0>(L);
        }
        return launch_pass_tpb<Store, P, MAXS, MODE, kThreadsND, kPassSep, 0>(L);
    case kPassFwd:
        if constexpr (MODE != 1) return launch_pass_tpb<Store, P, MAXS, MODE, kThreadsND, kPassFwd, 0>(L);
        return hipErrorInvalidValue;
    case kPassMid:
        if constexpr (MODE == 0) return launch_pass_tpb<Store, P, MAXS, MODE, kThreadsND, kPassMid, 0>(L);
        return hipErrorInvalidValue;
    case kPassInv:
        if constexpr (MODE != 2) return launch_pass_tpb<Store, P, MAXS, MODE, kThreadsND, kPassInv, 0>(L);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename Store, int P, int MAXS>
static hipError_t launch_pass_p(const LaunchND &L)
{
    // an evolve call opens on the first pass of axis 0 and closes every stage
    // on its last pass; with d >= 2 these never fall on the same pass
    if (L.apply_open && L.apply_close) return hipErrorInvalidValue;
    if (L.apply_close) return launch_pass_mode<Store, P, MAXS, 1>(L);
    if (L.apply_open) return launch_pass_mode<Store, P, MAXS, 2>(L);
    return launch_pass_mode<Store, P, MAXS, 0>(L);
}

template <typename Store>
static hipError_t launch_pass_store(const LaunchND &L)
{
    switch (points_per_thread_nd(L.n[L.axis])) {
    case 1: return launch_pass_p<Store, 1, 1>(L);
    case 2: return launch_pass_p<Store, 2, 1>(L);
    case 4: return launch_pass_p<Store, 4, 1>(L);
    // axes up to 512 points need at most 3 radix passes: the smaller register
    // file of the MAXS = 3 instance leaves the drift-only passes spill-free
    case 8: return L.n[L.axis] <= 512 ? launch_pass_p<Store, 8, 3>(L) : launch_pass_p<Store, 8, 4>(L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_nd_pass(const LaunchND &L)
{
    if (L.n_inst <= 0) return hipSuccess;
    if (!L.generic && !L.apply_open && nd_fixed_shape(L.n, L.axis, nd_pass_threads(L))) {
        if (L.kind == kPassSep) return launch_nd_pass_fixed(L);
        return launch_nd_pass_fixed_coupled(L);
    }
    return L.c64 ? launch_pass_store<float2>(L) : launch_pass_store<double2>(L);
}

// Threads per workgroup of a pass: 512 only for separable c64 passes along a
// strided axis with 8 points per thread whose 512-thread group holds more
// pencils than a 256-thread one -- by default where nd_threads selects it, or
// as a tuned choice (L.tpb); 256 otherwise.
int nd_pass_threads(const LaunchND &L)
{
    if (L.kind != kPassSep || !L.c64) return kThreadsND;
    if (L.tpb == kThreadsND) return kThreadsND;
    if (L.tpb == 512 && L.axis > 0 && points_per_thread_nd(L.n[L.axis]) == 8 &&
        nd_group_log(L.n, L.axis, 512) > nd_group_log(L.n, L.axis, kThreadsND))
        return 512;
    return nd_threads(L.n, L.axis, 1);
}

// A pass runs a fixed-shape instance when its axis has 128 .. 1024 points and
// a tpb-thread workgroup holds its full complement of pencils (every thread
// busy).
bool nd_fixed_shape(const int *n, int axis, int tpb)
{
    const int na = n[axis];
    if (na < 128 || na > 1024 || (na & (na - 1)) != 0) return false;
    int logn = 0, ltpb = 0;
    while ((1 << logn) < na) ++logn;
    while ((1 << ltpb) < tpb) ++ltpb;
    return nd_group_log(n, axis, tpb) == ltpb - (logn - 3);
}

template <typename Store, int P, int MAXS>
static hipError_t launch_kin_p(const LaunchND &L, int nblk, double *part)
{
    hipLaunchKernelGGL((kin_nd_kernel<Store, P, MAXS>), dim3(L.n_inst * nblk), dim3(kThreadsND), 0, L.stream,
                       L.insts, nblk, (const Store *)L.psi, make_shape(L), L.axis, part);
    return hipGetLastError();
}

template <typename Store>
static hipError_t launch_kin_store(const LaunchND &L, int nblk, double *part)
{
    switch (points_per_thread_nd(L.n[L.axis])) {
    case 1: return launch_kin_p<Store, 1, 1>(L, nblk, part);
    case 2: return launch_kin_p<Store, 2, 1>(L, nblk, part);
    case 4: return launch_kin_p<Store, 4, 1>(L, nblk, part);
    case 8: return launch_kin_p<Store, 8, 4>(L, nblk, part);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kinetic_nd(const LaunchND &L, int nblk, double *part)
{
    if (L.n_inst <= 0) return hipSuccess;
    return L.c64 ? launch_kin_store<float2>(L, nblk, part) : launch_kin_store<double2>(L, nblk, part);
}

__global__ void advance_base_kernel(int *base, int by) { *base += by; }
__global__ void set_base_kernel(int *base, int v) { *base = v; }

hipError_t launch_set_base(int *base, int v, hipStream_t s)
{
    hipLaunchKernelGGL(set_base_kernel, dim3(1), dim3(1), 0, s, base, v);
    return hipGetLastError();
}

hipError_t launch_advance_base(int *base, int by, hipStream_t s)
{
    hipLaunchKernelGGL(advance_base_kernel, dim3(1), dim3(1), 0, s, base, by);
    return hipGetLastError();
}

int points_per_thread_nd(int n)
{
    if (n <= 1) return 1;
    if (n <= 4) return n;
    if (n <= 2048) return 8;
    return 0;
}

}  // namespace hfgpe
