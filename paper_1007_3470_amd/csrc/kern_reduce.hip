// kern_reduce.hip -- pointwise FP64 reductions for the norm and the potential
// and interaction energies (Sec. 1: preserved norm; GPE energy).
//
// Grid (n_inst * nblk): block b of instance k sums the strided range
// {b*256 + tid + r*nblk*256} of the instance with a per-thread Neumaier
// accumulator, then the 256 per-thread (sum, carry) pairs are combined in a
// fixed order in LDS.  Partials go to part[(k*nblk + b)*4 + q]; the host adds
// the nblk partials of an instance, again compensated.  No atomics, so the
// result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "coeff.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace hfgpe {

struct Ksum {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double v)
    {
        double t = s + v;
        c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
        s = t;
    }
    __device__ __forceinline__ double val() const { return s + c; }
};

template <typename Store>
__global__ __launch_bounds__(256) void reduce_kernel(const InstDev *__restrict__ insts, int nblk,
                                                     const Store *__restrict__ psi, int energy,
                                                     double t, const void *__restrict__ vi, int vi_f32,
                                                     double *__restrict__ part)
{
    __shared__ double sh[3][256];
    const int inst = blockIdx.x / nblk;
    const int blk = blockIdx.x % nblk;
    const InstDev &I = insts[inst];
    const int nd = I.ndim;
    const int64_t total = (int64_t)I.n[0] * I.n[1] * I.n[2];
    const Store *u = psi + I.offset;
    double hw[3];  // mu omega_j(t)^2 / 2
    for (int j = 0; j < 3; ++j) {
        hw[j] = (j < nd) ? 0.5 * I.mu * tf_square(I.om[j], t) : 0.0;
    }
    const double sig = tf_value(I.sig, t), vm = tf_value(I.vmod, t);
    double wx[3];  // W_xy, W_xz, W_yz at t
    for (int k = 0; k < 3; ++k) wx[k] = I.wx[k] * tf_value(I.wxm[k], t);
    Ksum a, b, c;
    for (int64_t idx = (int64_t)blk * 256 + threadIdx.x; idx < total; idx += (int64_t)nblk * 256) {
        double re = (double)u[idx].x, im = (double)u[idx].y;
        double a2 = fma(re, re, im * im);
        a.add(a2);
        if (energy) {
            int64_t rest = idx;
            double V = 0.0, VI = 1.0, xs[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < nd; ++j) {
                int i = (int)(rest & (I.n[j] - 1));
                rest >>= I.logn[j];
                double x = I.lo[j] + (double)i * I.dx[j];
                xs[j] = x;
                V += hw[j] * x * x;
                VI *= vfactor(I.vf[j], x);
            }
            if (I.coupled)  // off-diagonal part of (mu/2) x^T W x
                V += I.mu * (wx[0] * xs[0] * xs[1] + wx[1] * xs[0] * xs[2] + wx[2] * xs[1] * xs[2]);
            V += vm * (vi ? vi_at(vi, vi_f32, I.offset + idx) : I.eps * VI);
            b.add(V * a2);
            c.add(0.5 * sig * a2 * a2);
        }
    }
    sh[0][threadIdx.x] = a.val();
    sh[1][threadIdx.x] = b.val();
    sh[2][threadIdx.x] = c.val();
    __syncthreads();
    if (threadIdx.x < 3) {
        Ksum r;
        for (int i = 0; i < 256; ++i) r.add(sh[threadIdx.x][i]);
        part[((int64_t)inst * nblk + blk) * 4 + threadIdx.x] = r.val();
    }
    if (threadIdx.x == 3) part[((int64_t)inst * nblk + blk) * 4 + 3] = 0.0;
}

hipError_t launch_reduce_pointwise(const LaunchReduce &L)
{
    if (L.n_inst <= 0) return hipSuccess;
    dim3 grid((unsigned)(L.n_inst * L.nblk));
    if (L.c64)
        hipLaunchKernelGGL(reduce_kernel<float2>, grid, dim3(256), 0, L.stream, L.insts, L.nblk,
                           (const float2 *)L.psi, L.energy, L.t, L.vi, L.vi_f32, L.part);
    else
        hipLaunchKernelGGL(reduce_kernel<double2>, grid, dim3(256), 0, L.stream, L.insts, L.nblk,
                           (const double2 *)L.psi, L.energy, L.t, L.vi, L.vi_f32, L.part);
    return hipGetLastError();
}

}  // namespace hfgpe
