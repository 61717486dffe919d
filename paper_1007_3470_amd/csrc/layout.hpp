// layout.hpp -- device-side data layout shared by the host runtime and the
// kernels: per-instance descriptors, per-stage coefficient records and work
// items.  All floating-point fields are FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace hfgpe {

constexpr int kMaxStages = 16;

// A time-dependent coefficient (omega_j or sigma); kind 0: v = v0 (1 + amp sin(freq t + phase));
// 1: v^2 = v0 (1 + amp sin(freq t + phase)); 2: v = v0 (1 + amp t / cosh^2(freq (t - phase))).
struct TFunc {
    double v0, amp, freq, phase;
    int kind;
    int pad_;
};

struct VFac {
    double c0, c2, c4, gs, k, phi;  // (c0 + c2 x^2 + c4 x^4) exp(-x^2/gs) cos(k x + phi)
};

// One instance as the kernels see it.
struct InstDev {
    int64_t offset;  // first complex element in the packed buffer
    int ndim;
    int n[3];
    int logn[3];
    int pad_;
    double lo[3];
    double dx[3];
    double kscale[3];  // 2 pi / L_j
    double mu;
    double eps;
    TFunc om[3];
    TFunc sig;
    VFac vf[3];
    double wx[3];  // coupled trap: W_xy, W_xz, W_yz of (mu/2) x^T W x, times wxm
    int coupled;   // 1 when some wx used by the grid's axes is non-zero
    int pad2_;
    TFunc vmod;    // time factor of eps V_I (v0 = 1; amp = 0: constant 1)
    TFunc wxm[3];  // time factors of W_xy, W_xz, W_yz (v0 = 1)
};

// The pointwise x-space phase applied after stage i of a step:
//   u <- exp(-i (sum_j chi_j x_j^2/2 + w eps V_I(x) + s |u|^2)) u
// (chi merges the closing chirp f_i with the next opening chirp e_{i+1};
// w = dt * b (merged B weight); s = w * sigma(tau)), and the kinetic
// coefficient g_j of the stage's drift.  64 bytes.
struct Rec {
    double g[3];
    double chi[3];
    double w;
    double s;
};

// Off-diagonal entries (xy, xz, yz) of the drift matrix G and of the merged
// chirp matrix of a coupled trap, beside the Rec of the same stage.
struct RecX {
    double gx[3];
    double chix[3];
};

// Composition in device-friendly form (Eq. prod-gen; b has m+1 weights;
// cum[i] = a_0 + ... + a_{i-1}, the stage-start offsets within a step).
struct SchemeDev {
    int m;
    int rule;
    int ndim;
    int substeps;  // Magnus sub-steps per stage of the fundamental-matrix rule
    double a[kMaxStages];
    double b[kMaxStages + 1];
    double cum[kMaxStages + 1];
};

// A group of `count` same-size 1-D instances processed by one workgroup.
struct Item1D {
    int first;  // index into the plan's instance permutation
    int count;
    int logn;
    int pad_;
};

// eps V_I at element k of a caller's array held in FP64 (f32 = 0) or FP32.
__host__ __device__ inline double vi_at(const void *vi, int f32, int64_t k)
{
    return f32 ? (double)static_cast<const float *>(vi)[k] : static_cast<const double *>(vi)[k];
}

__host__ __device__ inline double vfactor(const VFac &v, double x)
{
    double x2 = x * x;
    double poly = v.c0 + x2 * (v.c2 + x2 * v.c4);
    double gauss = (v.gs > 0.0) ? exp(-x2 / v.gs) : 1.0;
    return poly * gauss * cos(v.k * x + v.phi);
}

}  // namespace hfgpe
