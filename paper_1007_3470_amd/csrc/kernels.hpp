// kernels.hpp -- host-side launchers of the gfx950 kernels (one per .hip file).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace hfgpe {

// ---- coefficient kernel (kern_coeff.hip) ---------------------------------
struct LaunchCoeff {
    const InstDev *insts;
    int n_inst;
    const SchemeDev *scheme;  // device copy
    Rec *rec;                 // [n_inst][k_steps][m] (coupled trap: m effective stages)
    Rec *rec_open;            // [n_inst]
    RecX *recx;               // coupled trap: off-diagonal parts, same layout; else null
    RecX *recx_open;
    double t0, dt;
    int64_t step0;            // global index of the chunk's first step
    int k_steps;              // steps in this chunk
    int64_t nsteps_total;     // steps of the whole evolve call
    int *err;                 // device error word
    int rule;                 // HO rule of the scheme (selects the kernel instance)
    int ndim;
    hipStream_t stream;
};
hipError_t launch_coeff(const LaunchCoeff &L);

// ---- 1-D resident step kernel (kern_1d.hip) ------------------------------
struct Launch1D {
    const Item1D *items;
    int n_items;
    int P;      // points per thread of this item group
    int fixed;  // 1: every item has 64 <= N <= 2048 (fixed-shape kernel)
    const int *perm;
    const InstDev *insts;
    const Rec *rec;
    const Rec *rec_open;
    const double2 *cistab;  // the phase table (CisTable layout), 16-byte words
    const void *vi;         // caller's eps V_I per point (state layout), or null
    int vi_f32;             // 1: vi holds floats, 0: doubles
    void *psi;
    int m;
    int K;            // steps advanced by this launch
    int rec_steps;    // steps per instance held in rec (row stride)
    int step_base;    // first step of this launch within rec
    int apply_opening;
    int c64;
    // in-kernel stage records (fixed shapes): coef_rule = the HO rule; -1 =
    // records from rec / rec_open
    int coef_rule;
    const SchemeDev *scheme;  // device copy
    double t0, dt;
    int64_t step0;            // global index of the chunk's first step
    int64_t nsteps_total;     // steps of the evolve call
    int *err;                 // device error word
    hipStream_t stream;
};
hipError_t launch_hf1d(const Launch1D &L);
hipError_t launch_hf1d_fused(const Launch1D &L);  // coef_rule >= 0, fixed shapes
int points_per_thread_1d(int n);
bool fixed_shape_1d(int n);

// ---- observables (kern_reduce.hip) ----------------------------------------
// Per-instance partial sums written to part[(inst * nblk + blk) * 4 + q] as
// (sum |u|^2, sum V |u|^2, sum sigma/2 |u|^4, unused).
struct LaunchReduce {
    const InstDev *insts;
    int n_inst;
    int nblk;          // blocks per instance
    const void *psi;
    int c64;
    int energy;        // 0: only |u|^2
    double t;          // time for omega(t), sigma(t)
    const void *vi;    // caller's eps V_I per point, or null (factor form)
    int vi_f32;        // 1: vi holds floats, 0: doubles
    double *part;
    hipStream_t stream;
};
hipError_t launch_reduce_pointwise(const LaunchReduce &L);

// Kinetic energy of 1-D instances: kin[inst] = sum_k k^2 |u^_k|^2 / (2 mu N)
// (times the cell size on the host).
struct LaunchKin1D {
    const Item1D *items;
    int n_items;
    int P;
    const int *perm;
    const InstDev *insts;
    const void *psi;
    int c64;
    double *kin;  // [n_inst]
    hipStream_t stream;
};
hipError_t launch_kinetic_1d(const LaunchKin1D &L);

// ---- d-D axis passes (kern_nd.hip) ----------------------------------------
// All instances of a d-D plan share the grid shape n[].
struct LaunchND {
    const InstDev *insts;
    int n_inst;
    const Rec *rec;
    const Rec *rec_open;
    const RecX *recx;       // coupled trap: off-diagonal G and chirp entries, else null
    const RecX *recx_open;
    int kind;               // 0 separable stage pass, 1 forward only, 2 forward + whole drift + inverse, 3 inverse only
    const void *vi;         // caller's eps V_I per point (state layout), or null
    int vi_f32;             // 1: vi holds floats, 0: doubles
    const double *vtab;  // [n_inst][3][vtab_stride]: V_I factor of each axis on its grid
    int vtab_stride;
    const double2 *cistab;
    const double2 *twtab;  // exp(-2 pi i q / 2^twlog), q < 2^twlog
    int twlog;
    void *psi;
    int c64;
    int ndim;
    int n[3];
    int axis, stage, m, rec_steps, step;
    const int *step_base;  // device int added to step (graph replay), or null
    int apply_open, apply_close;
    int grid;     // persistent workgroups; 0: as many as the device holds at once for the pass's kernel
    int n_cu;     // compute units of the device
    int generic;  // 1: runtime-shaped FFT for every axis length
    int per_cu;   // with grid = 0: workgroups per CU (capped by what fits); 0: the default policy
    int tpb;      // threads per group, 256 or 512 (c64 separable strided passes only); 0: default
    hipStream_t stream;
};
hipError_t launch_nd_pass(const LaunchND &L);
// fixed-shape passes for the shapes nd_fixed_shape accepts: separable
// (kern_nd_fix.hip) and coupled-trap kinds (kern_nd_fix_coupled.hip)
int nd_pass_threads(const LaunchND &L);
bool nd_fixed_shape(const int *n, int axis, int tpb);
hipError_t launch_nd_pass_fixed(const LaunchND &L);
hipError_t launch_nd_pass_fixed_coupled(const LaunchND &L);
// Kinetic energy partials along L.axis: part[inst * nblk + b].
hipError_t launch_kinetic_nd(const LaunchND &L, int nblk, double *part);
int points_per_thread_nd(int n);
int nd_group_log(const int *n, int axis, int tpb);
int nd_threads(const int *n, int axis, int c64);
// one-thread kernels that set / advance the device-side step base of a graph
hipError_t launch_set_base(int *base, int v, hipStream_t s);
hipError_t launch_advance_base(int *base, int by, hipStream_t s);

}  // namespace hfgpe
