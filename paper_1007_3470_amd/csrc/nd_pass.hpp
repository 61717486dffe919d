// nd_pass.hpp -- the 2-D / 3-D axis-pass kernel template, shared by the
// runtime-shaped instances (kern_nd.hip) and the fixed-shape ones
// (kern_nd_fix.hip).
//
// The d-D drift D(g) = F^-1 exp(-i sum_j g_j k_j^2/2) F factors into one 1-D
// drift per axis (the kinetic phase is separable and the per-axis transforms
// commute), so a stage is d axis passes, each one HBM read and one HBM write
// of the state:
//   pass j: load pencils along axis j  [opening x-phase on the first pass of
//           an evolve call]  ->  FFT_j  ->  exp(-i g_j k_j^2/2)/N_j  ->
//           FFT_j^-1  [merged closing x-phase on the last axis]  ->  store.
// Workgroups are persistent over groups of G pencils.  Along x the G pencils
// are consecutive rows and a pencil's points are consecutive lanes; along a
// strided axis the G pencils are G consecutive x positions, lanes run over
// the pencils first (coalesced rows of G elements) and LDS is interleaved by
// pencil.  The drift factors of a thread's P wavenumbers are computed once per
// (workgroup, instance) and reused for every pencil it processes.
//
// A coupled trap (off-diagonal W) has a full quadratic drift k^T G k / 2 that
// no longer factors per axis.  A stage is then 2d - 1 passes: forward
// transforms along the axes 0 .. d-2, one pass along the last axis that
// transforms forward, applies the whole drift (the other wavenumbers are fixed
// along a pencil) and transforms back, then inverse transforms along
// d-2 .. 0, the last of which applies the merged closing x-phase.  The x-phase
// carries the off-diagonal chirp terms along a pencil as a linear term in the
// pass coordinate.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>

#include "devmath.hpp"
#include "fft_lds.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace hfgpe {

constexpr int kThreadsND = 256;
constexpr int kMaxAxisND = 1024;  // longest axis of a d-D plan

struct NdShape {
    int ndim;
    int n[3];
    int logn[3];
};

// KIND of pass: separable stage along one axis, or (coupled trap) forward
// transform only, forward + whole drift + inverse, inverse transform only.
enum { kPassSep = 0, kPassFwd = 1, kPassMid = 2, kPassInv = 3 };

// MODE: 0 = no x-phase, 1 = closing x-phase at the end of the pass, 2 = opening
// x-phase at its start (separate instantiations keep unused phase code out of
// the register allocation).
// FFT of a pass: the runtime-shaped Fft1D (FIX = 0), or for FIX = 2 LOGN + s a
// fixed-shape radix-8 FFT of 2^LOGN points, on padded rows (s = 0, axis 0) or
// interleaved pencils (s = 1, strided axes, TPB / (N/8) pencils per group).
template <typename Xch, int P, int MAXS, int FIX, int TPB, bool = (FIX != 0), bool = ((FIX & 1) != 0)>
struct NdFft {
    using type = Fft1D<Xch, P, MAXS>;
};
template <typename Xch, int P, int MAXS, int FIX, int TPB>
struct NdFft<Xch, P, MAXS, FIX, TPB, true, false> {
    using type = FftFix8<(FIX >> 1), Xch>;
};
template <typename Xch, int P, int MAXS, int FIX, int TPB>
struct NdFft<Xch, P, MAXS, FIX, TPB, true, true> {
    using type = FftFixS8<(FIX >> 1), (TPB >> ((FIX >> 1) - 3)), Xch>;
};

// LDS exchange type of a pass.  The c64 passes round the state to c64 at
// every HBM store anyway; exchanging FP32 between the FFT's radix passes adds
// a few such roundings per pass (arithmetic, twiddles and phase factors stay
// FP64) and halves the LDS bytes of passes whose time is spent in exchanges.
// The c128 passes exchange FP64.
template <typename Store>
struct NdXch {
#ifdef HFGPE_ND_XCH64
    using type = double2;
#else
    using type = Store;
#endif
};

template <typename Store, int P, int MAXS, int MODE, int TPB, int KIND, int FIX>
__global__ __launch_bounds__(TPB, (TPB <= 256 ? 2 : 1)) void hfnd_pass_kernel(
    const InstDev *__restrict__ insts, int n_inst, const Rec *__restrict__ rec,
    const Rec *__restrict__ rec_open, const RecX *__restrict__ recx, const RecX *__restrict__ recx_open,
    const void *__restrict__ vi, int vi_f32, const double *__restrict__ vtab, int vtab_stride,
    const double2 *__restrict__ cistab, const double2 *__restrict__ twtab, int twlog,
    Store *__restrict__ psi, NdShape sh, int axis, int lG, int stage, int m, int rec_steps, int step_off,
    const int *__restrict__ step_base)
{
    // step within the coefficient records: a fixed offset, plus a device-side
    // base when the launch is replayed from a captured graph
    const int step = step_off + (step_base ? *step_base : 0);
    constexpr int LOGP = Log2<P>::value;
    // fixed shape: axis length 2^FLOGN, layout (padded rows / interleaved) and
    // pencils per group known at compile time
    constexpr int FLOGN = FIX >> 1;
    constexpr bool FSTRIDED = (FIX & 1) != 0;
    static_assert(FIX == 0 || P == 8, "fixed-shape passes are radix 8");
    constexpr int LDS_ELEMS = (FIX != 0 && FSTRIDED) ? TPB * P : TPB * P + ((TPB * P) >> kPadShift);
    using Xch = typename NdXch<Store>::type;
    __shared__ Xch lds[LDS_ELEMS];
    __shared__ CisTable ctab;
    constexpr int kAxisTab = FIX ? (1 << FLOGN) : kMaxAxisND;
    __shared__ double2 kfl[kAxisTab];  // drift factor of every wavenumber of the axis
    // passes with an x-phase: (x_i, V_I factor at x_i) of every point of the axis
    __shared__ double2 xvt[MODE != 0 ? kAxisTab : 1];
    load_cis_table(&ctab, cistab);
    __syncthreads();

    const int lnj = FIX ? FLOGN : sh.logn[axis];
    const bool xaxis = FIX ? !FSTRIDED : (axis == 0);
    const int nj = 1 << lnj;
    const int logT = lnj - LOGP;
    const int T = 1 << logT;
    int lstride = 0;
    for (int j = 0; j < axis; ++j) lstride += sh.logn[j];
    const int ltot = sh.logn[0] + sh.logn[1] + sh.logn[2];
    const int64_t npencil = (int64_t)1 << (ltot - lnj);
    // G = 2^lg pencils per group; the block has exactly G * T threads
    const int lg = FIX ? Log2<TPB>::value - (FLOGN - LOGP) : lG;
    const int G = 1 << lg;
    const int64_t gpi = npencil >> lg;  // groups per instance
    const int tid = threadIdx.x;
    int slot, tl;
    typename NdFft<Xch, P, MAXS, FIX, TPB>::type fft;
    if (xaxis) {
        slot = tid >> logT;
        tl = tid & (T - 1);
    } else {
        slot = tid & (G - 1);
        tl = tid >> lg;
    }
    if constexpr (FIX == 0) {
        fft.istride = xaxis ? 1 : G;
        fft.pad = xaxis;
        fft.init(lnj, tl, lds + (xaxis ? slot * (nj + (nj >> kPadShift)) : slot), twtab, twlog);
    } else {
        fft.init(tl, slot, lds, twtab, twlog);
    }

    const double invN = 1.0 / (double)nj;
    int kf_inst = -1;

    // each workgroup takes a contiguous range of groups (the drift factors change
    // only when the instance does; neighbouring pencils share cache lines).
    // Strided axes whose group rows are shorter than a 128-byte line: two
    // workgroups on the same XCD (ids b and b + 8; workgroups are dispatched to
    // the 8 XCDs round robin) share one range and take its even and odd groups
    // in step, so both halves of every line are requested together and the
    // second is served by that XCD's L2 instead of a second HBM read.
    const int64_t total = (int64_t)n_inst * gpi;
    const bool paired = !xaxis && G * (int)sizeof(Store) < 128 && (gridDim.x & 15) == 0 && total > 1;
    int64_t j_begin, j_end, gmul, goff;
    if (paired) {
        const int b = blockIdx.x, k = b >> 3;
        const int64_t pair = ((int64_t)(k >> 1) << 3) | (b & 7);
        const int64_t total2 = (total + 1) >> 1, npairs = gridDim.x >> 1;
        const int64_t per2 = (total2 + npairs - 1) / npairs;
        j_begin = pair * per2;
        j_end = (pair + 1) * per2 < total2 ? (pair + 1) * per2 : total2;
        gmul = 2;
        goff = k & 1;
    } else {
        const int64_t per = (total + gridDim.x - 1) / gridDim.x;
        j_begin = blockIdx.x * per;
        j_end = (blockIdx.x + 1) * per < total ? (blockIdx.x + 1) * per : total;
        gmul = 1;
        goff = 0;
    }
    // group of range position j (past the last group for the odd half of an odd total)
    auto group_of = [&](int64_t j) { return j * gmul + goff; };
    const int estr = xaxis ? 1 : (1 << lstride);
    // Element (tl + c T) estr of this thread's pencil in group gq sits at
    // ubase + lane0 + (tl + c T) estr within its instance (offsets within an
    // instance fit in 32 bits).  ubase (instance, group) and c T estr are the
    // same for the whole workgroup and stay in scalar registers; the lane part
    // lane0 + tl estr is the same for every group, so each lane keeps one
    // 32-bit byte offset instead of one 64-bit address per point (it stays
    // below 2^31 bytes for every shape the library accepts).
    const int lane0 = xaxis ? (slot << lnj) : slot;
    const uint32_t loff = (uint32_t)(lane0 + tl * estr) * (uint32_t)sizeof(Store);
    auto point = [&](Store *ub, int c) -> Store & {
        return *reinterpret_cast<Store *>(reinterpret_cast<char *>(ub + (size_t)c * T * estr) + loff);
    };
    // instance and workgroup-shared first element of group gq
    auto locate = [&](int64_t gq, int &inst_q, int &ubase_q) {
        inst_q = (int)(gq / gpi);
        const int64_t g = gq - (int64_t)inst_q * gpi;
        if (xaxis) {
            ubase_q = (int)((g << lg) << lnj);
        } else {
            const int64_t ipo = ((int64_t)1 << lstride) >> lg;  // groups per outer index
            const int inner = (int)((g % ipo) * G);
            const int outer = (int)(g / ipo);
            ubase_q = outer * (nj << lstride) + inner;
        }
    };
    // c64: the next group's points are loaded while the current one is
    // transformed (the 16 extra registers fit; for c128 the 32 they would take
    // cost more in spills than the hidden latency gains)
    constexpr bool kPrefetch = sizeof(Store) == 8;
    Store nxt[kPrefetch ? P : 1];
    int inst_n = 0, ubase_n = 0;
    if constexpr (kPrefetch) {
        if (j_begin < j_end && group_of(j_begin) < total) {
            locate(group_of(j_begin), inst_n, ubase_n);
            Store *src = psi + insts[inst_n].offset + ubase_n;
#pragma unroll
            for (int c = 0; c < P; ++c) nxt[c] = point(src, c);
        }
    }
    for (int64_t j = j_begin; j < j_end; ++j) {
        const int64_t gg = group_of(j);
        if (gg >= total) break;  // uniform across the workgroup
        double2 u[P];
        int inst, ubase;
        if constexpr (kPrefetch) {
            inst = inst_n;
            ubase = ubase_n;
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = to_d2(nxt[c]);
            if (j + 1 < j_end && group_of(j + 1) < total) {
                locate(group_of(j + 1), inst_n, ubase_n);
                Store *src = psi + insts[inst_n].offset + ubase_n;
#pragma unroll
                for (int c = 0; c < P; ++c) nxt[c] = point(src, c);
            }
        } else {
            locate(gg, inst, ubase);
            Store *src = psi + insts[inst].offset + ubase;
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = to_d2(point(src, c));
        }
        const int base = ubase + lane0;  // this thread's pencil, first element
        const InstDev &I = insts[inst];
        const Rec &r = rec[((size_t)inst * rec_steps + step) * m + stage];
        if constexpr (KIND == kPassSep || MODE != 0) {
            if (inst != kf_inst) {  // uniform across the workgroup
                __syncthreads();
                if constexpr (KIND == kPassSep) {
                    const double gk = r.g[axis], ks = I.kscale[axis];
                    for (int q = threadIdx.x; q < nj; q += blockDim.x) {
                        int sq = q - ((2 * q >= nj) ? nj : 0);
                        double k = ks * (double)sq;
                        double2 f = cis_neg_tab(gk * (0.5 * k * k), ctab);
                        kfl[q] = make_double2(f.x * invN, f.y * invN);
                    }
                }
                if constexpr (MODE != 0) {
                    const double loa = I.lo[axis], dxa = I.dx[axis];
                    const double *va = vtab + ((size_t)inst * 3 + axis) * vtab_stride;
                    for (int q = threadIdx.x; q < nj; q += blockDim.x)
                        xvt[q] = make_double2(loa + (double)q * dxa, va[q]);
                }
                __syncthreads();
                kf_inst = inst;
            }
        }
        Store *u0 = psi + I.offset + ubase;

        // merged x-phase: along a pencil only the pass axis's coordinate varies, so
        // the other axes' chirp and V_I factors are formed once per pencil
        // (xpencil, evaluated before the transforms so that its loads overlap
        // them) and the pass axis's coordinate and V_I factor come from xvt
        struct XPen {
            double th0, wv0, lin;
        };
        auto xpencil = [&](const Rec &q, const RecX *qx) -> XPen {
            double th0 = 0.0, v0 = I.eps, lin = 0.0;
            double xo[3] = {0.0, 0.0, 0.0};  // coordinates of the pencil off the pass axis
            int shift = 0;
            for (int j = 0; j < sh.ndim; ++j) {
                if (j != axis) {
                    int i = (base >> shift) & (sh.n[j] - 1);
                    double x = I.lo[j] + (double)i * I.dx[j];
                    xo[j] = x;
                    th0 = fma(q.chi[j], 0.5 * x * x, th0);
                    v0 *= vtab[((size_t)inst * 3 + j) * vtab_stride + i];
                }
                shift += sh.logn[j];
            }
            if (qx) {  // off-diagonal chirp: sum_{i<j} C_ij x_i x_j
#pragma unroll
                for (int pr = 0; pr < 3; ++pr) {
                    const int a = (pr == 2) ? 1 : 0, b = (pr == 0) ? 1 : 2;
                    if (b >= sh.ndim) continue;
                    const double c = qx->chix[pr];
                    if (a == axis) lin = fma(c, xo[b], lin);
                    else if (b == axis) lin = fma(c, xo[a], lin);
                    else th0 = fma(c, xo[a] * xo[b], th0);
                }
            }
            return XPen{th0, q.w * v0, lin};
        };
        auto xpoints = [&](const Rec &q, const XPen &pen) {
            const double chia = q.chi[axis];
            // phase angles of the thread's points, then the factors in batches
            // of XB (the table reads of a batch in flight together)
            constexpr int XB = (P >= 4) ? 4 : P;
#pragma unroll
            for (int c0 = 0; c0 < P; c0 += XB) {
                double th[XB];
#pragma unroll
                for (int cc = 0; cc < XB; ++cc) {
                    const int c = c0 + cc;
                    const int i = tl + c * T;
                    const double2 xv = xvt[i];
                    double a2 = fma(u[c].x, u[c].x, u[c].y * u[c].y);
                    // eps V_I: the caller's value at the point, or the factor form
                    const double rest = fma(q.s, a2, pen.th0);
                    const double bv =
                        vi ? fma(q.w, vi_at(vi, vi_f32, I.offset + base + i * estr), rest) : fma(pen.wv0, xv.y, rest);
                    th[cc] = fma(xv.x, fma(chia, 0.5 * xv.x, pen.lin), bv);
                }
                cis_apply_batch<XB>(u + c0, th, ctab);
            }
        };

        if constexpr (MODE == 2) {
            const RecX *qx = recx_open ? recx_open + inst : nullptr;
            xpoints(rec_open[inst], xpencil(rec_open[inst], qx));
        }
        XPen pen_close{0.0, 0.0, 0.0};
        if constexpr (MODE == 1)
            pen_close = xpencil(r, recx ? recx + ((size_t)inst * rec_steps + step) * m + stage : nullptr);
        if constexpr (KIND != kPassInv) fft.template run<-1>(u);
        if constexpr (KIND == kPassSep) {
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = cmul(u[c], kfl[tl + c * T]);
        }
        if constexpr (KIND == kPassMid) {
            // whole drift k^T G k / 2 with the other wavenumbers of the pencil
            // fixed: c0 + k_a (c1 + G_aa k_a / 2); scaled by 1 / N_total
            const RecX &qx = recx[((size_t)inst * rec_steps + step) * m + stage];
            double ko[3] = {0.0, 0.0, 0.0};
            double scale = invN;
            int shift = 0;
            for (int j = 0; j < sh.ndim; ++j) {
                if (j != axis) {
                    const int i = (base >> shift) & (sh.n[j] - 1);
                    const int sq = i - ((2 * i >= sh.n[j]) ? sh.n[j] : 0);
                    ko[j] = I.kscale[j] * (double)sq;
                    scale *= 1.0 / (double)sh.n[j];
                }
                shift += sh.logn[j];
            }
            double c0 = 0.0, c1 = 0.0;
            for (int j = 0; j < sh.ndim; ++j)
                if (j != axis) c0 = fma(r.g[j], 0.5 * ko[j] * ko[j], c0);
#pragma unroll
            for (int pr = 0; pr < 3; ++pr) {
                const int a = (pr == 2) ? 1 : 0, b = (pr == 0) ? 1 : 2;
                if (b >= sh.ndim) continue;
                const double g = qx.gx[pr];
                if (a == axis) c1 = fma(g, ko[b], c1);
                else if (b == axis) c1 = fma(g, ko[a], c1);
                else c0 = fma(g, ko[a] * ko[b], c0);
            }
            const double gaa = r.g[axis], ksa = I.kscale[axis];
#pragma unroll
            for (int c = 0; c < P; ++c) {
                const int q = tl + c * T;
                const int sq = q - ((2 * q >= nj) ? nj : 0);
                const double k = ksa * (double)sq;
                const double2 f = cis_neg_tab(fma(k, fma(gaa, 0.5 * k, c1), c0), ctab);
                u[c] = cmul(u[c], make_double2(f.x * scale, f.y * scale));
            }
        }
        if constexpr (KIND != kPassFwd) fft.template run<+1>(u);
        if constexpr (MODE == 1) xpoints(r, pen_close);
#pragma unroll
        for (int c = 0; c < P; ++c) point(u0, c) = from_d2<Store>(u[c]);
    }
}

inline NdShape make_shape(const LaunchND &L)
{
    NdShape sh;
    sh.ndim = L.ndim;
    for (int j = 0; j < 3; ++j) {
        sh.n[j] = L.n[j];
        sh.logn[j] = 0;
        while ((1 << sh.logn[j]) < L.n[j]) ++sh.logn[j];
    }
    return sh;
}


template <typename Store, int P, int MAXS, int MODE, int TPB, int KIND, int FIX>
hipError_t launch_pass_tpb(const LaunchND &L)
{
    NdShape sh = make_shape(L);
    int lG = nd_group_log(L.n, L.axis, TPB);
    int threads = 1 << (lG + sh.logn[L.axis] - Log2<P>::value);
    if (FIX != 0 && threads != TPB) return hipErrorInvalidValue;
    int grid = L.grid;
    if (grid <= 0) {
        // persistent grid sized to what the device holds at once for this
        // instance (its registers and LDS set the workgroups per CU); a
        // fixed-shape instance always runs TPB threads, so its figure is kept.
        // Passes along x (contiguous rows) stay at two per CU: a third made
        // them 1-4% slower, while strided passes gained 4-13%.  So do strided
        // passes whose rows are under 64 bytes (a quarter line or less: with a
        // third workgroup the c64 fwd+drift+inv pass on 512-point axes read
        // 1.55x its bytes instead of 1.01x).  No pass takes more than three:
        // the forward and inverse kinds that fit four measured no better.
        static std::atomic<int> fixed_per_cu{0};
        int per_cu = FIX != 0 ? fixed_per_cu.load(std::memory_order_relaxed) : 0;
        if (per_cu <= 0) {
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, hfnd_pass_kernel<Store, P, MAXS, MODE, TPB, KIND, FIX>, threads, 0);
            if (e != hipSuccess) return e;
            per_cu = per_cu > 0 ? per_cu : 1;
            if (FIX != 0) fixed_per_cu.store(per_cu, std::memory_order_relaxed);
        }
        if (L.per_cu > 0) {
            // a tuned count, never more than fit at once
            per_cu = per_cu < L.per_cu ? per_cu : L.per_cu;
        } else {
            if ((L.axis == 0 || ((1 << lG) * (int)sizeof(Store)) < 64) && per_cu > 2) per_cu = 2;
            if (per_cu > 3) per_cu = 3;
        }
        const int64_t pts = (int64_t)L.n[0] * L.n[1] * L.n[2];
        const int64_t groups = (int64_t)L.n_inst * ((pts / L.n[L.axis]) >> lG);
        const int64_t want = (int64_t)per_cu * (L.n_cu > 0 ? L.n_cu : 1);
        grid = (int)(groups < want ? (groups > 0 ? groups : 1) : want);
    }
    hipLaunchKernelGGL((hfnd_pass_kernel<Store, P, MAXS, MODE, TPB, KIND, FIX>), dim3(grid), dim3(threads), 0,
                       L.stream, L.insts, L.n_inst, L.rec, L.rec_open, L.recx, L.recx_open, L.vi, L.vi_f32, L.vtab,
                       L.vtab_stride, L.cistab, L.twtab, L.twlog, (Store *)L.psi, sh, L.axis, lG, L.stage, L.m,
                       L.rec_steps, L.step, L.step_base);
    return hipGetLastError();
}

}  // namespace hfgpe
