// devmath.hpp -- FP64 complex arithmetic, the phase factor exp(-i theta) and
// in-register radix-2^k DFT butterflies for the gfx950 kernels.
//
// Every constant that multiplies data (sqrt(1/2), cos/sin(pi/8), the phase
// table) enters as a hi + lo pair: a single rounded constant is biased in
// magnitude by up to half an ulp, and a bias that repeats every step grows
// linearly over thousands of steps (a rounded sqrt(1/2) alone drove a 2e-12
// norm drift over 10^4 steps).
#pragma once
#include <hip/hip_runtime.h>

namespace hfgpe {

// ---------------------------------------------------------------------------
// Complex helpers (double2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// exp(-i theta) with a 256-entry table: theta = n pi/128 + r, |r| <= pi/256,
// exp(-i theta) = T_n exp(-i r) with T_n = exp(-i n pi/128) (n mod 256).
// The table holds T_n rounded to FP64, t, together with its rounding error
// written as a relative correction: T_n = t (1 + a + i b), |a|, |b| ~ 1e-16
// (kept as floats).  Up to O(1e-32), T_n exp(-i r) = t (1 + a) exp(-i (r - b)),
// so the angle error enters the series argument and the magnitude error the
// cosine term; the product with t is then rounded once and the table adds no
// magnitude bias.  Series: sin through rho^7, cos - 1 through rho^6
// (truncation < 2e-20 on |rho| <= pi/256).
// ---------------------------------------------------------------------------
constexpr int kCisTable = 256;

struct CisTable {
    double2 t[kCisTable];  // exp(-i n pi/128) rounded to FP64
    float2 c[kCisTable];   // (b, a): angle and magnitude parts of the rounding error
};

__device__ __forceinline__ double2 cis_neg_tab(double theta, const CisTable &tab)
{
    const double K = 40.743665431525208;          // 128 / pi
    const double C_HI = 0.024543692606170259;     // pi/128 (leading word)
    const double C_LO = 9.5714723039735938e-19;   // pi/128 - C_HI
    double n = rint(theta * K);
    double r = fma(-n, C_HI, theta);
    r = fma(-n, C_LO, r);
    const int j = ((int)n) & (kCisTable - 1);
    const float2 cor = tab.c[j];
    const double2 t = tab.t[j];
    const double rho = r - (double)cor.x;
    const double r2 = rho * rho;
    double ps = fma(r2, -1.984126984126984e-04, 8.333333333333333e-03);  // -1/7!, 1/5!
    ps = fma(ps, r2, -1.6666666666666666e-01);                           // -1/3!
    const double sn = fma(rho * r2, ps, rho);
    double pc = fma(r2, -1.3888888888888889e-03, 4.1666666666666664e-02);  // -1/6!, 1/4!
    pc = fma(pc, r2, -0.5);
    const double cm = fma(r2, pc, (double)cor.y);  // cos(rho) - 1 + a
    // t (1 + cm - i sn)
    return make_double2(fma(t.x, cm, fma(t.y, sn, t.x)), fma(t.y, cm, fma(-t.x, sn, t.y)));
}

// u[c] <- u[c] exp(-i theta[c]) for c < NP, written as three sweeps (angles
// and table indices; all table reads; series and products) so the LDS reads of
// the NP evaluations are in flight together instead of one after another.
// Same arithmetic as cis_neg_tab.  scale multiplies the factor (exactly, when
// it is a power of two).
template <int NP>
__device__ __forceinline__ void cis_apply_batch(double2 *u, const double *theta, const CisTable &tab,
                                                double scale = 1.0)
{
    const double K = 40.743665431525208;
    const double C_HI = 0.024543692606170259;
    const double C_LO = 9.5714723039735938e-19;
    double r[NP];
    int j[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double n = rint(theta[c] * K);
        double rr = fma(-n, C_HI, theta[c]);
        r[c] = fma(-n, C_LO, rr);
        j[c] = ((int)n) & (kCisTable - 1);
    }
    double2 t[NP];
    float2 cor[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        t[c] = tab.t[j[c]];
        cor[c] = tab.c[j[c]];
    }
    // keep the reads ahead of the series (the scheduler would otherwise sink
    // each read next to its use and wait for it alone)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double rho = r[c] - (double)cor[c].x;
        const double r2 = rho * rho;
        double ps = fma(r2, -1.984126984126984e-04, 8.333333333333333e-03);
        ps = fma(ps, r2, -1.6666666666666666e-01);
        const double sn = fma(rho * r2, ps, rho);
        double pc = fma(r2, -1.3888888888888889e-03, 4.1666666666666664e-02);
        pc = fma(pc, r2, -0.5);
        const double cm = fma(r2, pc, (double)cor[c].y);
        const double tx = t[c].x * scale, ty = t[c].y * scale;
        const double2 f = make_double2(fma(tx, cm, fma(ty, sn, tx)), fma(ty, cm, fma(-tx, sn, ty)));
        u[c] = cmul(u[c], f);
    }
}

// f[c] = exp(-i theta[c]) for c < NP: the factors of cis_apply_batch (same
// arithmetic, table reads issued together) without the multiply.
template <int NP>
__device__ __forceinline__ void cis_batch(const double *theta, double2 *f, const CisTable &tab)
{
    const double K = 40.743665431525208;
    const double C_HI = 0.024543692606170259;
    const double C_LO = 9.5714723039735938e-19;
    double r[NP];
    int j[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double n = rint(theta[c] * K);
        double rr = fma(-n, C_HI, theta[c]);
        r[c] = fma(-n, C_LO, rr);
        j[c] = ((int)n) & (kCisTable - 1);
    }
    double2 t[NP];
    float2 cor[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        t[c] = tab.t[j[c]];
        cor[c] = tab.c[j[c]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double rho = r[c] - (double)cor[c].x;
        const double r2 = rho * rho;
        double ps = fma(r2, -1.984126984126984e-04, 8.333333333333333e-03);
        ps = fma(ps, r2, -1.6666666666666666e-01);
        const double sn = fma(rho * r2, ps, rho);
        double pc = fma(r2, -1.3888888888888889e-03, 4.1666666666666664e-02);
        pc = fma(pc, r2, -0.5);
        const double cm = fma(r2, pc, (double)cor[c].y);
        const double tx = t[c].x, ty = t[c].y;
        f[c] = make_double2(fma(tx, cm, fma(ty, sn, tx)), fma(ty, cm, fma(-tx, sn, ty)));
    }
}

// copy the table (as raw 16-byte words) from global memory into LDS
__device__ __forceinline__ void load_cis_table(CisTable *lds_tab, const double2 *__restrict__ gtab)
{
    double2 *dst = reinterpret_cast<double2 *>(lds_tab);
    constexpr int kWords = (int)(sizeof(CisTable) / sizeof(double2));
    for (int j = threadIdx.x; j < kWords; j += blockDim.x) dst[j] = gtab[j];
}

// ---------------------------------------------------------------------------
// In-register DFT of length R (power of two, R <= 16), natural order in and
// out, sign SGN = -1 (forward) or +1 (inverse, unscaled).  Radix-2
// decimation in time, unrolled at compile time.
// ---------------------------------------------------------------------------
template <int R, int K, int SGN>
__device__ __forceinline__ double2 twiddle_const(double2 v)
{
    // v * exp(SGN * 2 pi i K / R) with exact special cases
    constexpr int Kn = (K * 16) / R;  // angle in units of 2 pi / 16
    if constexpr (Kn == 0) {
        return v;
    } else if constexpr (Kn == 4) {
        // exp(SGN i pi/2) = SGN i
        return SGN < 0 ? make_double2(v.y, -v.x) : make_double2(-v.y, v.x);
    } else if constexpr (Kn == 2 || Kn == 6) {
        // exp(SGN i pi/4) = h (1 + SGN i); exp(SGN i 3pi/4) = h (-1 + SGN i), with
        // h = sqrt(1/2) applied as a hi + lo pair so each product is rounded once
        // (a rounded h alone would scale every such product by 1 + 8e-17).
        const double HH = 0.7071067811865476, HL = -4.833646656726457e-17;
        double a = v.x, b = v.y;
        double p, q;
        if constexpr (Kn == 2) {
            p = (SGN < 0) ? (a + b) : (a - b);
            q = (SGN < 0) ? (b - a) : (a + b);
        } else {
            p = (SGN < 0) ? (b - a) : -(a + b);
            q = (SGN < 0) ? -(a + b) : (a - b);
        }
        return make_double2(fma(p, HH, p * HL), fma(q, HH, q * HL));
    } else {
        // cos, sin (pi/8) as hi + lo pairs
        const double C1H = 0.9238795325112867, C1L = 1.7645047084336677e-17;
        const double S1H = 0.3826834323650898, S1L = -1.0050772696461588e-17;
        double crh, crl, cih, cil;
        if constexpr (Kn == 1) { crh = C1H; crl = C1L; cih = S1H; cil = S1L; }
        else if constexpr (Kn == 3) { crh = S1H; crl = S1L; cih = C1H; cil = C1L; }
        else if constexpr (Kn == 5) { crh = -S1H; crl = -S1L; cih = C1H; cil = C1L; }
        else { crh = -C1H; crl = -C1L; cih = S1H; cil = S1L; }  // Kn == 7
        if constexpr (SGN < 0) { cih = -cih; cil = -cil; }
        double re = fma(v.x, crh, fma(-v.y, cih, v.x * crl - v.y * cil));
        double im = fma(v.x, cih, fma(v.y, crh, v.x * cil + v.y * crl));
        return make_double2(re, im);
    }
}

template <int R, int SGN>
struct Dft {
    template <int K>
    __device__ __forceinline__ static void combine(double2 *v, const double2 *e, const double2 *o)
    {
        if constexpr (K < R / 2) {
            double2 t = twiddle_const<R, K, SGN>(o[K]);
            v[K] = cadd(e[K], t);
            v[K + R / 2] = csub(e[K], t);
            combine<K + 1>(v, e, o);
        }
    }
    __device__ __forceinline__ static void run(double2 *v)
    {
        double2 e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        Dft<R / 2, SGN>::run(e);
        Dft<R / 2, SGN>::run(o);
        combine<0>(v, e, o);
    }
};

template <int SGN>
struct Dft<1, SGN> {
    __device__ __forceinline__ static void run(double2 *) {}
};

template <int SGN>
struct Dft<2, SGN> {
    __device__ __forceinline__ static void run(double2 *v)
    {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

}  // namespace hfgpe
