// devmath.hpp -- FP64 complex arithmetic, the phase factor exp(-i theta) and
// in-register radix-2^k DFT butterflies for the gfx950 kernels.
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
// exp(-i theta) in FP64, accurate to a few ulp for |theta| < 2^30.
// Cody-Waite reduction by pi/2 with a two-word constant and FMA, then the
// Taylor series of sin and cos on [-pi/4, pi/4] (sin through x^17, cos
// through x^18, so the one-signed truncation error stays below 1e-19 and
// |exp(-i theta)| carries no systematic bias), then the quadrant rotation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cis_neg(double theta)
{
    const double TWO_OVER_PI = 0.6366197723675814;
    const double PIO2_HI = 1.5707963267948966;     // 0x1.921fb54442d18p+0
    const double PIO2_LO = 6.123233995736766e-17;  // pi/2 - PIO2_HI
    double n = rint(theta * TWO_OVER_PI);
    double r = fma(-n, PIO2_HI, theta);
    r = fma(-n, PIO2_LO, r);
    double r2 = r * r;
    // sin r = r - r^3/3! + r^5 (1/5! + r^2 (-1/7! + ...)); 1/3! and 1/4! enter as
    // hi + lo pairs (their rounding would otherwise bias |exp(-i theta)|)
    double ps = 2.8114572543455206e-15;         //  1/17!
    ps = fma(ps, r2, -7.647163731819816e-13);   // -1/15!
    ps = fma(ps, r2, 1.6059043836821613e-10);   //  1/13!
    ps = fma(ps, r2, -2.505210838544172e-08);   // -1/11!
    ps = fma(ps, r2, 2.7557319223985893e-06);   //  1/9!
    ps = fma(ps, r2, -1.984126984126984e-04);   // -1/7!
    ps = fma(ps, r2, 8.333333333333333e-03);    //  1/5!
    double r3 = r * r2;
    double st = fma(r3, -9.251858538542971e-18, r3 * r2 * ps);
    double s = r + fma(r3, -1.6666666666666666e-01, st);
    // cos r = 1 - r^2/2 + r^4/4! + r^6 (-1/6! + r^2 (1/8! + ...))
    double pc = -1.5619206968586225e-16;        // -1/18!
    pc = fma(pc, r2, 4.779477332387385e-14);    //  1/16!
    pc = fma(pc, r2, -1.1470745597729725e-11);  // -1/14!
    pc = fma(pc, r2, 2.08767569878681e-09);     //  1/12!
    pc = fma(pc, r2, -2.755731922398589e-07);   // -1/10!
    pc = fma(pc, r2, 2.48015873015873e-05);     //  1/8!
    pc = fma(pc, r2, -1.3888888888888889e-03);  // -1/6!
    double r4 = r2 * r2;
    double ct = fma(r4, 2.3129646346357427e-18, r4 * r2 * pc);
    double hr = 0.5 * r2;
    double w = 1.0 - hr;
    double c = w + (((1.0 - w) - hr) + fma(r4, 4.1666666666666664e-02, ct));
    // theta = n pi/2 + r: rotate (cos r, sin r) by the quadrant
    int q = ((int)n) & 3;
    double cq = (q & 1) ? s : c;
    double sq = (q & 1) ? c : s;
    if (q == 1 || q == 2) cq = -cq;
    if (q >= 2) sq = -sq;
    return make_double2(cq, -sq);
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
