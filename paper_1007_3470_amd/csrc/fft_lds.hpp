// fft_lds.hpp -- workgroup-level complex FFT of power-of-two length on FP64
// registers with LDS exchange (Stockham auto-sort, radix-P passes), shared by
// the 1-D resident kernel and the d-D axis-pass kernels.
//
// An FFT of length N is split over T = N/P threads.  Thread t holds the P
// points {t + c T} before the first pass and after the last one.  Pass s
// (s >= 1) is a radix-P butterfly preceded by twiddles exp(-2 pi i r k /(L P))
// (k = t mod L, L = product of the earlier radices); the first pass uses the
// radix R0 = N / P^(S-1) <= P.  Between passes the values go through LDS at
// element offsets map(idx) = (pad ? idx + idx/16 : idx) * istride.
#pragma once
#include <hip/hip_runtime.h>

#include "devmath.hpp"

namespace hfgpe {

constexpr int kThreads1D = 256;
#ifndef HFGPE_PAD_SHIFT
#define HFGPE_PAD_SHIFT 3
#endif
constexpr int kPadShift = HFGPE_PAD_SHIFT;  // one padding element every 2^kPadShift in LDS

__device__ __forceinline__ int lds_pad(int idx) { return idx + (idx >> kPadShift); }

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename T>
__device__ __forceinline__ T from_d2(double2 v);
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }

template <int P>
struct Log2 {
    static constexpr int value = (P <= 1) ? 0 : 1 + Log2<P / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

template <typename Xch, int P, int MAXS>
struct Fft1D {
    int istride = 1;
    bool pad = true;
    __device__ __forceinline__ int map(int idx) const { return (pad ? lds_pad(idx) : idx) * istride; }

    static constexpr int LOGP = Log2<P>::value;
    static constexpr int NTW = (MAXS > 1) ? MAXS - 1 : 1;
    static constexpr int PW = (P > 1) ? P - 1 : 1;

    int logn, logT, S, r0log, tl;
    Xch *buf;
    // Twiddles of passes 1..S-1: for radix 8 only w^1, w^2, w^4 are kept and
    // the rest formed by products when a pass runs (fewer registers); other
    // radices keep all P-1 powers.
    static constexpr int NKEEP = (P == 8) ? 3 : PW;
    double2 tw[NTW][NKEEP];

    // twtab (optional): exp(-2 pi i q / 2^twlog) for q < 2^twlog, twlog >= logn
    __device__ void init(int logn_, int tl_, Xch *buf_, const double2 *__restrict__ twtab = nullptr,
                         int twlog = 0)
    {
        logn = logn_;
        tl = tl_;
        buf = buf_;
        logT = logn - LOGP;
        S = (logn == 0 || LOGP == 0) ? 0 : (logn + LOGP - 1) / (LOGP > 0 ? LOGP : 1);
        r0log = (S == 0) ? 0 : logn - LOGP * (S - 1);
        const double invN = 1.0 / (double)(1 << logn);
#pragma unroll
        for (int s = 1; s < MAXS; ++s) {
            if (s < S) {
                int logL = r0log + LOGP * (s - 1);
                int k = tl & ((1 << logL) - 1);
                int slog = logn - logL - LOGP;
#pragma unroll
                for (int q = 0; q < NKEEP; ++q) {
                    int r = (P == 8) ? (1 << q) : q + 1;
                    int e = (r * k) << slog;
                    if (twtab) {
                        tw[s - 1][q] = twtab[e << (twlog - logn)];
                    } else {
                        double sn, cs;
                        sincospi(-2.0 * (double)e * invN, &sn, &cs);
                        tw[s - 1][q] = make_double2(cs, sn);
                    }
                }
            }
        }
    }

    // twiddle r (1..P-1) of pass s
    __device__ __forceinline__ void twiddles(int s, double2 *w) const
    {
        if constexpr (P == 8) {
            const double2 w1 = tw[s - 1][0], w2 = tw[s - 1][1], w4 = tw[s - 1][2];
            const double2 w3 = cmul(w1, w2);
            w[0] = w1;
            w[1] = w2;
            w[2] = w3;
            w[3] = w4;
            w[4] = cmul(w1, w4);
            w[5] = cmul(w2, w4);
            w[6] = cmul(w3, w4);
        } else {
#pragma unroll
            for (int r = 0; r < PW; ++r) w[r] = tw[s - 1][r];
        }
    }

    template <int R, int SGN>
    __device__ __forceinline__ void pass0(double2 *u)
    {
        constexpr int NB = P / R;
        const int T = 1 << logT;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double2 v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = u[b + r * NB];
            Dft<R, SGN>::run(v);
            int j = tl + b * T;
#pragma unroll
            for (int rp = 0; rp < R; ++rp) buf[map(j * R + rp)] = from_d2<Xch>(v[rp]);
        }
    }

    template <int SGN>
    __device__ __forceinline__ void run(double2 *u)
    {
        if constexpr (P == 1) {
            return;
        } else {
            if (S == 1) {  // N == P: one thread holds the whole instance
                Dft<P, SGN>::run(u);
                return;
            }
            switch (r0log) {
            case 1: pass0<2, SGN>(u); break;
            case 2: pass0<4, SGN>(u); break;
            case 3: if constexpr (P >= 8) pass0<8, SGN>(u); break;
            case 4: if constexpr (P >= 16) pass0<16, SGN>(u); break;
            default: break;
            }
            const int T = 1 << logT;
#pragma unroll
            for (int s = 1; s < MAXS; ++s) {
                if (s < S) {
                    __syncthreads();
#pragma unroll
                    for (int c = 0; c < P; ++c) u[c] = to_d2(buf[map(tl + c * T)]);
                    __syncthreads();
                    double2 w[PW];
                    twiddles(s, w);
#pragma unroll
                    for (int r = 1; r < P; ++r) u[r] = (SGN < 0) ? cmul(u[r], w[r - 1]) : cmulc(u[r], w[r - 1]);
                    Dft<P, SGN>::run(u);
                    if (s < S - 1) {
                        int logL = r0log + LOGP * (s - 1);
                        int L = 1 << logL;
                        int k = tl & (L - 1);
                        int base = (tl - k) * P + k;
#pragma unroll
                        for (int rp = 0; rp < P; ++rp) buf[map(base + rp * L)] = from_d2<Xch>(u[rp]);
                    }
                }
            }
        }
    }
};

// Fixed-shape radix-8 FFT on padded rows: N = 2^LOGN points split over
// T = N/8 threads (T a multiple of 8), one padding element every 8 (as Fft1D
// with pad = true, istride = 1).  Xch is the LDS exchange type: double2 for
// the resident 1-D kernel and the c128 passes, float2 for the c64 d-D passes
// (arithmetic and twiddles stay FP64 either way).  With the shape known at
// compile time each LDS address is a per-thread base plus a constant, so the
// addresses of all passes fold into instruction offsets instead of occupying
// registers across the step loop.  The padding algebra used below:
// pad(x + y) = pad(x) + y + (y >> 3) whenever (x mod 8) + (y mod 8) < 8.
template <int LOGN, typename Xch = double2, int NBUF = 1, int BSTRIDE = 0>
struct FftFix8 {
    static constexpr int P = 8, LOGP = 3;
    static constexpr int N = 1 << LOGN;
    static constexpr int LOGT = LOGN - LOGP;
    static constexpr int T = 1 << LOGT;
    static constexpr int S = (LOGN + LOGP - 1) / LOGP;  // passes
    static constexpr int R0LOG = LOGN - LOGP * (S - 1);  // pass 0 has radix 2^R0LOG
    static constexpr int R0 = 1 << R0LOG;
    static constexpr int ROW = N + (N >> kPadShift);     // padded elements per instance
    static constexpr int TP = T + (T >> 3);              // padded stride of the points {t + cT}
    static_assert(kPadShift == 3 && T % 8 == 0 && S >= 2, "fixed-shape FFT: N >= 64");

    Xch *lds;
    int roff;             // pad(t) + instance row
    int w0off;            // pad(t R0) + instance row
    int woff[S > 2 ? S - 2 : 1];  // pass s write base, s = 1 .. S-2
    double2 tw[S - 1][3];         // w^1, w^2, w^4 of passes 1 .. S-1

    // twtab (optional): exp(-2 pi i q / 2^twlog) for q < 2^twlog, twlog >= LOGN;
    // without it the twiddles are evaluated with sincospi
    __device__ __forceinline__ void init(int tl, int slot, Xch *lds_, const double2 *__restrict__ twtab = nullptr,
                                         int twlog = 0)
    {
        lds = lds_;
        const int row = slot * ROW;
        roff = row + tl + (tl >> 3);
        const int x0 = tl * R0;
        w0off = row + x0 + (x0 >> 3);
        constexpr double invN = 1.0 / (double)N;
#pragma unroll
        for (int s = 1; s < S; ++s) {
            const int logL = R0LOG + LOGP * (s - 1);
            const int k = tl & ((1 << logL) - 1);
            if (s < S - 1) {
                const int base = (tl - k) * P + k;
                woff[s - 1] = row + base + (base >> 3);
            }
            const int slog = LOGN - logL - LOGP;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int e = ((1 << q) * k) << slog;
                if (twtab) {
                    tw[s - 1][q] = twtab[e << (twlog - LOGN)];
                } else {
                    double sn, cs;
                    sincospi(-2.0 * (double)e * invN, &sn, &cs);
                    tw[s - 1][q] = make_double2(cs, sn);
                }
            }
        }
    }

    // With NBUF = 2 the passes alternate between two buffers BSTRIDE elements
    // apart: pass s reads the buffer pass s - 1 wrote and writes the other,
    // so one barrier per pass suffices (a pass writes the buffer the previous
    // pass read, and every wave has finished those reads at the barrier
    // before its own reads).  Pass 0 writes buffer START; the call after this
    // one must start at next_start(START), the buffer the last pass did not
    // read, since nothing separates the last reads from the next writes.
    static constexpr int next_start(int start) { return (NBUF == 2) ? ((start + S - 1) & 1) : 0; }

    template <int SGN, int START = 0>
    __device__ __forceinline__ void run(double2 *u)
    {
        static_assert(NBUF == 1 || NBUF == 2, "one or two exchange buffers");
        constexpr auto buf = [](int k) { return (NBUF == 2) ? (k & 1) * BSTRIDE : 0; };
        // pass 0: radix R0 on the thread's own points {t + cT}
        constexpr int NB = P / R0;
        constexpr int BSTR = T * R0 + ((T * R0) >> 3);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double2 v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = u[b + r * NB];
            Dft<R0, SGN>::run(v);
#pragma unroll
            for (int rp = 0; rp < R0; ++rp) lds[buf(START) + w0off + b * BSTR + rp] = from_d2<Xch>(v[rp]);
        }
#pragma unroll
        for (int s = 1; s < S; ++s) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = to_d2(lds[buf(START + s - 1) + roff + c * TP]);
            if constexpr (NBUF == 1) __syncthreads();
            const double2 w1 = tw[s - 1][0], w2 = tw[s - 1][1], w4 = tw[s - 1][2];
            const double2 w3 = cmul(w1, w2);
            const double2 w[7] = {w1, w2, w3, w4, cmul(w1, w4), cmul(w2, w4), cmul(w3, w4)};
#pragma unroll
            for (int r = 1; r < P; ++r) u[r] = (SGN < 0) ? cmul(u[r], w[r - 1]) : cmulc(u[r], w[r - 1]);
            Dft<P, SGN>::run(u);
            if (s < S - 1) {
                const int L = 1 << (R0LOG + LOGP * (s - 1));
#pragma unroll
                for (int rp = 0; rp < P; ++rp)
                    lds[buf(START + s) + woff[s - 1] + rp * L + ((rp * L) >> 3)] = from_d2<Xch>(u[rp]);
            }
        }
    }
};

// Fixed-shape radix-8 FFT of the strided d-D axis passes: the G pencils of a
// workgroup are interleaved in LDS (point idx of pencil `slot` at idx * G +
// slot, no padding), a pencil's N = 2^LOGN points are split over T = N/8
// threads, and the passes and twiddles are those of Fft1D.  As in FftFix8 every
// LDS address is a per-thread base plus a compile-time constant, and Xch is
// the exchange type.
template <int LOGN, int G, typename Xch = double2>
struct FftFixS8 {
    static constexpr int P = 8, LOGP = 3;
    static constexpr int N = 1 << LOGN;
    static constexpr int LOGT = LOGN - LOGP;
    static constexpr int T = 1 << LOGT;
    static constexpr int S = (LOGN + LOGP - 1) / LOGP;
    static constexpr int R0LOG = LOGN - LOGP * (S - 1);
    static constexpr int R0 = 1 << R0LOG;
    static_assert(S >= 2 && G >= 1, "fixed-shape strided FFT: N >= 16");

    Xch *lds;
    int roff;                     // tl G + slot: point tl of the pencil
    int w0off;                    // tl R0 G + slot: pass 0 write base
    int woff[S > 2 ? S - 2 : 1];  // pass s write base, s = 1 .. S-2
    double2 tw[S - 1][3];         // w^1, w^2, w^4 of passes 1 .. S-1

    __device__ __forceinline__ void init(int tl, int slot, Xch *lds_, const double2 *__restrict__ twtab,
                                         int twlog)
    {
        lds = lds_;
        roff = tl * G + slot;
        w0off = tl * R0 * G + slot;
#pragma unroll
        for (int s = 1; s < S; ++s) {
            const int logL = R0LOG + LOGP * (s - 1);
            const int k = tl & ((1 << logL) - 1);
            if (s < S - 1) woff[s - 1] = ((tl - k) * P + k) * G + slot;
            const int slog = LOGN - logL - LOGP;
#pragma unroll
            for (int q = 0; q < 3; ++q) tw[s - 1][q] = twtab[(((1 << q) * k) << slog) << (twlog - LOGN)];
        }
    }

    template <int SGN>
    __device__ __forceinline__ void run(double2 *u)
    {
        constexpr int NB = P / R0;
        constexpr int BSTR = T * R0 * G;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double2 v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = u[b + r * NB];
            Dft<R0, SGN>::run(v);
#pragma unroll
            for (int rp = 0; rp < R0; ++rp) lds[w0off + b * BSTR + rp * G] = from_d2<Xch>(v[rp]);
        }
#pragma unroll
        for (int s = 1; s < S; ++s) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < P; ++c) u[c] = to_d2(lds[roff + c * T * G]);
            __syncthreads();
            const double2 w1 = tw[s - 1][0], w2 = tw[s - 1][1], w4 = tw[s - 1][2];
            const double2 w3 = cmul(w1, w2);
            const double2 w[7] = {w1, w2, w3, w4, cmul(w1, w4), cmul(w2, w4), cmul(w3, w4)};
#pragma unroll
            for (int r = 1; r < P; ++r) u[r] = (SGN < 0) ? cmul(u[r], w[r - 1]) : cmulc(u[r], w[r - 1]);
            Dft<P, SGN>::run(u);
            if (s < S - 1) {
                const int L = 1 << (R0LOG + LOGP * (s - 1));
#pragma unroll
                for (int rp = 0; rp < P; ++rp) lds[woff[s - 1] + rp * L * G] = from_d2<Xch>(u[rp]);
            }
        }
    }
};

}  // namespace hfgpe
