// fft_engine.h -- device-side Stockham FFT of one line held by a group of threads.
//
// The 2D transforms of the split step (Sec. 3.1: FFT forward and inverse along x and y)
// are done line by line.  A line of N points is held by T = N / R threads, R points
// each, thread t owning positions t + m*T (m < R).  The transform runs as a sequence of
// Stockham passes of radix R (the last pass may have a smaller radix): every pass
// applies its twiddles and a radix butterfly in registers and exchanges data through
// LDS; the first pass reads and the last pass leaves its values in registers, in the
// same t + m*T layout, so a line can be loaded coalesced from global memory, transformed
// and stored coalesced with only (passes - 1) LDS exchanges.
//
// Arithmetic type: `Real` (double on the production path).  On CDNA3/CDNA4 a double FMA
// issues at the same rate as a non-packed single FMA, and FP64 twiddles keep the
// forward/inverse round trip free of the systematic modulus bias that single-precision
// twiddles add at every step; complex64 is kept for HBM storage only.
#pragma once
#include <hip/hip_runtime.h>

#ifndef GPE_TW_POW2
#define GPE_TW_POW2 1
#endif

namespace gpe {

template <typename Real> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward transform) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot_mi(C a)
{
    if constexpr (INV) return {-a.y, a.x};
    else return {a.y, -a.x};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// cos and sin of 2 pi e / 16 for e = 0..15 (exact decimal expansions, rounded by the
// compiler to the arithmetic type).
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// a * W_M^E with W_M = exp(-2 pi i / M) (forward) or its conjugate (inverse); M | 16.
template <int E, int M, bool INV, typename C> __device__ __forceinline__ C twc(C a)
{
    constexpr int e = ((E % M) + M) % M;
    constexpr int k = e * (16 / M);  // exponent on the 16-th roots
    if constexpr (k == 0) {
        return a;
    } else if constexpr (k == 8) {
        return {-a.x, -a.y};
    } else if constexpr (k == 4) {
        return rot_mi<INV>(a);
    } else if constexpr (k == 12) {
        return rot_mi<!INV>(a);
    } else {
        using R = decltype(a.x);
        const R c = (R)kC16[k];
        const R s = INV ? (R)kS16[k] : -(R)kS16[k];
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// In-place DFT of size P on a[0..P-1] (natural order in and out), P in {1,2,4,8,16}.
template <int P, bool INV, typename C> struct Dft;

template <bool INV, typename C> struct Dft<1, INV, C> {
    static __device__ __forceinline__ void run(C *) {}
};
template <bool INV, typename C> struct Dft<2, INV, C> {
    static __device__ __forceinline__ void run(C *a)
    {
        C t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};
template <bool INV, typename C> struct Dft<4, INV, C> {
    static __device__ __forceinline__ void run(C *a)
    {
        C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        C t2 = cadd(a[1], a[3]), t3 = rot_mi<INV>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};
// P = P1 * 4 with input index n = P1*n1 + n2 ... written as the standard two-level
// split: X[k1 + 4 k2] = sum_{n2} W_P^{n2 k1} [sum_{n1} a[S n1 + n2] W_4^{n1 k1}] W_S^{n2 k2},
// S = P / 4 (inner DFT-4 over stride-S inputs, twiddle, outer DFT-S).
template <int P, bool INV, typename C> struct Dft {
    static constexpr int S = P / 4;
    template <int N2> static __device__ __forceinline__ void inner(C *a, C (&b)[4][S])
    {
        if constexpr (N2 < S) {
            C q[4] = {a[N2], a[S + N2], a[2 * S + N2], a[3 * S + N2]};
            Dft<4, INV, C>::run(q);
            b[0][N2] = q[0];
            b[1][N2] = twc<N2 * 1, P, INV>(q[1]);
            b[2][N2] = twc<N2 * 2, P, INV>(q[2]);
            b[3][N2] = twc<N2 * 3, P, INV>(q[3]);
            inner<N2 + 1>(a, b);
        }
    }
    static __device__ __forceinline__ void run(C *a)
    {
        C b[4][S];
        inner<0>(a, b);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            Dft<S, INV, C>::run(b[k1]);
#pragma unroll
            for (int k2 = 0; k2 < S; ++k2) a[k1 + 4 * k2] = b[k1][k2];
        }
    }
};

// Pass schedule of an N-point transform with R points per thread: NFULL passes of
// radix R, then one pass of radix RL = N / R^NFULL when that is > 1.
template <int N, int R> struct FftShape {
    static constexpr int T = N / R;
    static constexpr int LGN = ilog2(N), LGR = ilog2(R);
    static constexpr int NFULL = LGN / LGR;
    static constexpr int RL = 1 << (LGN - NFULL * LGR);
    static constexpr int NPASS = NFULL + (RL > 1 ? 1 : 0);
    static_assert((1 << LGN) == N && (1 << LGR) == R && R <= N, "powers of two only");
};

// One Stockham pass.  Ns = product of the radices before this pass.  View: LDS line
// accessor with operator()(int idx) -> C& (exchange storage of N points).  tw holds
// W_{TS N}^m: an N-point transform takes every TS-th entry of a longer line's table.
template <int N, int R, bool INV, int PASS, int TS = 1, typename C, typename View>
__device__ __forceinline__ void fft_pass(C (&v)[R], const View &lds, int t, const C *__restrict__ tw)
{
    using S = FftShape<N, R>;
    if constexpr (PASS < S::NPASS) {
        constexpr int Rp = (PASS < S::NFULL) ? R : S::RL;
        constexpr int Q = R / Rp;
        constexpr int Ns = 1 << (PASS * S::LGR);
        constexpr int T = S::T;
        constexpr bool LAST = (PASS == S::NPASS - 1);
        if constexpr (PASS > 0) {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = lds.template ld<C>(t + m * T);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int u = t + q * T;
            const int j = u & (Ns - 1);
            C a[Rp];
#pragma unroll
            for (int r = 0; r < Rp; ++r) a[r] = v[q + r * Q];
            if constexpr (Ns > 1) {
                constexpr int stride = TS * (N / (Ns * Rp));
#if GPE_TW_POW2
                // powers w^1, w^2, w^4 (and w^8) from the table, the others as FP64
                // products (rounding ~1e-16 per product, far below the complex64 storage)
                C w[Rp];
                w[1] = tw[j * stride];
                if constexpr (Rp > 2) w[2] = tw[2 * j * stride];
                if constexpr (Rp > 4) w[4] = tw[4 * j * stride];
                if constexpr (Rp > 8) w[8 % Rp] = tw[8 * j * stride];
                if constexpr (Rp > 2) w[3] = cmul(w[1], w[2]);
                if constexpr (Rp > 4) {
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
                if constexpr (Rp > 8)
#pragma unroll
                    for (int r = 9; r < Rp; ++r) w[r] = cmul(w[r - 8], w[8 % Rp]);
                static_assert(Rp <= 16, "power-of-two twiddle reconstruction is written for radix <= 16");
#pragma unroll
                for (int r = 1; r < Rp; ++r) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
#else
#pragma unroll
                for (int r = 1; r < Rp; ++r) {
                    C w = tw[r * j * stride];
                    a[r] = INV ? cmulc(a[r], w) : cmul(a[r], w);
                }
#endif
            }
            Dft<Rp, INV, C>::run(a);
#pragma unroll
            for (int r = 0; r < Rp; ++r) v[q + r * Q] = a[r];
        }
        if constexpr (!LAST) {
            __syncthreads();  // every thread has finished reading this pass's inputs
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int u = t + q * T;
                const int j = u & (Ns - 1);
                const int base = (u / Ns) * Ns * Rp + j;
#pragma unroll
                for (int r = 0; r < Rp; ++r) lds.st(base + r * Ns, v[q + r * Q]);
            }
            __syncthreads();
            fft_pass<N, R, INV, PASS + 1, TS>(v, lds, t, tw);
        }
    }
}

// Full transform of one line: in v[m] = x[t + m*T], out v[m] = X[t + m*T], unscaled.
// Every thread of the work-group must call this (it contains work-group barriers).
template <int N, int R, bool INV, int TS = 1, typename C, typename View>
__device__ __forceinline__ void fft_line(C (&v)[R], const View &lds, int t, const C *__restrict__ tw)
{
    fft_pass<N, R, INV, 0, TS>(v, lds, t, tw);
}


// Twiddles of every pass of an N-point transform for thread t, loaded once (before the
// data arrives) and kept in registers for the forward and the inverse transform alike:
// pass PASS, sub-butterfly q holds w^1, w^2, w^4 of its W_{Ns Rp}^j (as many as the radix
// uses; the other powers are formed as products, as in fft_pass).
template <int N, int R, typename C> struct TwPre {
    static constexpr int NP = FftShape<N, R>::NPASS;
    C w[NP > 0 ? NP : 1][R][3];
};

template <int N, int R, int PASS, typename C>
__device__ __forceinline__ void tw_preload(TwPre<N, R, C> &p, const C *__restrict__ tw, int t)
{
    using S = FftShape<N, R>;
    if constexpr (PASS < S::NPASS) {
        constexpr int Rp = (PASS < S::NFULL) ? R : S::RL;
        constexpr int Q = R / Rp;
        constexpr int Ns = 1 << (PASS * S::LGR);
        if constexpr (Ns > 1) {
            constexpr int stride = N / (Ns * Rp);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int j = (t + q * S::T) & (Ns - 1);
                p.w[PASS][q][0] = tw[j * stride];
                if constexpr (Rp > 2) p.w[PASS][q][1] = tw[2 * j * stride];
                if constexpr (Rp > 4) p.w[PASS][q][2] = tw[4 * j * stride];
            }
        }
        tw_preload<N, R, PASS + 1>(p, tw, t);
    }
}

// fft_pass with the twiddles taken from a TwPre (same arithmetic).
template <int N, int R, bool INV, int PASS, typename C, typename View>
__device__ __forceinline__ void fft_pass_pre(C (&v)[R], const View &lds, int t, const TwPre<N, R, C> &tp)
{
    using S = FftShape<N, R>;
    if constexpr (PASS < S::NPASS) {
        constexpr int Rp = (PASS < S::NFULL) ? R : S::RL;
        constexpr int Q = R / Rp;
        constexpr int Ns = 1 << (PASS * S::LGR);
        constexpr int T = S::T;
        constexpr bool LAST = (PASS == S::NPASS - 1);
        static_assert(Rp <= 8, "power-of-two twiddle reconstruction is written for radix <= 8");
        if constexpr (PASS > 0) {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = lds.template ld<C>(t + m * T);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            C a[Rp];
#pragma unroll
            for (int r = 0; r < Rp; ++r) a[r] = v[q + r * Q];
            if constexpr (Ns > 1) {
                C w[Rp];
                w[1] = tp.w[PASS][q][0];
                if constexpr (Rp > 2) w[2] = tp.w[PASS][q][1];
                if constexpr (Rp > 4) w[4] = tp.w[PASS][q][2];
                if constexpr (Rp > 2) w[3] = cmul(w[1], w[2]);
                if constexpr (Rp > 4) {
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
#pragma unroll
                for (int r = 1; r < Rp; ++r) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
            }
            Dft<Rp, INV, C>::run(a);
#pragma unroll
            for (int r = 0; r < Rp; ++r) v[q + r * Q] = a[r];
        }
        if constexpr (!LAST) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int u = t + q * T;
                const int j = u & (Ns - 1);
                const int base = (u / Ns) * Ns * Rp + j;
#pragma unroll
                for (int r = 0; r < Rp; ++r) lds.st(base + r * Ns, v[q + r * Q]);
            }
            __syncthreads();
            fft_pass_pre<N, R, INV, PASS + 1>(v, lds, t, tp);
        }
    }
}

template <int N, int R, bool INV, typename C, typename View>
__device__ __forceinline__ void fft_line_pre(C (&v)[R], const View &lds, int t, const TwPre<N, R, C> &tp)
{
    fft_pass_pre<N, R, INV, 0>(v, lds, t, tp);
}

// Two lines transformed together (same length, same direction, same twiddles): the
// twiddles are read once and applied to both, the exchanges of both lines share their
// barriers.  Used by the adjoint passes (state and adjoint move through the same
// transforms).  lds_b must not overlap lds_a.
template <int N, int R, bool INV, int PASS, typename C, typename View>
__device__ __forceinline__ void fft_pass2(C (&v)[R], C (&u)[R], const View &la, const View &lb, int t,
                                          const C *__restrict__ tw)
{
    using S = FftShape<N, R>;
    if constexpr (PASS < S::NPASS) {
        constexpr int Rp = (PASS < S::NFULL) ? R : S::RL;
        constexpr int Q = R / Rp;
        constexpr int Ns = 1 << (PASS * S::LGR);
        constexpr int T = S::T;
        constexpr bool LAST = (PASS == S::NPASS - 1);
        if constexpr (PASS > 0) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                v[m] = la.template ld<C>(t + m * T);
                u[m] = lb.template ld<C>(t + m * T);
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int uu = t + q * T;
            const int j = uu & (Ns - 1);
            C a[Rp], b[Rp];
#pragma unroll
            for (int r = 0; r < Rp; ++r) {
                a[r] = v[q + r * Q];
                b[r] = u[q + r * Q];
            }
            if constexpr (Ns > 1) {
                constexpr int stride = N / (Ns * Rp);
#pragma unroll
                for (int r = 1; r < Rp; ++r) {
                    C w = tw[r * j * stride];
                    a[r] = INV ? cmulc(a[r], w) : cmul(a[r], w);
                    b[r] = INV ? cmulc(b[r], w) : cmul(b[r], w);
                }
            }
            Dft<Rp, INV, C>::run(a);
            Dft<Rp, INV, C>::run(b);
#pragma unroll
            for (int r = 0; r < Rp; ++r) {
                v[q + r * Q] = a[r];
                u[q + r * Q] = b[r];
            }
        }
        if constexpr (!LAST) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int uu = t + q * T;
                const int j = uu & (Ns - 1);
                const int base = (uu / Ns) * Ns * Rp + j;
#pragma unroll
                for (int r = 0; r < Rp; ++r) {
                    la.st(base + r * Ns, v[q + r * Q]);
                    lb.st(base + r * Ns, u[q + r * Q]);
                }
            }
            __syncthreads();
            fft_pass2<N, R, INV, PASS + 1>(v, u, la, lb, t, tw);
        }
    }
}

template <int N, int R, bool INV, typename C, typename View>
__device__ __forceinline__ void fft_line2(C (&v)[R], C (&u)[R], const View &la, const View &lb, int t,
                                          const C *__restrict__ tw)
{
    fft_pass2<N, R, INV, 0>(v, u, la, lb, t, tw);
}

// LDS accessors: ld<C>(i) / st(i, v) convert between the arithmetic type C and the
// storage element type S (double2 or float2).
template <typename S, typename C> __device__ __forceinline__ S to_store(C v)
{
    using E = decltype(S{}.x);
    return {(E)v.x, (E)v.y};
}

// Contiguous line with one spare slot every 2^SH points, which keeps the stride-R
// writes of the first pass (R = 2^SH) off a single bank group.
template <typename S, int SH> struct LinePad {
    S *base;
    template <typename C> __device__ __forceinline__ C ld(int i) const
    {
        S s = base[i + (i >> SH)];
        return {s.x, s.y};
    }
    template <typename C> __device__ __forceinline__ void st(int i, C v) const
    {
        base[i + (i >> SH)] = to_store<S>(v);
    }
    static constexpr int words(int n) { return n + (n >> SH); }
};

// Interleaved lines of a tile: element i of line c at base[c + i*W + (i >> SH)], W
// lines side by side (lanes that differ in c touch neighbouring words).
template <typename S, int SH> struct LineTile {
    S *base;  // already offset by the line index c
    int w;
    template <typename C> __device__ __forceinline__ C ld(int i) const
    {
        S s = base[i * w + (i >> SH)];
        return {s.x, s.y};
    }
    template <typename C> __device__ __forceinline__ void st(int i, C v) const
    {
        base[i * w + (i >> SH)] = to_store<S>(v);
    }
    static constexpr int words(int n, int w) { return n * w + (n >> SH) + w; }
};

// Strided line inside a 2D grid held in LDS (row pitch or column stride).
template <typename S> struct LineStride {
    S *base;
    int stride;
    template <typename C> __device__ __forceinline__ C ld(int i) const
    {
        S s = base[i * stride];
        return {s.x, s.y};
    }
    template <typename C> __device__ __forceinline__ void st(int i, C v) const
    {
        base[i * stride] = to_store<S>(v);
    }
};

}  // namespace gpe
