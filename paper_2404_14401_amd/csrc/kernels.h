#pragma once
// kernels.h -- device code of the split-step GPE path shared by the kernel sources
// (kernels_plan.hip, kernels_batch.hip, kernels_adj.hip): pass bodies and kernel templates.
//
// Multi-pass path (any size): a step is a row pass and a column pass over the caller's
// complex64 array, updated in place.  Between passes the array holds the x-transformed
// field; only the first and last pass of a call see real space.
//   row entry : psi -> half kick at t_n -> FFT_x                         (Sec. 3.1, Eq. 4)
//   column    : FFT_y -> kinetic factor e^{-i k^2 dt/2}/(NxNy) -> IFFT_y  (Sec. 3.1)
//   row mid   : IFFT_x -> the two half kicks of t_{n+1} merged -> FFT_x  (real time: a
//               phase kick leaves |psi| unchanged, so the second half kick of step n and
//               the first of step n+1 see the same density; Sec. 3.1 "most recent psi")
//   row exit  : IFFT_x -> half kick at t_{n+1} -> psi
// Imaginary time (Sec. 3.3) cannot merge the kicks (the renormalisation sits between
// them), so each step is entry, column, exit, plus a one-work-group reduction.
// Reductions (norm, cavity overlap Theta, moments) are fused into the row passes as
// per-work-group partials, reduced in a fixed order by work-group 0 of the next column
// pass (or by the tail kernel), which also advances the cavity field.
//
// LDS path (nx ny <= 16384): the whole grid stays in one work-group's LDS for all steps.
#include <hip/hip_ext.h>

#include "fft_engine.h"
#include "physics.h"

namespace gpe {

// Points per thread of the multi-pass kernels (radix of the Stockham passes) and the
// element type of the LDS exchanges between passes.
#ifndef GPE_RADIX
#define GPE_RADIX 8
#endif
#ifndef GPE_XCHG_FLOAT
#define GPE_XCHG_FLOAT 1
#endif
#ifndef GPE_ADJ_TW_LDS
#define GPE_ADJ_TW_LDS 1
#endif
// host-side helper defined with the plan's launchers (threads of an LDS-resident grid)
int lds_threads(int nx, int ny);

constexpr int kRadix = GPE_RADIX;
constexpr int kLgR = ilog2(GPE_RADIX);
#if GPE_XCHG_FLOAT
using XchgT = float2;
#else
using XchgT = double2;
#endif

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) / 16 * 16; }

#ifndef GPE_NT_STORE
#define GPE_NT_STORE 0
#endif
// Store of one complex64 result of a pass.  The non-temporal form streams the line
// past L2 (it is read next by work-groups on other XCDs), leaving no dirty L2 lines
// for the end-of-kernel write-back.
__device__ __forceinline__ void store_c64(float2 *p, double2 v)
{
    const float2 f = make_float2((float)v.x, (float)v.y);
#if GPE_NT_STORE
    union {
        float2 f;
        unsigned long long u;
    } cv;
    cv.f = f;
    __builtin_nontemporal_store(cv.u, (unsigned long long *)p);
#else
    *p = f;
#endif
}



// --------------------------------------------------------------------- row pass
// Phase factors exp(-i th[m]) on every point of a thread.  When every phase of the
// wave is small, the short polynomial runs for all points in one straight block (a
// wave-uniform branch: no per-point control flow, so no load or wait is held behind
// it); otherwise each point takes its own range of sincos_d.  Same values either way.
template <int R> __device__ __forceinline__ void kick_real_all(double2 (&v)[R], const double (&th)[R])
{
#if GPE_FAST_KICK
    bool small = true;
#pragma unroll
    for (int m = 0; m < R; ++m) small = small && fabs(th[m]) < 0.0625;
    if (__all(small)) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            double sn, cs;
            sincos_small(th[m], &sn, &cs);
            v[m] = {v[m].x * cs + v[m].y * sn, v[m].y * cs - v[m].x * sn};
        }
        return;
    }
#endif
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = kick_real(v[m], th[m]);
}

// One work-group transforms `lines` rows.  `row` is this thread's row; the caller has
// placed `smem` (the exchange lines).  Lines of kPreloadLine points (PRE) issue every
// load the body will need -- the state, the per-point x tables, the user potential and
// the twiddles of all transform passes -- before any arithmetic, so that the latencies of
// the tables overlap that of the state, and kick all points in one straight block.  This
// holds ~80 more registers (two waves per SIMD instead of three); measured on the MI355X
// it pays for 1024-point lines in batches (12% on four 1024^2 grids) and costs at other
// lengths (256 and 512: -19% on the mixed 208-member batch; 4096: -12%), which load
// tables and twiddles where they are used.  Same arithmetic either way.
constexpr int kPreloadLine = 1024;
#ifndef GPE_PROBE_DEPTH
#define GPE_PROBE_DEPTH 4
#endif
template <int N, int R, int MODE, bool IMAG>
__device__ __forceinline__ void row_body(const float2 *__restrict__ src_base, float2 *dst_base, const GridDev &gd,
                                         const PotDev &pot, DevState *st, double *partials, int n, int lb,
                                         int lines, XchgT *smem, double *red, double t_shift = 0.0,
                                         const double *probe = nullptr, int nprobe = 0, bool theta_only = false,
                                         float2 *traj = nullptr, const double *scale_partials = nullptr,
                                         int nscale = 0)
{
    using C = double2;
    constexpr int T = N / R;
    using View = LinePad<XchgT, ilog2(R)>;
    constexpr bool PRE = N == kPreloadLine;
    constexpr bool PROBE = MODE == ROW_PROBE_REAL || MODE == ROW_PROBE_MID;
    constexpr bool USES_V = !PROBE && MODE != ROW_INV;  // kicks and the energy pass
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int row = lb * lines + line;
    View lds{smem + line * View::words(N)};
    const float2 *src = src_base + (size_t)row * N;
    float2 *dst = dst_base + (size_t)row * N;

    float2 f[R];
#pragma unroll
    for (int m = 0; m < R; ++m) f[m] = src[t + m * T];
    C v[R];
    const float *vup = pot.vuser ? pot.vuser + (size_t)row * N : nullptr;
    const bool has_vu = USES_V && vup != nullptr;
    float4 tx[R];
    float vu[R];
    TwPre<N, R, C> tp;
    if constexpr (PRE) {
        if constexpr (MODE != ROW_INV)
#pragma unroll
            for (int m = 0; m < R; ++m) tx[m] = pot.tx[t + m * T];
        if (has_vu)
#pragma unroll
            for (int m = 0; m < R; ++m) vu[m] = vup[t + m * T];
        if constexpr (MODE != ROW_PROBE_REAL) tw_preload<N, R, 0>(tp, gd.tw_x, t);
    }
    // the transforms: twiddles from registers (PRE) or from the table
    auto fft_inv = [&]() {
        if constexpr (PRE) fft_line_pre<N, R, true>(v, lds, t, tp);
        else fft_line<N, R, true>(v, lds, t, gd.tw_x);
    };
    auto fft_fwd = [&]() {
        if constexpr (PRE) fft_line_pre<N, R, false>(v, lds, t, tp);
        else fft_line<N, R, false>(v, lds, t, gd.tw_x);
    };
    auto tx_at = [&](int m) -> float4 {
        if constexpr (PRE) return tx[m];
        else return pot.tx[t + m * T];
    };
    const float4 ty = pot.ty[row];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = {(double)f[m].x, (double)f[m].y};

    const double cy = ty.z, yv = ty.w;
    if constexpr (PROBE) {
        // integrals of the density about to be kicked: norm, Theta, C
        if constexpr (MODE == ROW_PROBE_MID) fft_inv();
        double part[NPART] = {};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const double cx = tx_at(m).z;
            const double d = v[m].x * v[m].x + v[m].y * v[m].y;
            part[0] += d;
            part[1] += cx * cy * d;
            part[4] += cx * cx * d;
        }
        block_sum<NPART>(part, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) partials[k] = part[k];
        return;
    }

    if constexpr (MODE == ROW_INV) {
        fft_inv();
#pragma unroll
        for (int m = 0; m < R; ++m) store_c64(dst + t + m * T, v[m]);
        return;
    }
    // kick time: t_n for the entry kick, t_{n+1} for the others; imaginary time freezes
    // V; the energy pass evaluates V at the call's own time
    double tk = st->t0;
    if (!IMAG && MODE != ROW_FWD) tk += (MODE == ROW_ENTRY ? n : n + 1) * gd.dt + t_shift;
    double are, aim;
    // (probe partials reach the real-time kicks only: other modes keep their registers)
    constexpr int KD = (!IMAG && MODE != ROW_FWD) ? GPE_PROBE_DEPTH : 1;
    if (probe) {
        // adiabatic field of the probed density, the same sum in every work-group, of the
        // three integrals it needs (norm, Theta, C)
        double s[3] = {};
        strided_sum<KD>(probe, nprobe, NPART, {0, 1, 4}, s);
        block_sum<3>(s, red);
        if (threadIdx.x == 0) alpha_adiabatic(pot, tk, s[0], s[1], s[2], &red[0], &red[1]);
        __syncthreads();
        are = red[0];
        aim = red[1];
        __syncthreads();
        if (lb == 0 && threadIdx.x == 0) {
            st->alpha_re = are;
            st->alpha_im = aim;
        }
    } else {
        are = st->alpha_re;
        aim = st->alpha_im;
    }
    const VLine vl = vline_cav(pot, row, tk, are, aim);

    if constexpr (MODE == ROW_MID || MODE == ROW_EXIT) fft_inv();

    double part[NPART] = {};
    double fin = 0.0;  // sum of this thread's densities: non-finite iff one of its points is
    if constexpr (MODE == ROW_ENTRY && IMAG) {
        // the pending renormalisation: 1/sqrt(norm) of the previous step's exit state,
        // from its partials (the same fixed-order sum in every work-group) or the state
        double sc;
        if (scale_partials) {
            double s1[1] = {0.0};
            strided_sum(scale_partials, nscale, NPART, {0}, s1);
            block_sum<1>(s1, red);
            if (threadIdx.x == 0) red[0] = sqrt(1.0 / (s1[0] * gd.dA));
            __syncthreads();
            sc = red[0];
            __syncthreads();
        } else {
            sc = st->scale;
        }
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = {v[m].x * sc, v[m].y * sc};
    }
    const double hk = (MODE == ROW_MID) ? gd.dt : 0.5 * gd.dt;
    double th[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const float4 tm = tx_at(m);
        double V = vpoint(vl, tm);
        if (has_vu) V += (double)(PRE ? vu[m] : vup[t + m * T]);
        const double d = v[m].x * v[m].x + v[m].y * v[m].y;
        fin += d;
        if constexpr (MODE == ROW_FWD) {
            part[0] += d;
            part[1] += V * d;
            part[2] += d * d;
        } else {
            th[m] = (V + gd.g * d) * hk;
            if constexpr (IMAG) {
                v[m] = kick_imag(v[m], th[m]);
                if (MODE == ROW_EXIT) {
                    const double d2 = v[m].x * v[m].x + v[m].y * v[m].y;
                    part[0] += d2;
                    part[1] += (double)tm.z * cy * d2;
                    part[2] += (double)tm.w * d2;
                    part[3] += yv * d2;
                    if (pot.cavity == 2) part[4] += (double)tm.z * tm.z * d2;
                }
            } else {
                // |psi| is the same before and after a phase kick
                part[1] += (double)tm.z * cy * d;
                if (!theta_only) {
                    part[0] += d;
                    part[2] += (double)tm.w * d;
                    part[3] += yv * d;
                    if (pot.cavity == 2) part[4] += (double)tm.z * tm.z * d;
                }
                if constexpr (!PRE) v[m] = kick_real(v[m], th[m]);
            }
        }
    }
    if constexpr (MODE != ROW_FWD && !IMAG && PRE) kick_real_all<R>(v, th);
    // every kicking pass flags a non-finite input, whether or not it reduces anything
    // (a plain store of the same value from any work-group: no atomics needed)
    if constexpr (MODE != ROW_FWD)
        if (!isfinite(fin)) st->nonfinite = 1;
    if constexpr (!IMAG && (MODE == ROW_ENTRY || MODE == ROW_MID)) {
        // the adjoint's stored trajectory: this kick's output in real space
        if (traj)
#pragma unroll
            for (int m = 0; m < R; ++m) store_c64(traj + (size_t)row * N + t + m * T, v[m]);
    }
    if (partials) {
        // the C overlap is only needed by the adiabatic field, and the field ODE alone
        // needs only Theta: skip the other sums' shuffles
        if (theta_only)
            block_sum<1>(*reinterpret_cast<double(*)[1]>(part + 1), red);
        else if (pot.cavity == 2)
            block_sum<NPART>(part, red);
        else
            block_sum<NPART - 1>(*reinterpret_cast<double(*)[NPART - 1]>(part), red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) partials[k] = part[k];
    }

    if constexpr (MODE != ROW_EXIT) fft_fwd();

#pragma unroll
    for (int m = 0; m < R; ++m) store_c64(dst + t + m * T, v[m]);
}

// Points per thread of the plan's row passes: kRadix, except for 8192-point lines, whose
// 512 threads at radix 16 stay within the row pass's 512-thread bound (radix 8 would need
// 1024 threads, which caps a thread at 128 registers; the fused row pass holds more).
template <int N> constexpr int kRowRadix = N >= 8192 ? 16 : kRadix;

template <int N, int MODE, bool IMAG>
__global__ void __launch_bounds__(512) row_pass(RowArgs a)
{
    extern __shared__ XchgT smem[];
    __shared__ double red[8 * NPART];
    row_body<N, kRowRadix<N>, MODE, IMAG>(a.src, a.dst, a.grid, a.pot, a.st,
                                          a.reduce ? a.partials + blockIdx.x * NPART : nullptr, a.n, blockIdx.x,
                                          a.lines_per_wg, smem, red, a.t_shift, a.probe, a.nprobe, a.reduce == 2,
                                          nullptr, a.scale_partials, a.nscale);
}

// Batched: work-group b serves instance b / blocks_per_inst (real time, no reductions).
// A member with the adiabatic field carries probe partials: the probe modes write them,
// the kick modes turn them into alpha; other members skip the probe modes.
// (CAV is a template flag so that groups without a cavity field keep the kernel without
// probe sums and reductions; TRAJ likewise for the adjoint's forward sweep that records
// every kick's output.)
template <int N, int R, int MODE, bool CAV, bool TRAJ>
__global__ void __launch_bounds__(512) row_pass_b(BatchPassArgs a)
{
    extern __shared__ XchgT smem[];
    __shared__ double red[8 * NPART];
    const InstDesc &I = a.inst[blockIdx.x / a.blocks_per_inst];
    const int lb = blockIdx.x % a.blocks_per_inst;
    // kick k's output goes to trajectory slot k (entry kick k = 0, merged kick of step n: n + 1)
    float2 *tj = nullptr;
    if constexpr (TRAJ && (MODE == ROW_ENTRY || MODE == ROW_MID))
        tj = I.traj + (size_t)(MODE == ROW_ENTRY ? 0 : a.n + 1) * ((size_t)I.grid.nx * I.grid.ny);
    if constexpr (MODE == ROW_PROBE_REAL || MODE == ROW_PROBE_MID) {
        if (!I.probe) return;
        row_body<N, R, MODE, false>(I.psi, I.psi, I.grid, I.pot, I.st, I.probe + lb * NPART, a.n, lb, a.per_wg, smem,
                                    red);
    } else if constexpr (CAV) {
        // adiabatic members take the field from their probe sums; field-ODE members reduce
        // Theta for the column pass's recurrence (the entry kick only when the history starts)
        double *pt = (I.partials && (MODE != ROW_ENTRY || I.first_theta)) ? I.partials + lb * NPART : nullptr;
        row_body<N, R, MODE, false>(I.psi, I.psi, I.grid, I.pot, I.st, pt, a.n, lb, a.per_wg, smem, red, 0.0,
                                    I.probe, a.blocks_per_inst, true, tj);
    } else {
        row_body<N, R, MODE, false>(I.psi, I.psi, I.grid, I.pot, I.st, nullptr, a.n, lb, a.per_wg, smem, red, 0.0,
                                    nullptr, 0, false, tj);
    }
}

// ------------------------------------------------------------------ column pass
template <int N, int R, int MODE>
__device__ __forceinline__ void col_body(const float2 *__restrict__ src, float2 *dst, const GridDev &gd,
                                         double *partials, int tile, int w, XchgT *smem, double *red,
                                         double scale = 1.0)
{
    using C = double2;
    constexpr int T = N / R;
    using View = LineTile<XchgT, ilog2(R)>;
    const int c = threadIdx.x % w, t = threadIdx.x / w;
    const int col = tile * w + c;
    const int nx = gd.nx;
    View lds{smem + c, w};
    const double2 *twy = gd.tw_y;
    const double2 *kiny = gd.kin_y;

    C v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        float2 f = src[(size_t)(t + m * T) * nx + col];
        v[m] = {(double)f.x, (double)f.y};
    }
    if constexpr (MODE == COL_KHALF_INV || MODE == COL_KHALF_INV_IM) {
        // Fourier-space state: kinetic half step (imaginary time: with the pending
        // renormalisation), then back to real space along y
        if constexpr (MODE == COL_KHALF_INV) {
            const C kx = gd.kh_x[col];
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = cmul(v[m], cmul(kx, gd.kh_yin[t + m * T]));
        } else {
            const double kx = gd.khi_x[col] * scale;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const double f = kx * gd.khi_yin[t + m * T];
                v[m] = {v[m].x * f, v[m].y * f};
            }
        }
        fft_line<N, R, true>(v, lds, t, twy);
#pragma unroll
        for (int m = 0; m < R; ++m) store_c64(dst + (size_t)(t + m * T) * nx + col, v[m]);
        return;
    }
    fft_line<N, R, false>(v, lds, t, twy);
    if constexpr (MODE == COL_FWD_KHALF) {
        const C kx = gd.kh_x[col];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            v[m] = cmul(v[m], cmul(kx, gd.kh_yout[t + m * T]));
            store_c64(dst + (size_t)(t + m * T) * nx + col, v[m]);
        }
        return;
    }
    if constexpr (MODE == COL_FWD_KHALF_IM) {
        // kinetic half step, then the norm by Parseval: sum |psi_k|^2 / (nx ny) per work-group
        const double kx = gd.khi_x[col];
        double part[NPART] = {};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const double f = kx * gd.khi_yout[t + m * T];
            v[m] = {v[m].x * f, v[m].y * f};
            part[0] += v[m].x * v[m].x + v[m].y * v[m].y;
            store_c64(dst + (size_t)(t + m * T) * nx + col, v[m]);
        }
        part[0] *= 1.0 / ((double)gd.nx * gd.ny);
        block_sum<1>(*reinterpret_cast<double(*)[1]>(part), red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) partials[k] = part[k];
        return;
    }
    if constexpr (MODE == COL_KIN_APPLY) {
        // the kinetic operator |k|^2/2 applied in Fourier space (its expectation reduced on
        // the way), then back along y; the 1/(nx ny) of the round trip is folded in
        const int ix = col >= nx / 2 ? col - nx : col;
        const double kx = 2.0 * M_PI * ix / gd.lx;
        const double inv = 1.0 / ((double)gd.nx * gd.ny);
        double part[NPART] = {};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int j = t + m * T;
            const int iy = j >= N / 2 ? j - N : j;
            const double ky = 2.0 * M_PI * iy / gd.ly;
            const double e = 0.5 * (kx * kx + ky * ky);
            part[0] += e * (v[m].x * v[m].x + v[m].y * v[m].y);
            v[m] = {v[m].x * e * inv, v[m].y * e * inv};
        }
        block_sum<1>(*reinterpret_cast<double(*)[1]>(part), red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) partials[k] = part[k];
        fft_line<N, R, true>(v, lds, t, twy);
#pragma unroll
        for (int m = 0; m < R; ++m) store_c64(dst + (size_t)(t + m * T) * nx + col, v[m]);
        return;
    }
    if constexpr (MODE == COL_EKIN) {
        const int ix = col >= nx / 2 ? col - nx : col;
        const double kx = 2.0 * M_PI * ix / gd.lx;
        double part[NPART] = {};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int j = t + m * T;
            const int iy = j >= N / 2 ? j - N : j;
            const double ky = 2.0 * M_PI * iy / gd.ly;
            part[0] += 0.5 * (kx * kx + ky * ky) * (v[m].x * v[m].x + v[m].y * v[m].y);
        }
        block_sum<NPART>(part, red);
        if (threadIdx.x == 0) partials[0] = part[0];
        return;
    } else {
        if constexpr (MODE == COL_KIN_REAL) {
            const C kx = gd.kin_x[col];
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = cmul(v[m], cmul(kx, kiny[t + m * T]));
        } else {
            const double kx = gd.kim_x[col];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const double f = kx * gd.kim_y[t + m * T];
                v[m] = {v[m].x * f, v[m].y * f};
            }
        }
        fft_line<N, R, true>(v, lds, t, twy);
#pragma unroll
        for (int m = 0; m < R; ++m) store_c64(dst + (size_t)(t + m * T) * nx + col, v[m]);
    }
}

// Work-groups are dealt round-robin to the 8 XCDs; with the swizzle, the tiles of one
// XCD are contiguous, so the 128-byte lines shared by neighbouring tiles are fetched
// once into that XCD's L2.
__device__ __forceinline__ int xcd_tile(int swz)
{
    return swz ? (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : (int)blockIdx.x;
}

template <int N, int MODE>
__global__ void __launch_bounds__(1024) col_pass(ColArgs a)
{
    extern __shared__ XchgT smem[];
    __shared__ double red[16 * NPART];
    if (a.do_tail && blockIdx.x == 0) run_tail(a.tail, a.grid, a.pot, a.st, red);
    const double sc = MODE == COL_KHALF_INV_IM ? a.st->scale : 1.0;
    col_body<N, kRadix, MODE>(a.src, a.dst, a.grid, a.partials + blockIdx.x * NPART, xcd_tile(a.xcd_swizzle),
                              a.cols_per_wg, smem, red, sc);
}

template <int N, int R, bool ODE>
__global__ void __launch_bounds__(1024) col_pass_b(BatchPassArgs a)
{
    extern __shared__ XchgT smem[];
    __shared__ double red[16 * NPART];
    const int tile = xcd_tile(a.xcd_swizzle);
    const InstDesc &I = a.inst[tile / a.blocks_per_inst];
    const int lt = tile % a.blocks_per_inst;
    if constexpr (ODE) {
        if (lt == 0 && I.partials) {
            // this member's cavity field: Theta of the last kick into the overlap history
            // (at a call's first step only when the history starts), then alpha_{n+1}
            TailArgs ta{};
            ta.partials = I.partials;
            ta.npartials = (a.first && !I.first_theta) ? 0 : a.row_blocks;
            ta.first_theta = (a.first && I.first_theta) ? 1 : 0;
            ta.theta_only = 1;
            ta.advance_alpha = 1;
            run_tail(ta, I.grid, I.pot, I.st, red);
        }
    }
    col_body<N, R, COL_KIN_REAL>(I.psi, I.psi, I.grid, nullptr, lt, a.per_wg, smem, red);
}


// ------------------------------------------------- long columns in three passes
// The column step on lines of NY = NA * NB points as a four-step transform (k = k2 + NA k1,
// n = n1 + NB n2), so that every pass moves whole 128-byte lines where a single pass would
// hold a one-column tile and fetch each line once per column:
//   PHASE 0: for a residue n1 < NB, the NA-point transform of rows n1 + NB n2 (over n2),
//            times W_NY^{n1 k2}, back to row n1 + NB k2;
//   PHASE 1: for a k2 < NA, the NB-point transform of the NB contiguous rows NB k2 + n1
//            (over n1, output index k1 = frequency k2 + NA k1), the kinetic factor, the
//            inverse NB-point transform, back in place;
//   PHASE 2: for a residue n1, times W_NY^{-n1 k2}, the inverse NA-point transform over
//            k2, back to rows n1 + NB n2.
// The sub-transforms take every (NY/NA)-th or (NY/NB)-th twiddle of the line's table.
// Work-group b: tile b % (nx / w) of w columns, group (n1 or k2) b / (nx / w); work-group
// 0 of PHASE 0 runs the tail, as the single column pass does.
constexpr int kSplitA = 128;
template <int NY, int PHASE, int MODE>
__global__ void __launch_bounds__(256) col_split(ColArgs a)
{
    using C = double2;
    constexpr int NA = kSplitA, NB = NY / NA, R = kRadix;
    constexpr int N = PHASE == 1 ? NB : NA;
    constexpr int T = N / R;
    using View = LineTile<XchgT, ilog2(R)>;
    extern __shared__ XchgT smem[];
    __shared__ double red[16 * NPART];
    if (PHASE == 0 && a.do_tail && blockIdx.x == 0) run_tail(a.tail, a.grid, a.pot, a.st, red);
    const GridDev &gd = a.grid;
    const int nx = gd.nx, w = a.cols_per_wg;
    const int ntiles = nx / w;
    const int tile = blockIdx.x % ntiles, grp = blockIdx.x / ntiles;
    const int c = threadIdx.x % w, t = threadIdx.x / w;
    const int col = tile * w + c;
    View lds{smem + c, w};
    const double2 *tw = gd.tw_y;
    // row of element j of this work-group's line
    auto row = [&](int j) -> size_t { return PHASE == 1 ? (size_t)NB * grp + j : (size_t)grp + (size_t)NB * j; };

    C v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const float2 f = a.src[row(t + m * T) * nx + col];
        v[m] = {(double)f.x, (double)f.y};
    }
    if constexpr (PHASE == 0) {
        fft_line<NA, R, false, NY / NA>(v, lds, t, tw);
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = cmul(v[m], tw[grp * (t + m * T)]);  // n1 k2 < NY
    } else if constexpr (PHASE == 1) {
        fft_line<NB, R, false, NY / NB>(v, lds, t, tw);
        if constexpr (MODE == COL_KIN_REAL) {
            const C kx = gd.kin_x[col];
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = cmul(v[m], cmul(kx, gd.kin_y[grp + NA * (t + m * T)]));
        } else {
            const double kx = gd.kim_x[col];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const double f = kx * gd.kim_y[grp + NA * (t + m * T)];
                v[m] = {v[m].x * f, v[m].y * f};
            }
        }
        fft_line<NB, R, true, NY / NB>(v, lds, t, tw);
    } else {
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = cmulc(v[m], tw[grp * (t + m * T)]);
        fft_line<NA, R, true, NY / NA>(v, lds, t, tw);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) store_c64(a.dst + row(t + m * T) * nx + col, v[m]);
}

// ------------------------------------------------------------- whole grid in LDS
// One work-group owns one grid for all steps; psi stays in LDS as complex64 (row pitch
// NX + 1), each transform line is lifted to double registers.  Steps follow the
// definition literally: half kick, FFT2, kinetic factor, IFFT2, half kick, then the
// reductions (imaginary time: renormalise; cavity: overlap and field update).  The
// launch uses exactly NX*NY/8 threads (at most 1024), so every thread owns a slice of
// a line in both the row and the column sweeps.
constexpr int kLdsRadix = 8;

// s0, nsteps: this launch runs steps s0 .. s0 + nsteps - 1 of the call (long batched
// calls are split into launches of bounded length; real-time kicks are timed from
// st->t0 + s0 dt).
template <int NX, int NY> __device__ __forceinline__ void lds_body(const LdsArgs &a, int64_t s0, int nsteps)
{
    using C = double2;
    constexpr int R = kLdsRadix;
    constexpr int TX = NX / R, TY = NY / R;
    constexpr int P = NX + 1;
    constexpr int NTH = (NX * NY / R) < 1024 ? NX * NY / R : 1024;
    constexpr int LR = NTH / TX, LC = NTH / TY;  // lines per sweep
    static_assert(LR <= NY && LC <= NX && NY % LR == 0 && NX % LC == 0, "sweep shape");
    extern __shared__ float2 g[];
    __shared__ double red[16 * NPART];
    __shared__ double bc[NPART];
    __shared__ double s_scale, s_are, s_aim, s_th, s_thp;

    const GridDev &gd = a.grid;
    const PotDev &pot = a.pot;
    DevState *st = a.st;
    const int rl = threadIdx.x % LR, rt = threadIdx.x / LR;
    const int cl = threadIdx.x % LC, ct = threadIdx.x / LC;
    const bool cav = pot.cavity == 1 && !a.imag;  // field ODE (real time only)
    const bool adia = pot.cavity == 2;             // adiabatic field, both times
    const bool want = cav || adia || a.obs != nullptr || a.imag;
    const double t0 = a.imag ? st->t0 : st->t0 + (double)s0 * gd.dt;

    for (int i = threadIdx.x; i < NX * NY; i += NTH) g[(i / NX) * P + (i % NX)] = a.psi[i];
    if (threadIdx.x == 0) {
        s_scale = 1.0;
        s_are = st->alpha_re;
        s_aim = st->alpha_im;
        s_th = st->theta;
        s_thp = st->theta_prev;
    }
    __syncthreads();

    // sum NPART per-thread values over the work-group, times dA, broadcast to all
    auto reduce_all = [&](double (&part)[NPART]) {
        block_sum<NPART>(part, red);
        if (threadIdx.x == 0)
            for (int k = 0; k < NPART; ++k) bc[k] = part[k] * gd.dA;
        __syncthreads();
        for (int k = 0; k < NPART; ++k) part[k] = bc[k];
        __syncthreads();
    };
    // one half kick over the grid (optionally scaling first and reducing after)
    auto kick_rows = [&](double tk, double are, double aim, double sc, bool reduce, double (&part)[NPART]) {
        for (int r0 = 0; r0 < NY; r0 += LR) {
            const int row = r0 + rl;
            const VLine vl = vline_cav(pot, row, tk, are, aim);
            const float4 ty = pot.ty[row];
            for (int m = 0; m < R; ++m) {
                const int i = rt + m * TX;
                const float4 tx = pot.tx[i];
                float2 f = g[row * P + i];
                C p = {(double)f.x * sc, (double)f.y * sc};
                double V = vpoint(vl, tx);
                if (pot.vuser) V += (double)pot.vuser[row * NX + i];
                const double th = (V + gd.g * (p.x * p.x + p.y * p.y)) * (0.5 * gd.dt);
                p = a.imag ? kick_imag(p, th) : kick_real(p, th);
                if (reduce) {
                    const double d2 = p.x * p.x + p.y * p.y;
                    part[0] += d2;
                    part[1] += (double)tx.z * (double)ty.z * d2;
                    part[2] += (double)tx.w * d2;
                    part[3] += (double)ty.w * d2;
                    part[4] += (double)tx.z * (double)tx.z * d2;
                }
                g[row * P + i] = make_float2((float)p.x, (float)p.y);
            }
        }
    };
    auto rows_fft = [&](auto inv_tag) {
        constexpr bool INV = decltype(inv_tag)::value;
        for (int r0 = 0; r0 < NY; r0 += LR) {
            LineStride<float2> view{g + (r0 + rl) * P, 1};
            C v[R];
            for (int m = 0; m < R; ++m) v[m] = view.template ld<C>(rt + m * TX);
            fft_line<NX, R, INV>(v, view, rt, gd.tw_x);
            __syncthreads();
            for (int m = 0; m < R; ++m) view.st(rt + m * TX, v[m]);
            __syncthreads();
        }
    };
    auto cols_kin = [&]() {
        for (int c0 = 0; c0 < NX; c0 += LC) {
            const int col = c0 + cl;
            LineStride<float2> view{g + col, P};
            C v[R];
            for (int m = 0; m < R; ++m) v[m] = view.template ld<C>(ct + m * TY);
            fft_line<NY, R, false>(v, view, ct, gd.tw_y);
            if (!a.imag) {
                const C kx = gd.kin_x[col];
                for (int m = 0; m < R; ++m) v[m] = cmul(v[m], cmul(kx, gd.kin_y[ct + m * TY]));
            } else {
                const double kx = gd.kim_x[col];
                for (int m = 0; m < R; ++m) {
                    const double f = kx * gd.kim_y[ct + m * TY];
                    v[m] = {v[m].x * f, v[m].y * f};
                }
            }
            fft_line<NY, R, true>(v, view, ct, gd.tw_y);
            __syncthreads();
            for (int m = 0; m < R; ++m) view.st(ct + m * TY, v[m]);
            __syncthreads();
        }
    };

    // adiabatic field of the density now in LDS (norm, Theta, C), at time tk
    auto probe_alpha = [&](double tk) {
        double part[NPART] = {};
        for (int r0 = 0; r0 < NY; r0 += LR) {
            const int row = r0 + rl;
            const double cy = pot.ty[row].z;
            for (int m = 0; m < R; ++m) {
                const int i = rt + m * TX;
                const double cx = pot.tx[i].z;
                const float2 f = g[row * P + i];
                const double d = (double)f.x * f.x + (double)f.y * f.y;
                part[0] += d;
                part[1] += cx * cy * d;
                part[4] += cx * cx * d;
            }
        }
        block_sum<NPART>(part, red);
        if (threadIdx.x == 0) alpha_adiabatic(pot, tk, part[0], part[1], part[4], &s_are, &s_aim);
        __syncthreads();
    };
    if (adia) probe_alpha(t0);

    if (cav && !st->have_theta) {
        // Theta_0 starts the overlap history
        double part[NPART] = {};
        for (int r0 = 0; r0 < NY; r0 += LR) {
            const int row = r0 + rl;
            const double cy = pot.ty[row].z;
            for (int m = 0; m < R; ++m) {
                const int i = rt + m * TX;
                float2 f = g[row * P + i];
                part[1] += (double)pot.tx[i].z * cy * ((double)f.x * f.x + (double)f.y * f.y);
            }
        }
        reduce_all(part);
        if (threadIdx.x == 0) {
            s_th = part[1];
            s_thp = part[1];
        }
        __syncthreads();
    }

    for (int n = 0; n < nsteps; ++n) {
        const double tn = a.imag ? t0 : t0 + n * gd.dt;
        const double tn1 = a.imag ? t0 : t0 + (n + 1) * gd.dt;
        const double are0 = s_are, aim0 = s_aim, sc = s_scale;
        __syncthreads();
        if (cav && threadIdx.x == 0) {
            // alpha_{n+1} = e^{lambda dt} alpha_n + phi1 (-i eta (3 Theta_n - Theta_{n-1}) / 2)
            const double tb = 0.5 * (3.0 * s_th - s_thp);
            const double fi = -pot.eta * tb;
            const double nr = pot.ecav_re * are0 - pot.ecav_im * aim0 - pot.phi1_im * fi;
            const double ni = pot.ecav_re * aim0 + pot.ecav_im * are0 + pot.phi1_re * fi;
            s_are = nr;
            s_aim = ni;
        }
        double part[NPART] = {};
        kick_rows(tn, are0, aim0, sc, false, part);
        __syncthreads();
        rows_fft(std::integral_constant<bool, false>{});
        cols_kin();
        rows_fft(std::integral_constant<bool, true>{});
        if (adia && !a.imag) probe_alpha(tn1);  // real time: field of the density at t_{n+1}
        kick_rows(tn1, s_are, s_aim, 1.0, want, part);
        __syncthreads();
        if (want) {
            reduce_all(part);
            if (threadIdx.x == 0) {
                const double norm = part[0];
                if (!isfinite(norm)) st->nonfinite = 1;
                double *o = a.obs ? a.obs + (size_t)n * NOBS : nullptr;
                const double inv = a.imag ? 1.0 / norm : 1.0;
                if (a.imag) s_scale = sqrt(inv);
                if (cav) {
                    s_thp = s_th;
                    s_th = part[1];
                }
                if (o) {
                    o[0] = norm;
                    o[1] = part[1] * inv;
                    o[2] = s_are;
                    o[3] = s_aim;
                    o[4] = part[2] * inv;
                    o[5] = part[3] * inv;
                }
                // imaginary time: the field of the state just reduced drives the next step
                if (adia && a.imag) alpha_adiabatic(pot, t0, part[0], part[1], part[4], &s_are, &s_aim);
            }
            __syncthreads();
        }
    }
    const double sc = s_scale;
    double fin = 0.0;
    for (int i = threadIdx.x; i < NX * NY; i += NTH) {
        float2 f = g[(i / NX) * P + (i % NX)];
        fin += (double)f.x * f.x + (double)f.y * f.y;
        a.psi[i] = make_float2((float)(f.x * sc), (float)(f.y * sc));
    }
    // the state returned is checked even where no reduction ran during the steps
    if (!isfinite(fin)) st->nonfinite = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->alpha_re = s_are;
        st->alpha_im = s_aim;
        if (cav) {
            st->theta = s_th;
            st->theta_prev = s_thp;
            st->have_theta = 1;
        }
        st->scale = 1.0;
    }
}

template <int NX, int NY>
__global__ void __launch_bounds__((NX * NY / kLdsRadix) < 1024 ? NX * NY / kLdsRadix : 1024) lds_grid(LdsArgs a)
{
    lds_body<NX, NY>(a, 0, a.nsteps);
}

// Batched: work-group b runs member b of the batch for all steps.
template <int NX, int NY>
__global__ void __launch_bounds__((NX * NY / kLdsRadix) < 1024 ? NX * NY / kLdsRadix : 1024)
    lds_grid_b(const LdsArgs *arr, int64_t s0, int nsteps)
{
    lds_body<NX, NY>(arr[blockIdx.x], s0, nsteps);
}



// ------------------------------------------------------------- adjoint passes
// Reverse sweep of the real-time step for the discrete adjoint with respect to the
// x-lattice depth.  For a kick psi' = psi e^{-i theta}, theta = (V + g|psi|^2) tau,
// with real gradient G (dL = Re sum conj(G) d psi):
//   psi = psi' e^{+i theta}   (exact: |psi| = |psi'|),
//   s = Im(conj(G') psi'),  G = G' e^{+i theta} + 2 g tau s psi,  dL/dV(x) = tau s(x).
// The kinetic propagation U = IFFT2 M FFT2 is unitary, so both the state and G go
// back through U^H = IFFT2 conj(M) FFT2: the same passes with the conjugate factor.
// TRAJ: the kick outputs psi' were stored by the forward sweep (slot k for kick k, the
// last kick's output is psi(T) itself), so the passes transform lam alone.
template <int N, int R, int MODE, bool TRAJ>
__device__ __forceinline__ void row_adj_body(const AdjInst &I, int lb, int lines, int kick, XchgT *smem, double *red,
                                             int nprobe)
{
    using C = double2;
    constexpr int T = N / R;
    constexpr bool FIRST = MODE == ADJ_FIRST || MODE == ADJ_PROBE_FIRST;
    using View = LinePad<XchgT, ilog2(R)>;
    const GridDev &gd = I.grid;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int row = lb * lines + line;
    // exchange lines: [state lines][adjoint lines] (TRAJ: adjoint lines only), then the
    // staged tables
    constexpr int AREAS = TRAJ ? 1 : 2;
    View la{smem + line * View::words(N)};
    View lb2{smem + ((AREAS - 1) * lines + line) * View::words(N)};
#if GPE_ADJ_TW_LDS
    double2 *s_tw = (double2 *)((char *)smem + align16(AREAS * lines * View::words(N) * sizeof(XchgT)));
    float4 *s_tx = (float4 *)(s_tw + N);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        s_tw[i] = gd.tw_x[i];
        s_tx[i] = I.pot.tx[i];
    }
#else
    const double2 *s_tw = gd.tw_x;
    const float4 *s_tx = I.pot.tx;
#endif
    float2 *pp = I.psi + (size_t)row * N;
    float2 *pl = I.lam + (size_t)row * N;
    const float2 *ps = pp;
    if constexpr (TRAJ && !FIRST) ps = I.traj + (size_t)kick * ((size_t)N * gd.ny) + (size_t)row * N;
    C v[R], w[R];
    float2 vs[R];  // TRAJ: the stored state stays complex64 through lam's transform
#pragma unroll
    for (int m = 0; m < R; ++m) {
        float2 a = ps[t + m * T], b = pl[t + m * T];
        if constexpr (TRAJ) vs[m] = a;
        else v[m] = {(double)a.x, (double)a.y};
        w[m] = {(double)b.x, (double)b.y};
    }
    __syncthreads();
    if constexpr (!FIRST) {
        if constexpr (TRAJ)
            fft_line<N, R, true>(w, lb2, t, s_tw);
        else
            fft_line2<N, R, true>(v, w, la, lb2, t, s_tw);
    }
    if constexpr (TRAJ)
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = {(double)vs[m].x, (double)vs[m].y};
    const double cyc = I.pot.ty[row].z;  // cos(kc y) of this row
    if constexpr (MODE == ADJ_PROBE_FIRST || MODE == ADJ_PROBE_MID) {
        // sums for the adiabatic field and its adjoint: rho, rho cxcy, rho cc2, s cc2, s cxcy
        double part[NPART] = {};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const double cx = s_tx[t + m * T].z;
            const double d = v[m].x * v[m].x + v[m].y * v[m].y;
            const double s = w[m].x * v[m].y - w[m].y * v[m].x;
            part[0] += d;
            part[1] += cx * cyc * d;
            part[2] += cx * cx * d;
            part[3] += cx * cx * s;
            part[4] += cx * cyc * s;
        }
        block_sum<NPART>(part, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NPART; ++k) I.aprobe[lb * NPART + k] = part[k];
        return;
    }
    const double tk = I.st->t0 + kick * gd.dt;
    const double tau = (MODE == ADJ_MID) ? gd.dt : 0.5 * gd.dt;
    // adiabatic field (Sec. 5.3, Eqs. 14-15): alpha of the kicked density and the global
    // adjoint term of its density dependence, from the probe sums of this member
    double are = 0.0, aim = 0.0, bth = 0.0, bc = 0.0, thn = 0.0, c2n = 0.0, inv0 = 0.0, extra = 0.0;
    if (I.aprobe) {
        double sm[NPART] = {};
        strided_sum(I.aprobe, nprobe, NPART, {0, 1, 2, 3, 4}, sm);
        block_sum<NPART>(sm, red);
        if (threadIdx.x == 0) {
            const PotDev &p = I.pot;
            double ar, ai;
            alpha_adiabatic(p, tk, sm[0], sm[1], sm[2], &ar, &ai);
            const double tn = sm[1] / sm[0], cn = sm[2] / sm[0];
            const double sq = sqrt(fmax(sched_eval(p.sy, tk) * p.vc, 0.0));
            const double dr = p.delta_c - p.n_atoms * p.vc * cn, di = p.kappa, dd = dr * dr + di * di;
            // A = sum s dV/dalpha = 2 U0 alpha S_c + 2 sqrt(Vp U0) S_x
            const double Ar = 2.0 * p.vc * ar * sm[3] + 2.0 * sq * sm[4], Ai = 2.0 * p.vc * ai * sm[3];
            // dalpha/dTheta^ = N sq / (D + i kappa); dalpha/dC^ = alpha N U0 / (D + i kappa)
            const double tr = p.n_atoms * sq * dr / dd, ti = -p.n_atoms * sq * di / dd;
            const double cr = p.n_atoms * p.vc * (ar * dr + ai * di) / dd, ci = p.n_atoms * p.vc * (ai * dr - ar * di) / dd;
            red[0] = ar;
            red[1] = ai;
            red[2] = Ar * tr + Ai * ti;  // Re(conj(A) dalpha/dTheta^)
            red[3] = Ar * cr + Ai * ci;  // Re(conj(A) dalpha/dC^)
            red[4] = tn;
            red[5] = cn;
            red[6] = 1.0 / sm[0];
            // pump control: (U0 / sq) Re(alpha) S_x + Re(conj(A) dalpha/dVp), dalpha/dVp = N U0 Theta^ / (2 sq (D + i kappa))
            double ex = 0.0;
            if (I.control_axis && sq > 0.0) {
                const double f = p.n_atoms * p.vc * tn / (2.0 * sq);
                ex = (p.vc / sq) * ar * sm[4] + f * (Ar * dr - Ai * di) / dd;
            }
            red[7] = ex;
        }
        __syncthreads();
        are = red[0]; aim = red[1]; bth = red[2]; bc = red[3]; thn = red[4]; c2n = red[5]; inv0 = red[6]; extra = red[7];
        __syncthreads();
    }
    const VLine vl = vline_cav(I.pot, row, tk, are, aim);
    const float *vu = I.pot.vuser ? I.pot.vuser + (size_t)row * N : nullptr;
    const double wy = I.control_axis ? (double)I.pot.ty[row].y : 0.0;  // cos^2(ky_lat y) of this row
    double part[1] = {0.0};
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int i = t + m * T;
        const float4 tx = s_tx[i];
        double V = vpoint(vl, tx);
        if (vu) V += (double)vu[i];
        const double th = (V + gd.g * (v[m].x * v[m].x + v[m].y * v[m].y)) * tau;
        double sn, cs;
        sincos_d(th, &sn, &cs);
        const double s = w[m].x * v[m].y - w[m].y * v[m].x;  // Im(conj(G') psi')
        const C vin = {v[m].x * cs - v[m].y * sn, v[m].x * sn + v[m].y * cs};
        double wt = gd.g * s;
        if (I.aprobe) {
            const double cx = tx.z;
            wt += (bth * (cx * cyc - thn) + bc * (cx * cx - c2n)) * inv0;
        }
        const double k2 = 2.0 * tau * wt;
        w[m] = {w[m].x * cs - w[m].y * sn + k2 * vin.x, w[m].x * sn + w[m].y * cs + k2 * vin.y};
        v[m] = vin;
        part[0] += tau * s * (I.control_axis ? wy : (double)tx.y);  // dV/dV0 = cos^2 of the controlled lattice
    }
    if (lb == 0 && threadIdx.x == 0) part[0] += tau * extra;  // global pump term, once per kick
    block_sum<1>(part, red);
    if (threadIdx.x == 0) I.partials[lb] = part[0];
    if constexpr (MODE != ADJ_LAST) {
        if constexpr (TRAJ)
            fft_line<N, R, false>(w, lb2, t, s_tw);
        else
            fft_line2<N, R, false>(v, w, la, lb2, t, s_tw);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if constexpr (!TRAJ) store_c64(pp + t + m * T, v[m]);
        store_c64(pl + t + m * T, w[m]);
    }
}

template <int N, int R, int MODE, bool TRAJ>
__global__ void __launch_bounds__(512) row_adj_b(AdjPassArgs a)
{
    extern __shared__ XchgT smem[];
    __shared__ double red[8 * NPART];
    const AdjInst &I = a.inst[blockIdx.x / a.blocks_per_inst];
    if constexpr (MODE == ADJ_PROBE_FIRST || MODE == ADJ_PROBE_MID)
        if (!I.aprobe) return;
    row_adj_body<N, R, MODE, TRAJ>(I, blockIdx.x % a.blocks_per_inst, a.per_wg, a.kick, smem, red,
                                   a.blocks_per_inst);
}

// Sum one member's row partials (fixed order) into kick_grad[k]; one work-group.
__device__ __forceinline__ void adj_tail(const AdjInst &I, int nrow, int k, double *red)
{
    double s[1] = {0.0};
    strided_sum(I.partials, nrow, 1, {0}, s);
    block_sum<1>(s, red);
    if (threadIdx.x == 0) I.kick_grad[k] += s[0];
}

template <int N, int R, bool TRAJ>
__global__ void __launch_bounds__(512) col_adj_b(AdjPassArgs a)
{
    using C = double2;
    constexpr int T = N / R;
    using View = LineTile<XchgT, ilog2(R)>;
    extern __shared__ XchgT smem[];
    __shared__ double red[16];
    const int tile = xcd_tile(a.xcd_swizzle);
    const AdjInst &I = a.inst[tile / a.blocks_per_inst];
    const int lt = tile % a.blocks_per_inst;
    if (a.tail_kick >= 0 && lt == 0) adj_tail(I, a.row_blocks, a.tail_kick, red);
    const GridDev &gd = I.grid;
    const int w = a.per_wg;
    const int c = threadIdx.x % w, t = threadIdx.x / w;
    const int col = lt * w + c;
    const int nx = gd.nx;
    const size_t words = View::words(N, w);
    constexpr int AREAS = TRAJ ? 1 : 2;  // TRAJ: lam alone
    View la{smem + c, w};
    View lb{smem + (AREAS - 1) * words + c, w};
#if GPE_ADJ_TW_LDS
    double2 *s_tw = (double2 *)((char *)smem + align16(AREAS * words * sizeof(XchgT)));
    double2 *s_ky = s_tw + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        s_tw[i] = gd.tw_y[i];
        s_ky[i] = gd.kin_y[i];
    }
#else
    const double2 *s_tw = gd.tw_y;
    const double2 *s_ky = gd.kin_y;
#endif
    C v[R], u[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if constexpr (!TRAJ) {
            float2 f = I.psi[(size_t)(t + m * T) * nx + col];
            v[m] = {(double)f.x, (double)f.y};
        }
        float2 h = I.lam[(size_t)(t + m * T) * nx + col];
        u[m] = {(double)h.x, (double)h.y};
    }
    __syncthreads();
    if constexpr (TRAJ)
        fft_line<N, R, false>(u, lb, t, s_tw);
    else
        fft_line2<N, R, false>(v, u, la, lb, t, s_tw);
    const C kx = gd.kin_x[col];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const C f = cmul(kx, s_ky[t + m * T]);
        if constexpr (!TRAJ) v[m] = cmulc(v[m], f);
        u[m] = cmulc(u[m], f);
    }
    if constexpr (TRAJ)
        fft_line<N, R, true>(u, lb, t, s_tw);
    else
        fft_line2<N, R, true>(v, u, la, lb, t, s_tw);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if constexpr (!TRAJ) store_c64(I.psi + (size_t)(t + m * T) * nx + col, v[m]);
        store_c64(I.lam + (size_t)(t + m * T) * nx + col, u[m]);
    }
}

// After a batched call's exit pass: each field-ODE member's Theta of its last kick joins
// the overlap history (one work-group per member).

}  // namespace gpe
