// physics.h -- pointwise pieces of the split step on the device: potential, kicks,
// cavity-field recurrence, reductions.
#pragma once
#include "gpe_internal.h"

namespace gpe {

// Lattice depth at time t (const, ramp or piecewise-linear knots, clamped).
__device__ __forceinline__ double sched_eval(const Sched &s, double t)
{
    if (s.kind == 0) return s.v0;
    if (s.kind == 1) {
        if (t <= s.t0) return s.v0;
        if (t >= s.t1) return s.v1;
        return s.v0 + (s.v1 - s.v0) * (t - s.t0) / (s.t1 - s.t0);
    }
    if (s.kind == 3) return (t >= s.t0 && t < s.t1) ? s.v0 : s.v1;  // flashed lattice (Sec. 5.2)
    const int m = s.nknots;
    if (m == 1 || t <= s.t0) return s.knots[0];
    if (t >= s.t1) return s.knots[m - 1];
    double u = (t - s.t0) / (s.t1 - s.t0) * (m - 1);
    int i = (int)floor(u);
    if (i >= m - 1) i = m - 2;
    double w = u - i;
    return (1.0 - w) * s.knots[i] + w * s.knots[i + 1];
}

// Line-uniform part of V for row j at time t with field alpha:
// V(i, j) = base + tx.x + vx * tx.y + tx.z * (a2 * tx.z + ccy)  (+ v_user)
struct VLine {
    double base, vx, a2, ccy;
};

__device__ __forceinline__ VLine vline_cav(const PotDev &p, int j, double t, double are, double aim)
{
    const double vx = sched_eval(p.sx, t), vy = sched_eval(p.sy, t);
    const float4 ty = p.ty[j];
    VLine l;
    l.base = (double)ty.x + vy * (double)ty.y;
    l.vx = vx;
    if (p.cavity) {
        l.a2 = p.vc * (are * are + aim * aim);                     // Vc |alpha|^2 cos^2(kc x)
        l.ccy = 2.0 * sqrt(fmax(vy * p.vc, 0.0)) * are * (double)ty.z;  // 2 sqrt(V0 Vc) Re(alpha) cos(kc y)
    } else {
        l.a2 = 0.0;
        l.ccy = 0.0;
    }
    return l;
}

__device__ __forceinline__ double vpoint(const VLine &l, float4 tx)
{
    const double cx = tx.z;
    return l.base + (double)tx.x + l.vx * (double)tx.y + cx * (l.a2 * cx + l.ccy);
}

// sin and cos in double; Taylor polynomials on |x| < 0.785 (truncation < 3e-14),
// the library routine elsewhere.
#ifndef GPE_FAST_KICK
#define GPE_FAST_KICK 1
#endif
// |x| < 1/16: Taylor to x^9 and x^10 (truncation below 2e-19)
__device__ __forceinline__ void sincos_small(double x, double *s, double *c)
{
    const double x2 = x * x;
    *s = x * (1.0 + x2 * (-1.0 / 6 + x2 * (1.0 / 120 + x2 * (-1.0 / 5040 + x2 * (1.0 / 362880)))));
    *c = 1.0 + x2 * (-0.5 + x2 * (1.0 / 24 + x2 * (-1.0 / 720 + x2 * (1.0 / 40320 + x2 * (-1.0 / 3628800)))));
}

__device__ __forceinline__ void sincos_d(double x, double *s, double *c)
{
#if GPE_FAST_KICK
    if (fabs(x) < 0.0625) {
        sincos_small(x, s, c);
        return;
    }
#endif
    if (fabs(x) < 0.785) {
        const double x2 = x * x;
        *s = x * (1.0 + x2 * (-1.0 / 6 + x2 * (1.0 / 120 + x2 * (-1.0 / 5040 + x2 * (1.0 / 362880 +
                 x2 * (-1.0 / 39916800 + x2 * (1.0 / 6227020800.0)))))));
        *c = 1.0 + x2 * (-0.5 + x2 * (1.0 / 24 + x2 * (-1.0 / 720 + x2 * (1.0 / 40320 +
                 x2 * (-1.0 / 3628800 + x2 * (1.0 / 479001600.0 + x2 * (-1.0 / 87178291200.0)))))));
    } else {
        sincos(x, s, c);
    }
}

// psi * exp(-i theta)
__device__ __forceinline__ double2 kick_real(double2 p, double theta)
{
    double s, c;
    sincos_d(theta, &s, &c);
    return {p.x * c + p.y * s, p.y * c - p.x * s};
}

// psi * exp(-theta)
__device__ __forceinline__ double2 kick_imag(double2 p, double theta)
{
    const double e = exp(-theta);
    return {p.x * e, p.y * e};
}

// Wave-then-work-group sum of NV doubles; result valid in thread 0.  `red` must hold
// NV * (blockDim/64) doubles.  Fixed order: deterministic.
template <int NV> __device__ __forceinline__ void block_sum(double (&v)[NV], double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[w * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int i = 0; i < nw; ++i) s += red[i * NV + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Thread-strided sum of the components comp[] of records [n][stride]: thread t adds
// records t, t + b, t + 2b, ... (b = blockDim.x) in that order, whatever the timing, so
// that with block_sum the result is the same fixed-order sum everywhere; the loads go out
// D records at a time rather than as a chain of single L2 round trips.
template <int D = 8, int NK>
__device__ __forceinline__ void strided_sum(const double *p, int n, int stride, const int (&comp)[NK],
                                            double (&s)[NK])
{
    const int b = blockDim.x;
    int i = threadIdx.x;
    for (; i + (D - 1) * b < n; i += D * b) {
        double q[D][NK];
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < NK; ++k) q[j][k] = p[(size_t)(i + j * b) * stride + comp[k]];
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < NK; ++k) s[k] += q[j][k];
    }
    for (; i < n; i += b)
#pragma unroll
        for (int k = 0; k < NK; ++k) s[k] += p[(size_t)i * stride + comp[k]];
}

// Adiabatic cavity field (Sec. 5.3, Eqs. 14-15) of a density with integrals nrm,
// Theta = th and C = c2 at time t, with the on-axis probe of Sec. 5.4 (Eq. 17):
//   [N sqrt(Vp(t) U0) (th/nrm) + Omega_c e^{i (Delta_p t + phi)}] / (Delta_c - N U0 c2/nrm + i kappa).
__device__ __forceinline__ void alpha_adiabatic(const PotDev &p, double t, double nrm, double th, double c2,
                                                double *are, double *aim)
{
    const double vp = sched_eval(p.sy, t);
    const double inv = 1.0 / nrm;
    const double dtil = p.delta_c - p.n_atoms * p.vc * c2 * inv;
    double nr = p.n_atoms * sqrt(fmax(vp * p.vc, 0.0)) * th * inv, ni = 0.0;
    if (p.probe_omega != 0.0) {
        double s, c;
        sincos(p.probe_detuning * t + p.probe_phase, &s, &c);
        nr += p.probe_omega * c;
        ni += p.probe_omega * s;
    }
    const double den = dtil * dtil + p.kappa * p.kappa;
    *are = (nr * dtil + ni * p.kappa) / den;
    *aim = (ni * dtil - nr * p.kappa) / den;
}

// Cavity field over one step (exponential integrator, second-order extrapolated
// forcing): alpha <- ecav alpha + phi1 (-i eta (3 Theta_n - Theta_{n-1}) / 2).
__device__ __forceinline__ void cavity_advance(const PotDev &p, DevState *st)
{
    const double tb = 0.5 * (3.0 * st->theta - st->theta_prev);
    const double fr = 0.0, fi = -p.eta * tb;  // -i eta tb
    const double ar = st->alpha_re, ai = st->alpha_im;
    const double nr = p.ecav_re * ar - p.ecav_im * ai + p.phi1_re * fr - p.phi1_im * fi;
    const double ni = p.ecav_re * ai + p.ecav_im * ar + p.phi1_re * fi + p.phi1_im * fr;
    st->alpha_re = nr;
    st->alpha_im = ni;
}

// Reduce per-work-group partials [np][NPART] in a fixed order and update the state:
// observables, overlap history, imaginary-time scale, non-finite flag; then optionally
// advance the cavity field.  Called by every thread of one work-group.
__device__ __forceinline__ void run_tail(const TailArgs &ta, const GridDev &gd, const PotDev &pot,
                                         DevState *st, double *red)
{
    // (one load at a time: the column passes that inline this keep their register count)
    double s[NPART] = {};
    if (ta.npartials > 0 && ta.theta_only) {
        for (int i = threadIdx.x; i < ta.npartials; i += blockDim.x) s[1] += ta.partials[i * NPART + 1];
        block_sum<1>(*reinterpret_cast<double(*)[1]>(s + 1), red);
    } else if (ta.npartials > 0) {
        for (int i = threadIdx.x; i < ta.npartials; i += blockDim.x)
#pragma unroll
            for (int k = 0; k < NPART; ++k) s[k] += ta.partials[i * NPART + k];
        block_sum<NPART>(s, red);
    }
    if (threadIdx.x == 0) {
        if (ta.npartials > 0) {
            const double norm = s[0] * gd.dA, th = s[1] * gd.dA, mx = s[2] * gd.dA, my = s[3] * gd.dA;
            // (Theta-only partials leave the norm at zero; a non-finite psi reaches Theta too)
            if (!isfinite(norm) || !isfinite(th)) st->nonfinite = 1;
            st->norm = norm;
            if (ta.imag) {
                const double inv = 1.0 / norm;
                st->scale = sqrt(inv);
                if (ta.obs) {
                    ta.obs[0] = norm;
                    ta.obs[1] = th * inv;
                    ta.obs[2] = st->alpha_re;
                    ta.obs[3] = st->alpha_im;
                    ta.obs[4] = mx * inv;
                    ta.obs[5] = my * inv;
                }
            } else {
                if (pot.cavity == 1) {
                    if (ta.first_theta) {
                        st->theta = th;
                        st->theta_prev = th;
                        st->have_theta = 1;
                    } else {
                        st->theta_prev = st->theta;
                        st->theta = th;
                    }
                }
                if (ta.obs) {
                    ta.obs[0] = norm;
                    ta.obs[1] = th;
                    ta.obs[2] = st->alpha_re;
                    ta.obs[3] = st->alpha_im;
                    ta.obs[4] = mx;
                    ta.obs[5] = my;
                }
            }
        }
        // imaginary time: the adiabatic field of the state just reduced drives the next
        // step (after the observables above recorded the field this step used)
        if (ta.npartials > 0 && ta.alpha_from_partials && pot.cavity == 2)
            alpha_adiabatic(pot, st->t0, s[0], s[1], s[4], &st->alpha_re, &st->alpha_im);
        if (ta.advance_alpha && pot.cavity == 1) cavity_advance(pot, st);
    }
}

}  // namespace gpe
