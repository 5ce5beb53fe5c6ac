// gpe_internal.h -- structures shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpe {

// Lattice-depth schedule (device copy; knots in device memory).
struct Sched {
    int kind;  // 0 const, 1 ramp, 2 knots
    int nknots;
    double v0, v1, t0, t1;
    const double *knots;
};

// Everything a kernel needs to evaluate V(x, y, t; alpha) (Sec. 5.1-5.3).
// Per-axis tables hold {1/2 w^2 (x - x0)^2, cos^2(k_lat x), cos(kc x), x}.
struct PotDev {
    const float4 *tx;  // [nx]
    const float4 *ty;  // [ny]
    const float *vuser;  // [ny][nx] or null
    Sched sx, sy;
    int cavity;  // 0 off, 1 field ODE, 2 adiabatic field (Sec. 5.3, Eqs. 14-15)
    double vc;
    // cavity field step: alpha_{n+1} = ecav alpha_n + phi1 (-i eta Theta_bar)
    double ecav_re, ecav_im, phi1_re, phi1_im, eta;
    // adiabatic field: alpha = N sqrt(Vp U0) Theta / (Delta_c - N U0 C + i kappa),
    // plus the on-axis probe Omega_c e^{i (Delta_p t + phi)} over the same denominator
    double delta_c, kappa, n_atoms;
    double probe_omega, probe_detuning, probe_phase;
};

// Mutable device-side state of a plan (one per plan, in device memory).
struct DevState {
    double alpha_re, alpha_im;  // cavity field used by the next kick
    double theta, theta_prev;   // Theta_n, Theta_{n-1}
    double scale;               // imaginary time: pending 1/sqrt(norm)
    double norm;                // last reduced norm
    double t0;                  // time of the first step of the current call
    int have_theta;
    int nonfinite;
};

// Per-plan geometry and constant tables.
struct GridDev {
    int nx, ny;
    double lx, ly, dx, dy, dA, dt, g;
    const double2 *kin_x, *kin_y;    // real time: e^{-i kx^2 dt/2}, e^{-i ky^2 dt/2} / (nx ny)
    const double *kim_x, *kim_y;     // imaginary time: e^{-kx^2 dt/2}, e^{-ky^2 dt/2} / (nx ny)
    const double2 *tw_x, *tw_y;      // W_N^m, m < N, for the x and y transforms
    // kinetic half steps of the Fourier-space ordering: e^{-i kx^2 dt/4}, and
    // e^{-i ky^2 dt/4} with (entry) and without (exit) the 1/(nx ny) of the round trip
    const double2 *kh_x, *kh_yin, *kh_yout;
    const double *khi_x, *khi_yin, *khi_yout;  // the same in imaginary time: e^{-k^2 dt/4}
};

// Per-work-group partials: norm, Theta, x moment, y moment, C = cos^2(kc x) overlap.
constexpr int NPART = 5;
constexpr int NOBS = 6;

// Row-pass modes.
enum RowMode : int {
    ROW_ENTRY = 0,  // real-space psi -> (scale) -> half kick at t_n -> FFT_x
    ROW_MID = 1,    // IFFT_x -> merged kick at t_{n+1} -> FFT_x (real time)
    ROW_EXIT = 2,   // IFFT_x -> half kick at t_{n+1} -> real-space psi
    ROW_FWD = 3,    // real-space psi -> FFT_x, energy partials (E_pot, E_int, norm)
    ROW_PROBE_REAL = 4,  // real-space psi -> partials of norm, Theta, C (no store)
    ROW_PROBE_MID = 5,   // IFFT_x -> partials of norm, Theta, C (no store)
    ROW_INV = 6,         // IFFT_x only (back to real space)
};

// Column-pass modes.
enum ColMode : int {
    COL_KIN_REAL = 0,  // FFT_y -> e^{-i k^2 dt/2}/(nx ny) -> IFFT_y
    COL_KIN_IMAG = 1,  // FFT_y -> e^{-k^2 dt/2}/(nx ny) -> IFFT_y
    COL_EKIN = 2,      // FFT_y -> partials of sum k^2/2 |psi_k|^2 (no store)
    COL_KHALF_INV = 3, // (Fourier-space state) kinetic half step -> IFFT_y
    COL_FWD_KHALF = 4, // FFT_y -> kinetic half step (Fourier-space state out)
    COL_KHALF_INV_IM = 5,  // imaginary time: pending scale and kinetic half step -> IFFT_y
    COL_FWD_KHALF_IM = 6,  // imaginary time: FFT_y -> kinetic half step, partials of sum |psi_k|^2
    COL_KIN_APPLY = 7,     // FFT_y -> times |k|^2/2 /(nx ny), partials of sum |k|^2/2 |psi_k|^2 -> IFFT_y
};

struct RowArgs {
    const float2 *src;
    float2 *dst;
    GridDev grid;
    PotDev pot;
    DevState *st;
    double *partials;  // [gridDim.x][NPART]
    int n;             // step index within the call; kick time = st->t0 + (n or n+1) dt + t_shift
    int reduce;        // write partials: 1 all of them, 2 Theta only (the field ODE without observables)
    int lines_per_wg;
    double t_shift;    // -dt/2 for the midpoint kick of the Fourier-space ordering
    const double *probe;  // adiabatic field: partials of the density about to be kicked
    int nprobe;           // (0: take the field from the state)
    // imaginary-time entry pass: the previous exit pass's partials [nscale][NPART], from
    // whose norm every work-group forms the pending 1/sqrt(norm) itself (null: st->scale)
    const double *scale_partials;
    int nscale;
};

// Work done by work-group 0 of a column pass before its own columns: reduce the
// previous row pass's partials, record observables, advance the cavity field.
struct TailArgs {
    const double *partials;
    int npartials;     // 0: nothing to reduce
    int first_theta;   // the reduced Theta starts the overlap history
    double *obs;       // record slot (NOBS doubles) or null
    int imag;          // imaginary-time bookkeeping (scale, pre-normalisation norm)
    int advance_alpha; // compute alpha_{n+1} after the reduction
    int alpha_from_partials;  // adiabatic field of the reduced density (imaginary time)
    int theta_only;           // the partials hold Theta alone (slot 1)
};

struct ColArgs {
    const float2 *src;
    float2 *dst;
    GridDev grid;
    DevState *st;
    double *partials;
    int cols_per_wg;
    int xcd_swizzle;  // map consecutive column tiles onto one XCD (shared L2 lines)
    int reduce;
    PotDev pot;
    TailArgs tail;
    int do_tail;
};

// One member of a batch (device memory).
struct InstDesc {
    float2 *psi;
    GridDev grid;
    PotDev pot;
    DevState *st;
    double *probe;  // adiabatic field: [row work-groups][NPART] partials of the probe pass (else null)
    float2 *traj;   // adjoint forward sweep: post-kick real-space state of every kick but the
                    // last, [kick][ny][nx] (else null)
    double *partials;  // field ODE: [row work-groups][NPART] Theta partials of each kick (else null)
    int first_theta;   // field ODE: this call's first kick starts the overlap history
};

// A batched row or column pass over all members of one grid size.
struct BatchPassArgs {
    const InstDesc *inst;
    int blocks_per_inst;  // work-groups (row blocks or column tiles) per member
    int per_wg;           // rows or columns per work-group
    int n;                // step index within the call
    int xcd_swizzle;
    int cav;              // some member has a cavity field: kick kernels read the adiabatic members'
                          // probe partials and reduce the field-ODE members' Theta
    int traj;             // entry and merged kicks record their output in InstDesc::traj
    int ode;              // column pass: some member has the field ODE (its first tile runs the recurrence)
    int first;            // column pass of a call's first step
    int row_blocks;       // row work-groups per member (Theta partials to reduce)
};

// One member of an adjoint sweep (device memory): the state being reconstructed
// backwards and its adjoint, plus where the per-kick lattice gradient goes.
struct AdjInst {
    float2 *psi;
    float2 *lam;
    GridDev grid;
    PotDev pot;
    DevState *st;
    double *partials;   // [row work-groups] per-row-block sums of the current kick
    double *kick_grad;  // [nsteps + 1] dL/dV0 at t0 + k dt
    int control_axis;   // controlled lattice: 0 x, 1 y (the pump)
    double *aprobe;     // adiabatic field: [row work-groups][NPART] sums of rho, rho cos kx cos ky,
                        // rho cos^2 kx, s cos^2 kx, s cos kx cos ky over (psi', G') (else null)
    const float2 *traj; // stored post-kick states [kick][ny][nx] (the passes then carry lam alone)
};

enum AdjRowMode : int {
    ADJ_FIRST = 0,  // real-space (psi_K, lam_K) -> adjoint half kick at t_K -> FFT_x
    ADJ_MID = 1,    // IFFT_x -> adjoint merged kick at t_n -> FFT_x
    ADJ_LAST = 2,   // IFFT_x -> adjoint half kick at t_0 -> real space
    ADJ_PROBE_FIRST = 3,  // (adiabatic field) real-space (psi, G) -> field and adjoint sums
    ADJ_PROBE_MID = 4,    // (adiabatic field) IFFT_x of both -> field and adjoint sums
};

struct AdjPassArgs {
    const AdjInst *inst;
    int blocks_per_inst;
    int per_wg;
    int kick;           // step index of the kick (time st->t0 + kick dt)
    int xcd_swizzle;
    int tail_kick;      // column pass: add the previous row pass's sums to kick_grad[tail_kick] (-1: none)
    int row_blocks;     // number of row work-groups per member (partials to reduce)
    int traj;           // 1: states come from AdjInst::traj, the passes transform lam alone
};

// Whole grid resident in one work-group's LDS (small grids).
struct LdsArgs {
    float2 *psi;  // in/out real space, [ny][nx]
    GridDev grid;
    PotDev pot;
    DevState *st;
    double *obs;  // [nsteps][NOBS] or null
    int nsteps;
    int imag;
};

}  // namespace gpe
