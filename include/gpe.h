/*
 * gpe.h -- C ABI of the MI355X (gfx950) split-step Gross-Pitaevskii library.
 *
 * The library advances a 2D condensate wave function psi(x, y) under
 *   i d psi/dt = [ -1/2 laplacian + V(x, y, t; alpha) + g |psi|^2 ] psi
 * (the GPE of arXiv:2404.14401, Sec. 2, Eq. 1, in the dimensionless oscillator
 * units of Sec. 3.2: hbar = m = 1) with the symmetric split-step Fourier method
 * (Sec. 3.1, Eqs. 3-4) in real time and in imaginary time (Sec. 3.3).  Each step is
 *   psi' = psi  exp(-i [V(t_n) + g|psi|^2] dt/2)            half potential kick
 *   psi* = IFFT2( exp(-i k^2 dt/2) FFT2(psi') )             kinetic propagation
 *   psi_{n+1} = psi* exp(-i [V(t_{n+1}) + g|psi*|^2] dt/2)  half kick, newest density
 * (imaginary time: the same with -i dt -> -dt and psi renormalised to unit norm after
 * every step).  The potential is
 *   V = 1/2 wx^2 (x-x0)^2 + 1/2 wy^2 (y-y0)^2                     trap (Sec. 5.1)
 *     + Vx(t) cos^2(kx_lat x) + Vy(t) cos^2(ky_lat y)              lattices (Sec. 5.2, Eq. 9)
 *     + Vc |alpha|^2 cos^2(kc x)
 *     + 2 sqrt(Vy(t) Vc) Re(alpha) cos(kc x) cos(kc y)             cavity (Sec. 5.3, Eqs. 10-13)
 *     + V_user(x, y)                                              optional static array
 * and the cavity field alpha either (GPE_CAVITY_ODE) obeys
 *   d alpha/dt = (i Delta_c - kappa) alpha - i eta Theta,  Theta = <psi| cos kc x cos kc y |psi>
 * (the driven-damped form whose fixed point is Sec. 5.3, Eq. 14), advanced once per
 * step by an exponential integrator with the forcing extrapolated to second order, or
 * (GPE_CAVITY_ADIABATIC) is Eq. 14 itself with the dispersive shift of Eq. 15,
 *   alpha = N sqrt(Vy(t) Vc) Theta / (Delta_c - N Vc C + i kappa),  C = <psi| cos^2 kc x |psi>,
 * Theta and C per unit norm, N = n_atoms, evaluated from the density about to be kicked:
 * before every kick in real time (a probe pass reduces that density first), once per
 * step from the state entering it in imaginary time.  The on-axis cavity probe of
 * Sec. 5.4 (Eq. 17) adds Omega_c e^{i (Delta_p t + phi)} / (Delta_c - N Vc C + i kappa) to it.
 *
 * Grid: x_i = -lx/2 + i lx/nx (i < nx), likewise y; psi is stored row-major
 * [ny][nx] (x fastest) as interleaved (re, im) floats; periodic boundaries (the FFT
 * imposes them, Sec. 3.1).  Norm: sum |psi|^2 dx dy.
 *
 * Conventions of every entry point:
 *   - return 0 (GPE_OK) or a negative GPE_ERR_* code; no exception crosses the ABI;
 *     gpe_last_error() gives a thread-local message for the last failure.
 *   - argument errors are reported immediately; device-side failures (a NaN or an
 *     infinity in psi, seen by every kicking pass whether or not it reduces anything)
 *     are reported by the next synchronising call (gpe_sync, gpe_get_cavity; batches:
 *     gpe_batch_sync, gpe_batch_get_cavity); gpe_norm and gpe_energy report a
 *     non-finite input of their own.
 *   - device pointers are caller-owned and must stay valid until the work queued on
 *     the plan's stream has finished; all work is queued on that stream.
 *   - a plan or batch must not be used from two threads at once.
 */
#ifndef GPE_H
#define GPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPE_OK 0
#define GPE_ERR_INVALID (-1)     /* bad argument or plan state */
#define GPE_ERR_NOMEM (-2)       /* device allocation failed or exceeds max_bytes */
#define GPE_ERR_DEVICE (-3)      /* HIP runtime error */
#define GPE_ERR_NONFINITE (-4)   /* NaN/Inf detected in psi by a kick or a reduction */
#define GPE_ERR_UNSUPPORTED (-5) /* valid request the library does not implement */

typedef struct gpe_plan gpe_plan;
typedef struct gpe_batch gpe_batch;

/* One complex64 grid value, interleaved (re, im). */
typedef struct {
    float re, im;
} gpe_c64;

/* Plan description.  nx, ny: powers of two in [16, 8192]; lx, ly > 0: box lengths;
 * dt > 0: time step (imaginary time: dtau); g >= 0: interaction strength (already the
 * effective 2D, norm-absorbing value, Sec. 3.2); stream: a hipStream_t, NULL for the
 * null stream; max_bytes: cap on the plan's own device memory (0: none). */
typedef struct {
    int32_t nx, ny;
    double lx, ly;
    double dt;
    double g;
    void *stream;
    size_t max_bytes;
} gpe_plan_desc;

/* Lattice depth versus time, evaluated at each kick's time.  CONST: v0.  RAMP: v0 at
 * t0 to v1 at t1, linear, clamped outside.  KNOTS: nknots >= 2 values spread evenly on
 * [t0, t1], linear in between, clamped outside; the host array is copied when the
 * descriptor is set.  PULSE: the flashed lattice of Sec. 5.2, v0 for t0 <= t < t1 and
 * v1 otherwise; the kicks inside the pulse add up to its length t1 - t0 when its edges
 * fall half a step from kick times (kicks sit at t0_call + n dt in gpe_step_real, at
 * t0_call + (n + 1/2) dt in gpe_step_real_k), or on the first kick of a call. */
#define GPE_SCHED_CONST 0
#define GPE_SCHED_RAMP 1
#define GPE_SCHED_KNOTS 2
#define GPE_SCHED_PULSE 3
typedef struct {
    int32_t kind;
    int32_t nknots;
    double v0, v1, t0, t1;
    const double *knots;
} gpe_schedule;

/* Potential description (Sec. 5.1-5.3).  The pump lattice of the cavity model is the
 * y lattice (depth Vy(t)); its interference term uses kc and sqrt(Vy Vc), so the pump
 * schedule's values and vc must not differ in sign (GPE_ERR_INVALID).  cavity: one of
 * GPE_CAVITY_*; eta is the ODE's coupling, n_atoms the adiabatic field's N.  v_user:
 * optional device float array [ny][nx], borrowed for as long as the plan uses it.
 * Setting a potential resets the cavity field to alpha0 and forgets the overlap
 * history. */
#define GPE_CAVITY_OFF 0
#define GPE_CAVITY_ODE 1
#define GPE_CAVITY_ADIABATIC 2
typedef struct {
    double wx, wy, x0, y0;
    double kx_lat, ky_lat;
    gpe_schedule sx, sy;
    int32_t cavity;
    double vc, kc, delta_c, kappa, eta;
    double alpha0_re, alpha0_im;
    const float *v_user;
    double n_atoms;
    double probe_omega, probe_detuning, probe_phase;  // Omega_c, Delta_p, phi (adiabatic field only)
} gpe_potential_desc;

/* Per-step observables written by gpe_step_real / gpe_step_imag into a device array
 * of nsteps records of GPE_NOBS doubles each, for the state after every step:
 *   [0] norm (imaginary time: the norm before renormalisation, so that
 *       -ln(norm) / (2 dtau) estimates mu), [1] Theta, [2] Re alpha, [3] Im alpha,
 *   [4] integral x|psi|^2, [5] integral y|psi|^2. */
#define GPE_NOBS 6

/* Create a plan: allocates its tables and scratch once (the kernels allocate nothing
 * per step).  The potential starts as a unit isotropic trap with no lattice.  Grids
 * up to 32^2 (64^2 in imaginary time) run every step of a call in one work-group with
 * the grid in LDS, larger ones as two FFT passes per step over the chip (environment
 * GPE_PATH=lds|multipass forces either where it can). */
int gpe_plan_create(gpe_plan **out, const gpe_plan_desc *desc);
int gpe_plan_destroy(gpe_plan *plan);

/* Replace the potential (callable between steps, e.g. to displace the trap). */
int gpe_set_potential(gpe_plan *plan, const gpe_potential_desc *pot);

/* nsteps real-time split steps (Sec. 3.1) of psi in place, starting at time t0 (the
 * lattice schedules are evaluated at t0 + n dt).  psi: device [ny][nx] gpe_c64.
 * obs: device, nsteps * GPE_NOBS doubles, or NULL.  With the cavity on, the field
 * and the overlap history carry over from the previous call on this plan. */
int gpe_step_real(gpe_plan *plan, gpe_c64 *psi, int64_t nsteps, double t0, double *obs);

/* nsteps real-time steps in the ordering the paper prints (Sec. 3.1, Eq. 4) with the
 * state kept in Fourier space: psi_k <- e^{T/2} F[e^{V} F^{-1}[e^{T/2} psi_k]], the kick
 * over the full dt at the step midpoint t0 + (n + 1/2) dt.  psik: device [ny][nx]
 * gpe_c64 holding FFT2(psi) (unscaled forward transform), updated in place; momentum
 * populations are |psik|^2 directly (Sec. 5.2).  obs (nullable): per step, the
 * observables of the real-space state at the kick (norm, Theta, alpha, <x>, <y>).
 * The cavity must be off (GPE_ERR_UNSUPPORTED otherwise). */
int gpe_step_real_k(gpe_plan *plan, gpe_c64 *psik, int64_t nsteps, double t0, double *obs);

/* nsteps imaginary-time steps (Sec. 3.3) in the same Fourier-space ordering, potential
 * frozen at time t: psi_k <- e^{-T/2} F[e^{-V} F^{-1}[e^{-T/2} psi_k]], then psi_k is
 * renormalised to unit norm (the norm by Parseval, sum |psi_k|^2 dx dy / (nx ny)).
 * obs (nullable): per step the norm before renormalisation in [0] (the other fields
 * are zero).  The cavity must be off (GPE_ERR_UNSUPPORTED otherwise). */
int gpe_step_imag_k(gpe_plan *plan, gpe_c64 *psik, int64_t nsteps, double t, double *obs);

/* nsteps imaginary-time steps (Sec. 3.3) with the potential frozen at time t; the ODE
 * cavity field is held fixed, the adiabatic one follows the state (its value for the
 * returned state is left in the plan); psi ends with unit norm.  obs as for
 * gpe_step_real (the field recorded is the one the step used). */
int gpe_step_imag(gpe_plan *plan, gpe_c64 *psi, int64_t nsteps, double t, double *obs);

/* Energy functional of psi at time t with the plan's current cavity field
 * (synchronous): out = {E_kin, E_pot, E_int, E, mu, norm}, each per unit norm,
 * E_kin = sum_k |k|^2/2 |psi_k|^2 from the spectrum, E_int = g/2 int |psi|^4,
 * mu = E_kin + E_pot + 2 E_int.  GPE_ERR_NONFINITE (out still written) if a sum is not
 * finite. */
int gpe_energy(gpe_plan *plan, const gpe_c64 *psi, double t, double out[6]);

/* Populations of the momentum orders |2 n hbar k> of a Fourier-space state (Sec. 5.2:
 * read off the reciprocal-space amplitude), synchronous.  psik: device [ny][nx]
 * FFT2(psi) as kept by gpe_step_real_k.  axis: 0 (x) or 1 (y); order_step: FFT bins
 * between neighbouring orders, 2 k L / (2 pi) for a lattice commensurate with the box
 * (L the box length along the axis).  Bin j (signed, -n/2 <= j < n/2) belongs to order
 * floor((j + floor(order_step / 2)) / order_step).  out (host, 2 nmax + 2 doubles):
 * out[n + nmax] = sum of |psik|^2 in order n over the total, n = -nmax..nmax; then the
 * norm sum |psik|^2 dx dy / (nx ny).  Errors: GPE_ERR_INVALID for an axis outside
 * {0, 1}, order_step < 1, or (2 nmax + 1) order_step above the points on the axis. */
int gpe_momentum_orders(gpe_plan *plan, const gpe_c64 *psik, int axis, int order_step, int nmax, double *out);

/* sum |psi|^2 dx dy (synchronous); GPE_ERR_NONFINITE (out still written) if it is not
 * finite. */
int gpe_norm(gpe_plan *plan, const gpe_c64 *psi, double *out);

/* Cavity state (synchronous): {Re alpha, Im alpha, Theta_n, Theta_{n-1}}; and its
 * restore, for checkpoint/resume.  have_history = 0 makes the next real-time call
 * start its overlap history from the current psi. */
int gpe_get_cavity(gpe_plan *plan, double out[4]);
int gpe_set_cavity(gpe_plan *plan, const double state[4], int have_history);

/* Wait for the plan's stream; reports deferred device errors. */
int gpe_sync(gpe_plan *plan);

/* Instrumentation for roofline measurements.  gpe_set_timing(plan, every): when
 * every > 0, gpe_step_real launches the column pass and the middle row pass of the last
 * step of every window of `every` steps (steps every-1, 2 every-1, ... of a call, never its
 * last) with a pair of HIP events that record the kernel's own start and end on the
 * plan's stream (hipExtLaunchKernel; where 4096- or 8192-point columns take the column
 * step as three passes, the pair spans all three); every = 0 turns it off and clears the record.
 * gpe_get_timing (synchronous) returns {mean column-pass ms, column launches timed, mean
 * row-pass ms, row launches timed}. */
int gpe_set_timing(gpe_plan *plan, int every);
int gpe_get_timing(gpe_plan *plan, double out[4]);

/* Thread-local message of the last failed call ("" if none). */
const char *gpe_last_error(void);

/* ------------------------------------------------------------------ batched
 * n independent condensates, each with its own plan description (sizes may differ;
 * dt must be equal) and potential, advanced together: every step is one launch per
 * FFT pass over all members of a size.  Members up to 64^2 -- and 128^2 ones beside
 * larger sizes or at least 256 of them -- instead run all their steps in one
 * work-group each, the grid kept in LDS (environment GPE_BATCH_PATH=lds|multipass
 * forces either where it can).  The batched multi-pass kernels take lines of 64..2048
 * points: a member too large for LDS (a side above 128) with a side below 64 or above
 * 2048 is refused with GPE_ERR_UNSUPPORTED (a plan of its own takes it).  psis: host
 * array of n device pointers.  All members share the stream of desc[0]. */
int gpe_batch_create(gpe_batch **out, int n, const gpe_plan_desc *descs, const gpe_potential_desc *pots);
int gpe_batch_destroy(gpe_batch *b);
int gpe_step_batched(gpe_batch *b, gpe_c64 *const *psis, int64_t nsteps, double t0);

/* Autotune the launch schedule (radix 4 or 8, rows per work-group, number of column
 * tiles) of every multi-pass group by timing the candidates on the members' scratch
 * arrays; choices are read from and appended to the text file cache_path (NULL: no
 * cache), one line "arch nx ny count radix row_threads min_col_tiles us_per_step". */
int gpe_batch_tune(gpe_batch *b, const char *cache_path);

/* Description of size group g (synchronous): out = {nx, ny, members, lds-resident,
 * radix, row threads per work-group, column work-groups per member, number of groups}. */
int gpe_batch_info(gpe_batch *b, int group, int out[8]);

/* Wait for the batch's queued work and report deferred device errors: GPE_ERR_NONFINITE
 * if any member's wave function held a NaN or an infinity when one of its kicks (or, for
 * members kept in LDS, the end of a call) read it; first_bad (nullable, host) receives
 * the lowest such member index, -1 if none.  Like gpe_sync, the flag stays set until the
 * batch is destroyed. */
int gpe_batch_sync(gpe_batch *b, int *first_bad);

/* Cavity state of batch member m after the batch's last call, as gpe_get_cavity
 * (synchronous).  Members may carry either cavity model: the field ODE (its overlap
 * history carries over between calls, as on a plan) or the adiabatic field of Sec. 5.3,
 * Eqs. 14-15. */
int gpe_batch_get_cavity(gpe_batch *b, int member, double out[4]);

/* ------------------------------------------------------------------ adjoint
 * Gradient of a loss of psi(T), T = t0 + nsteps dt, with respect to the knot values
 * of a lattice-depth schedule (GPE_SCHED_KNOTS) of every member of a batch of
 * real-time problems of one grid size: control GPE_CONTROL_X_LATTICE differentiates the
 * x lattice Vx(t) cos^2(kx_lat x), GPE_CONTROL_PUMP the y lattice Vy(t) cos^2(ky_lat y),
 * the pump of the cavity set-up (Sec. 5.3).  Members run without the cavity or with the
 * adiabatic field (GPE_CAVITY_ADIABATIC, probe included): then the gradient also carries
 * alpha's dependence on the density and, for the pump, on Vy (sqrt(Vy Vc) coupling; the
 * pump knots must keep Vy Vc > 0).  The field ODE is rejected (GPE_ERR_UNSUPPORTED).
 * Losses:
 *   GPE_LOSS_FIDELITY: L = 1 - |<target|psi(T)>|^2, <a|b> = sum conj(a) b dx dy;
 *   GPE_LOSS_ENERGY:   L = E_kin + E_pot + E_int of psi(T) at time T (as gpe_energy's
 *                      terms times the norm; members without a cavity only, else
 *                      GPE_ERR_UNSUPPORTED).
 * The reverse sweep rebuilds the forward states by running each step backwards
 * (exact in real time) -- GPE_ADJ_RECONSTRUCT -- or from stored states every
 * ~sqrt(nsteps) steps -- GPE_ADJ_CHECKPOINT; GPE_ADJ_AUTO reconstructs and falls
 * back to checkpoints if the rebuilt psi(0) drifts from the input by more than
 * drift_tol (relative L2).  GPE_ADJ_STORE keeps every kick's output state from the
 * forward sweep (nsteps * nx * ny * 8 bytes per member, kept by the batch for later
 * calls, GPE_ERR_NOMEM if the device cannot hold it), so the reverse sweep transforms
 * the adjoint alone: the fastest mode where HBM allows it.
 * psi0, target: host arrays of nb device pointers ([ny][nx] gpe_c64 each; target may
 * be null for the energy loss and is ignored there); knots: host, nb * nknots finite values (they replace
 * the members' knots of the controlled lattice; pump knots of a cavity member must be nonzero with the
 * sign of vc; GPE_ERR_INVALID otherwise, before anything runs); loss: host, nb values; grad: host,
 * nb * nknots values, or NULL for the loss alone (the forward sweep only: no reverse sweep, no
 * checkpoints or stored trajectory, mode ignored);
 * psi_final (nullable): host array of nb device pointers receiving psi(T).
 * info (nullable): host, 4 doubles {mode used (0 loss alone, 1 reconstruct, 2 checkpoint, 3 store),
 * reconstruction drift, peak scratch bytes, number of forward steps run}. */
#define GPE_LOSS_FIDELITY 0
#define GPE_LOSS_ENERGY 1
#define GPE_ADJ_AUTO 0
#define GPE_ADJ_RECONSTRUCT 1
#define GPE_ADJ_CHECKPOINT 2
#define GPE_ADJ_STORE 3
#define GPE_CONTROL_X_LATTICE 0
#define GPE_CONTROL_PUMP 1
int gpe_adjoint(gpe_batch *b, const gpe_c64 *const *psi0, const gpe_c64 *const *target, int64_t nsteps,
                double t0, const double *knots, int nknots, int control, int loss_kind, int mode,
                double drift_tol, double *loss, double *grad, gpe_c64 *const *psi_final, double *info);

/* ------------------------------------------------------------ allocation-free
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the real-time steps of gpe_step_real
 * without a plan.  The call does what gpe_step_real does on a fresh plan created from
 * desc with potential pot (same kernels, same launch shapes): the cavity field starts at
 * alpha0 with no overlap history.  Instead of plan memory it uses one static device array
 * of 2 MiB (per device, held until the process ends): every call rebuilds the tables in
 * it with kernels and issues only kernel launches on desc->stream -- no hipMalloc, no
 * hipFree, no memset, no host-to-device copy, no graph of its own.  Calls on one device
 * share the array, so calls that overlap on one device (other streams or threads) race.
 * desc, pot: as for gpe_plan_create / gpe_set_potential (host, read during the call);
 * knot schedules hold at most 256 knots; every grid the plan takes (powers of two 16 to
 * 8192 per side) fits the array.  psi: device [ny][nx] gpe_c64, updated in place,
 * asynchronously.  nonfinite: optional device int that receives 1 if a kick met a NaN or
 * an infinity in psi, else 0 (the call itself cannot wait for the device); untouched when
 * nsteps = 0.  No observables.  Errors: GPE_ERR_INVALID for bad descriptors, negative
 * nsteps, more than 256 knots; GPE_ERR_DEVICE for a failed launch. */
int gpe_step_real_noalloc(const gpe_plan_desc *desc, const gpe_potential_desc *pot, gpe_c64 *psi, int64_t nsteps,
                          double t0, int *nonfinite);

#ifdef __cplusplus
}
#endif

#endif /* GPE_H */
