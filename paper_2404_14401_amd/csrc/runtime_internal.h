// runtime_internal.h -- host-side internals shared by the runtime files: the plan
// object, launch shapes and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/gpe.h"
#include "gpe_internal.h"

namespace gpe {
hipError_t launch_row(int n, int mode, bool imag, const RowArgs &a, int blocks, int threads, size_t shmem,
                      hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_col(int n, int mode, const ColArgs &a, int blocks, int threads, size_t shmem, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The column step of real or imaginary time (COL_KIN_REAL / COL_KIN_IMAG) on columns of
// ny = 4096 or 8192 points in three passes (phase 0, 1, 2; a's cols_per_wg per phase).
hipError_t launch_col_split(int ny, int phase, int mode, const ColArgs &a, int blocks, int threads, size_t shmem,
                            hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int col_split_a();
hipError_t launch_tail(const TailArgs &ta, const GridDev &gd, const PotDev &pot, DevState *st, hipStream_t s);
hipError_t launch_scale(float2 *psi, size_t n, const DevState *st, hipStream_t s);
hipError_t launch_set_call(DevState *st, double t0, int reset_scale, int clear_history, hipStream_t s);
hipError_t launch_energy_grad(const float2 *psi, float2 *lam, const GridDev &gd, const PotDev &pot,
                              const DevState *st, int axis, double *partials, hipStream_t s);
hipError_t launch_marginal(const float2 *psi, int nx, int ny, int axis, double *out, hipStream_t s);
hipError_t launch_norm(const float2 *psi, size_t n, double *partials, int blocks, hipStream_t s);
hipError_t launch_lds_grid(const LdsArgs &a, hipStream_t s);
hipError_t launch_row_batched(int n, int r, int mode, const BatchPassArgs &a, int blocks, int threads, size_t shmem,
                              hipStream_t s);
hipError_t launch_col_batched(int n, int r, const BatchPassArgs &a, int blocks, int threads, size_t shmem,
                              hipStream_t s);
hipError_t launch_lds_batched(int nx, int ny, const LdsArgs *arr, int count, int64_t s0, int nsteps, hipStream_t s);
hipError_t launch_set_call_batched(DevState *const *st, int n, double t0, hipStream_t s);
hipError_t launch_advance_t0(DevState *const *st, int n, double dt_total, hipStream_t s);
hipError_t launch_advance_one(DevState *st, double dt_total, hipStream_t s);
hipError_t launch_gather_flags(DevState *const *st, int n, int *out, hipStream_t s);
hipError_t launch_row_adj(int n, int mode, const AdjPassArgs &a, int blocks, int threads, size_t shmem, hipStream_t s);
hipError_t launch_col_adj(int n, const AdjPassArgs &a, int blocks, int threads, size_t shmem, hipStream_t s);
hipError_t launch_tail_batched(const InstDesc *inst, int count, int nrow, hipStream_t s);
hipError_t launch_adj_tail(const AdjInst *inst, int count, int nrow, int k, hipStream_t s);
hipError_t launch_pair_sums(const float2 *const *a, const float2 *const *b, size_t npts, int count, int per_inst,
                            double *out, hipStream_t s);
hipError_t launch_scaled_copy(float2 *const *dst, const float2 *const *src, const double2 *coef, size_t npts,
                              int count, int per_inst, hipStream_t s);
hipError_t launch_copy_members(float2 *const *dst, const float2 *const *src, size_t npts, int count, int per_inst,
                               hipStream_t s);
bool lds_supported(int nx, int ny);
int lds_threads(int nx, int ny);
int kernel_radix();
// points per thread of the plan's row passes for n-point lines
int row_radix(int n);
size_t xchg_bytes();
size_t adj_row_shmem(int n, int lines, int r, int arrays);
size_t adj_col_shmem(int n, int w, int r, int arrays);
}  // namespace gpe

using namespace gpe;

int gpe_fail(int code, const std::string &msg);
#define fail gpe_fail

// A failed HIP call is reported by the call that made it; its error is also taken off the
// thread's last-error state so that a later launch check does not report it again.
#define HIP_OK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return fail(GPE_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_));          \
        }                                                                                          \
    } while (0)

#define LAUNCH_OK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(GPE_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e_)); \
    } while (0)

static inline bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

// Launch shape of the multi-pass path.
struct Shape {
    int row_lines, row_threads, row_blocks;
    size_t row_shmem;
    int col_cols, col_threads, col_blocks;
    size_t col_shmem;
    // long columns: the column step in three passes when split_a > 0 (transform lengths
    // split_a and ny / split_a; tile widths, threads, work-groups and LDS of the outer
    // passes (a) and of the middle one (b))
    int split_a = 0;
    int split_wa = 0, split_ta = 0, split_ba = 0, split_wb = 0, split_tb = 0, split_bb = 0;
    size_t split_sha = 0, split_shb = 0;
};

struct gpe_plan {
    int nx = 0, ny = 0;
    double lx = 0, ly = 0, dt = 0, g = 0;
    hipStream_t stream = nullptr;
    size_t max_bytes = 0, bytes = 0;
    int path = 0;  // 0 auto, 1 multi-pass, 2 LDS
    int xcd = 1;   // XCD-aware column-tile order
    std::vector<void *> allocs;
    DevState *st = nullptr;
    float4 *tx = nullptr, *ty = nullptr;
    double2 *kin_x = nullptr, *kin_y = nullptr, *tw_x = nullptr, *tw_y = nullptr;
    double2 *kh_x = nullptr, *kh_yin = nullptr, *kh_yout = nullptr;
    double *khi_x = nullptr, *khi_yin = nullptr, *khi_yout = nullptr;
    double *kim_x = nullptr, *kim_y = nullptr;
    double *partials = nullptr, *partials2 = nullptr, *hpart = nullptr;
    double *probe = nullptr;  // partials of the density about to be kicked (adiabatic field)
    int npart_max = 0;
    float2 *scratch = nullptr;
    double *knots_x = nullptr, *knots_y = nullptr;
    int knots_cap_x = 0, knots_cap_y = 0;
    GridDev grid{};
    PotDev pot{};
    Shape shape{};
    bool have_theta = false;
    // chunks of steps captured as graphs and replayed (0 real time, 1 imaginary time) on
    // the plan's stream; captured on a private stream, rebuilt when psi or the potential
    // changes (kernel arguments are baked into a graph)
    bool replay = true;  // environment GPE_PLAN_GRAPH=0 at creation: launch every step
    hipStream_t cap = nullptr;
    hipGraph_t graph_def[2] = {nullptr, nullptr};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    const void *graph_psi[2] = {nullptr, nullptr};
    // pass timing (instrumentation)
    int timing_every = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_pairs;  // (kind 0 col / 1 row, index of start event)
};

hipEvent_t *timing_pair(gpe_plan *p, int kind);
int dalloc(gpe_plan *p, void **ptr, size_t bytes);
// Energy loss of psi at time t and its terminal adjoint (lam <- 2 dA H psi); *lat gets
// the loss's derivative by the controlled lattice depth (axis 0: x, 1: y).  Runs on s
// with the plan's own partial buffers and rpart (ny doubles); returns after a sync.
int energy_terminal(gpe_plan *p, const float2 *psi, float2 *lam, double t, int axis, double *rpart, hipStream_t s,
                    double *loss, double *lat);
// launch shape at R points per thread (row passes at row_r, when > 0)
Shape make_shape_r(int nx, int ny, int R, size_t eb, int row_threads, int min_col_tiles, int row_r = 0);
// the launch shape a plan of this size takes (environment overrides included)
Shape plan_shape(int nx, int ny);
// descriptor checks and device views shared by gpe_plan_create / gpe_set_potential and
// the allocation-free entry point
int check_plan_desc(const gpe_plan_desc *d);
int check_potential_desc(const gpe_potential_desc *v);
void griddev_from_desc(GridDev &gd, const gpe_plan_desc *d);
void potdev_from_desc(PotDev &d, const gpe_potential_desc *v, double dt, const float4 *tx, const float4 *ty,
                      const double *knots_x, const double *knots_y);
DevState initial_state(const gpe_potential_desc *v);
void plan_env(gpe_plan *p);

