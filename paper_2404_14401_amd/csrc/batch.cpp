// batch.cpp -- many independent condensates advanced together (gpe_batch_*).
//
// Members are grouped by grid size.  Groups small enough for one work-group's LDS
// run all their steps in a single launch (one work-group per member) on a side
// stream; the other groups run one batched row pass and one batched column pass per
// step over all their members, with chunks of steps replayed from a captured HIP
// graph.  Launch shapes (radix, rows per work-group, column-tile count) of each
// multi-pass group are chosen by gpe_batch_tune, which times the candidates on the
// members' own geometry and keeps the choice in a small text cache.
#include <algorithm>
#include <array>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "runtime_internal.h"

namespace {

struct Tuning {
    int radix = 8, row_threads = 256, min_col_tiles = 256;
};

struct BGroup {
    int nx = 0, ny = 0;
    bool lds = false;
    bool adia = false;  // some member has the adiabatic field: probe passes before its kicks
    bool ode = false;   // some member has the field ODE: Theta reductions and the recurrence
    std::vector<int> members;
    Tuning tune;
    Shape shape{};
    InstDesc *d_inst = nullptr;
    std::vector<InstDesc> h_inst;
    LdsArgs *d_lds = nullptr;
    std::vector<LdsArgs> h_lds;
};

constexpr int kCopyBlocks = 64;  // work-groups per member of a checkpoint save or restore

struct AdjWork {
    int nx = 0, ny = 0, nb = 0;
    int64_t cap_steps = 0;
    std::vector<float2 *> psi, lam;
    std::vector<double *> kick_grad, partials;
    std::vector<double *> probe, aprobe;  // adiabatic field: forward and adjoint probe partials
    bool any_adia = false;                // some member has the adiabatic field
    float2 *ckpt_buf = nullptr;  // checkpoint slots, [slot][member][ny][nx]
    std::vector<float2 *> ckpt;  // [slot * nb + member] into ckpt_buf
    int ckpt_slots = 0;
    float2 **d_ckpt = nullptr;   // device copy of ckpt
    float2 **d_psi = nullptr;    // device copy of psi (nb pointers)
    std::vector<float2 *> traj;  // per member: post-kick states [kick][ny][nx] (stored mode)
    int64_t traj_steps = 0;
    AdjInst *d_adj = nullptr;
    InstDesc *d_fwd = nullptr;
    const float2 **d_pa = nullptr, **d_pb = nullptr;
    float2 **d_dst = nullptr;
    double2 *d_coef = nullptr;
    double *d_sums = nullptr;
    size_t bytes = 0;
};
}  // namespace

struct gpe_batch {
    int n = 0;
    double dt = 0;
    std::vector<gpe_plan *> plans;
    std::vector<BGroup> groups;
    hipStream_t user = nullptr, work = nullptr, side = nullptr;
    hipEvent_t ev_in = nullptr, ev_fork = nullptr, ev_side = nullptr, ev_out = nullptr;
    DevState **d_states = nullptr;     // every member
    DevState **d_states_mp = nullptr;  // members of multi-pass groups
    int *d_flags = nullptr;            // gathered non-finite flags (gpe_batch_sync)
    int n_mp = 0;
    std::vector<void *> allocs;
    bool has_ode = false;  // some multi-pass member has the field ODE
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    int chunk = 50;
    bool warmed = false;
    AdjWork *adj = nullptr;  // adjoint workspace, created by the first gpe_adjoint call
};

static int balloc(gpe_batch *b, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // the failure is reported here, not by the next launch check
        *p = nullptr;
        return fail(GPE_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b->allocs.push_back(*p);
    return GPE_OK;
}

static void bfree(gpe_batch *b, void *p)
{
    if (!p) return;
    (void)hipFree(p);
    b->allocs.erase(std::remove(b->allocs.begin(), b->allocs.end(), p), b->allocs.end());
}

// Which size groups keep each member whole in one work-group's LDS (one work-group per
// member, all steps in one launch) instead of the batched multi-pass kernels.  Measured
// on the MI355X: 64^2 and smaller always pay; 128^2 pays only beside multi-pass groups,
// whose launches it overlaps on the side stream (208-member mixed sweep 8.0e10 vs 6.5e10
// grid-point-steps/s), or with at least one member per CU, while a batch of fewer
// 128^2 members alone runs faster multi-pass (80 adiabatic members: 2.7e10 vs 2.2e10).
// GPE_BATCH_PATH=lds or multipass overrides the choice for every group that can.
// The batched pass launchers are built for line lengths 64..2048 in both directions.
static bool multipass_lines(int nx, int ny) { return nx >= 64 && ny >= 64 && nx <= 2048 && ny <= 2048; }

static void choose_group_paths(std::vector<BGroup> &groups)
{
    const char *force = getenv("GPE_BATCH_PATH");
    const bool all_lds = force && !strcmp(force, "lds"), none = force && !strcmp(force, "multipass");
    bool any_mp = false;
    for (auto &g : groups) {
        g.lds = lds_supported(g.nx, g.ny);
        if (!g.lds) any_mp = true;
    }
    for (auto &g : groups) {
        if (!g.lds) continue;
        if (none) g.lds = !multipass_lines(g.nx, g.ny);
        else if (!all_lds && g.nx * g.ny > 64 * 64) g.lds = any_mp || g.members.size() >= 256;
    }
}

static Shape group_shape(const BGroup &g)
{
    return make_shape_r(g.nx, g.ny, g.tune.radix, xchg_bytes(), g.tune.row_threads, g.tune.min_col_tiles);
}

static void drop_graph(gpe_batch *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->graph_def) (void)hipGraphDestroy(b->graph_def);
    b->graph = nullptr;
    b->graph_def = nullptr;
}

// One multi-pass group: the row pass of relative step n (mode entry/mid/exit).
static int group_row(gpe_batch *b, BGroup &g, int mode, int n, hipStream_t s)
{
    BatchPassArgs a{};
    a.inst = g.d_inst;
    a.blocks_per_inst = g.shape.row_blocks;
    a.per_wg = g.shape.row_lines;
    a.n = n;
    a.cav = (g.adia || g.ode) ? 1 : 0;
    const int blocks = g.shape.row_blocks * (int)g.members.size();
    LAUNCH_OK(launch_row_batched(g.nx, g.tune.radix, mode, a, blocks, g.shape.row_threads, g.shape.row_shmem, s));
    (void)b;
    return GPE_OK;
}

// The column pass of one multi-pass group; first: the column pass of a call's first step.
static int group_col(gpe_batch *b, BGroup &g, hipStream_t s, bool first = false)
{
    BatchPassArgs a{};
    a.inst = g.d_inst;
    a.blocks_per_inst = g.shape.col_blocks;
    a.per_wg = g.shape.col_cols;
    a.ode = g.ode ? 1 : 0;
    a.first = first ? 1 : 0;
    a.row_blocks = g.shape.row_blocks;
    const int blocks = g.shape.col_blocks * (int)g.members.size();
    a.xcd_swizzle = (blocks % 8 == 0 && blocks >= 64) ? 1 : 0;
    LAUNCH_OK(launch_col_batched(g.ny, g.tune.radix, a, blocks, g.shape.col_threads, g.shape.col_shmem, s));
    (void)b;
    return GPE_OK;
}

// `count` middle steps (column pass + merged-kick row pass) of every multi-pass group,
// relative step indices n0 .. n0+count-1; first: the first of them is a call's step 0.
static int mid_steps(gpe_batch *b, int n0, int count, hipStream_t s, bool first = false)
{
    for (int k = 0; k < count; ++k)
        for (auto &g : b->groups) {
            if (g.lds) continue;
            int rc = group_col(b, g, s, first && k == 0);
            if (rc) return rc;
            if (g.adia && (rc = group_row(b, g, ROW_PROBE_MID, n0 + k, s))) return rc;
            if ((rc = group_row(b, g, ROW_MID, n0 + k, s))) return rc;
        }
    return GPE_OK;
}

// The last step of a call for every multi-pass group: column pass, probe (adiabatic
// field), exit row pass, then the field-ODE members' last Theta into their history.
static int exit_step(gpe_batch *b, int n, bool first)
{
    int rc;
    for (auto &g : b->groups)
        if (!g.lds && (rc = group_col(b, g, b->work, first))) return rc;
    for (auto &g : b->groups) {
        if (g.lds) continue;
        if (g.adia && (rc = group_row(b, g, ROW_PROBE_MID, n, b->work))) return rc;
        if ((rc = group_row(b, g, ROW_EXIT, n, b->work))) return rc;
        if (g.ode)
            LAUNCH_OK(launch_tail_batched(g.d_inst, (int)g.members.size(), g.shape.row_blocks, b->work));
    }
    return GPE_OK;
}

static bool has_multipass(const gpe_batch *b)
{
    for (auto &g : b->groups)
        if (!g.lds) return true;
    return false;
}

static int build_graph(gpe_batch *b)
{
    drop_graph(b);
    HIP_OK(hipStreamBeginCapture(b->work, hipStreamCaptureModeThreadLocal));
    int rc = mid_steps(b, 0, b->chunk, b->work);
    hipError_t e2 = launch_advance_t0(b->d_states_mp, b->n_mp, b->chunk * b->dt, b->work);
    hipError_t e = hipStreamEndCapture(b->work, &b->graph_def);
    if (rc) return rc;
    if (e2 != hipSuccess || e != hipSuccess) return fail(GPE_ERR_DEVICE, "graph capture failed");
    HIP_OK(hipGraphInstantiate(&b->graph, b->graph_def, nullptr, nullptr, 0));
    return GPE_OK;
}

extern "C" {

int gpe_batch_create(gpe_batch **out, int n, const gpe_plan_desc *descs, const gpe_potential_desc *pots)
{
    if (!out || !descs || !pots || n < 1) return fail(GPE_ERR_INVALID, "need n >= 1 descriptions and potentials");
    *out = nullptr;
    for (int i = 0; i < n; ++i)
        if (descs[i].dt != descs[0].dt) return fail(GPE_ERR_INVALID, "batch members must share dt");
    gpe_batch *b = new gpe_batch();
    b->n = n;
    b->dt = descs[0].dt;
    b->user = (hipStream_t)descs[0].stream;
    auto cleanup = [&](int rc) {
        gpe_batch_destroy(b);
        return rc;
    };
    int rc = 0;
    for (int i = 0; i < n; ++i) {
        gpe_plan_desc d = descs[i];
        d.stream = nullptr;
        gpe_plan *p = nullptr;
        if ((rc = gpe_plan_create(&p, &d))) return cleanup(rc);
        b->plans.push_back(p);
        if ((rc = gpe_set_potential(p, &pots[i]))) return cleanup(rc);
    }
    HIP_OK(hipStreamCreateWithFlags(&b->work, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    for (hipEvent_t *e : {&b->ev_in, &b->ev_fork, &b->ev_side, &b->ev_out})
        HIP_OK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    for (int i = 0; i < n; ++i) {
        gpe_plan *p = b->plans[i];
        auto it = std::find_if(b->groups.begin(), b->groups.end(),
                               [&](const BGroup &g) { return g.nx == p->nx && g.ny == p->ny; });
        if (it == b->groups.end()) {
            BGroup g;
            g.nx = p->nx;
            g.ny = p->ny;
            // untuned shape: 64 threads per row work-group (several lines each up to 512
            // points per row, one line from 1024 on; 2-3% faster than 128 on the 208-member mix,
            // 80 x 128^2 and 16 x 512^2), and 128 column tiles per member up to 512 points per
            // row, 256 beyond (which the member-count rule below refines up to 512 points;
            // against the 256/256 shape before it, us per batch step: 64 x 256^2 56.1 vs 75.3,
            // 16 x 512^2 53.0 vs 56.3, 2 x 1024^2 49.8 vs 50.5, 4 x 1024^2 76.9 vs 76.9)
            g.tune = Tuning{8, 64, g.nx <= 512 ? 128 : 256};
            b->groups.push_back(g);
            it = b->groups.end() - 1;
        }
        it->members.push_back(i);
    }
    choose_group_paths(b->groups);
    for (auto &g : b->groups)
        if (!g.lds && !multipass_lines(g.nx, g.ny))
            return cleanup(fail(GPE_ERR_UNSUPPORTED, "batch member of " + std::to_string(g.nx) + " x " +
                                                         std::to_string(g.ny) +
                                                         ": beyond one work-group's LDS, both sides must be 64..2048 "
                                                         "(a plan takes it)"));
    std::vector<DevState *> states(n);
    for (int i = 0; i < n; ++i) states[i] = b->plans[i]->st;
    if ((rc = balloc(b, (void **)&b->d_states, sizeof(DevState *) * n))) return cleanup(rc);
    if ((rc = balloc(b, (void **)&b->d_flags, sizeof(int) * n))) return cleanup(rc);
    HIP_OK(hipMemcpy(b->d_states, states.data(), sizeof(DevState *) * n, hipMemcpyHostToDevice));
    // the time base of multi-pass members is advanced by the graph while the LDS groups
    // (side stream) read theirs, so the two sets are kept apart
    std::vector<DevState *> mp;
    for (auto &g : b->groups)
        if (!g.lds)
            for (int i : g.members) mp.push_back(b->plans[i]->st);
    b->n_mp = (int)mp.size();
    if (b->n_mp) {
        if ((rc = balloc(b, (void **)&b->d_states_mp, sizeof(DevState *) * mp.size()))) return cleanup(rc);
        HIP_OK(hipMemcpy(b->d_states_mp, mp.data(), sizeof(DevState *) * mp.size(), hipMemcpyHostToDevice));
    }
    const char *tiles_env = getenv("GPE_BATCH_TILES");
    const bool fixed_tiles = tiles_env && !strcmp(tiles_env, "fixed");
    for (auto &g : b->groups) {
        const size_t m = g.members.size();
        if (g.lds) {
            g.h_lds.resize(m);
            for (size_t k = 0; k < m; ++k) {
                gpe_plan *p = b->plans[g.members[k]];
                LdsArgs a{};
                a.grid = p->grid;
                a.pot = p->pot;
                a.st = p->st;
                g.h_lds[k] = a;
            }
            if ((rc = balloc(b, (void **)&g.d_lds, sizeof(LdsArgs) * m))) return cleanup(rc);
        } else {
            if (!fixed_tiles && g.ny <= 512) {
                // untuned column tiles of columns up to 512 points: the widest that a
                // 1024-thread work-group and a 128-byte line of complex64 allow (16 columns),
                // halved while the group would launch fewer than 1024 column work-groups.
                // Measured against the default above, Gpts/s: 200 x 128^2 multi-pass 46.7 ->
                // 74.4, 80 x 128^2 adiabatic 27.2 -> 35.2, the 208-member mix 77.6 -> 80.8,
                // 16 x 512^2 77.7 -> 79.5; at 1024 points it lost (2 x 1024^2 43.6 -> 41.5,
                // 64 x 1024^2 74.5 -> 72.2), where the XCD tile order already shares the lines.
                // (GPE_BATCH_TILES=fixed keeps the default above everywhere.)
                const int tc = std::max(1, g.ny / g.tune.radix);
                int w = std::max(1, std::min({16, g.nx, 1024 / tc}));
                while (w > 1 && (int64_t)m * (g.nx / w) < 1024) w /= 2;
                g.tune.min_col_tiles = g.nx / w;
            }
            g.shape = group_shape(g);
            g.h_inst.resize(m);
            for (size_t k = 0; k < m; ++k) {
                gpe_plan *p = b->plans[g.members[k]];
                InstDesc d{};
                d.grid = p->grid;
                d.pot = p->pot;
                d.st = p->st;
                if (p->pot.cavity == GPE_CAVITY_ADIABATIC) {
                    // one partial record per row work-group, for any row shape the tuner picks
                    if ((rc = balloc(b, (void **)&d.probe, sizeof(double) * NPART * g.ny))) return cleanup(rc);
                    g.adia = true;
                }
                if (p->pot.cavity == GPE_CAVITY_ODE) {
                    if ((rc = balloc(b, (void **)&d.partials, sizeof(double) * NPART * g.ny))) return cleanup(rc);
                    g.ode = true;
                    b->has_ode = true;
                }
                g.h_inst[k] = d;
            }
            if ((rc = balloc(b, (void **)&g.d_inst, sizeof(InstDesc) * m))) return cleanup(rc);
        }
    }
    *out = b;
    return GPE_OK;
}

int gpe_batch_destroy(gpe_batch *b)
{
    if (!b) return GPE_OK;
    if (b->work) (void)hipStreamSynchronize(b->work);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graph(b);
    delete b->adj;
    for (gpe_plan *p : b->plans) gpe_plan_destroy(p);
    for (void *a : b->allocs) (void)hipFree(a);
    for (hipEvent_t e : {b->ev_in, b->ev_fork, b->ev_side, b->ev_out})
        if (e) (void)hipEventDestroy(e);
    if (b->work) (void)hipStreamDestroy(b->work);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
    return GPE_OK;
}

// Point every member's descriptor at its wave function (and, for the LDS groups, at
// the step count of this call).
static int bind_psis(gpe_batch *b, gpe_c64 *const *psis, int64_t nsteps, bool ensure_len = true)
{
    for (auto &g : b->groups) {
        const size_t m = g.members.size();
        if (g.lds) {
            for (size_t k = 0; k < m; ++k) {
                g.h_lds[k].psi = (float2 *)psis[g.members[k]];
                g.h_lds[k].nsteps = (int)nsteps;
            }
            HIP_OK(hipMemcpyAsync(g.d_lds, g.h_lds.data(), sizeof(LdsArgs) * m, hipMemcpyHostToDevice, b->work));
        } else {
            for (size_t k = 0; k < m; ++k) {
                g.h_inst[k].psi = (float2 *)psis[g.members[k]];
                g.h_inst[k].first_theta = b->plans[g.members[k]]->have_theta ? 0 : 1;
            }
            HIP_OK(hipMemcpyAsync(g.d_inst, g.h_inst.data(), sizeof(InstDesc) * m, hipMemcpyHostToDevice, b->work));
        }
    }
    (void)ensure_len;
    return GPE_OK;
}

int gpe_step_batched(gpe_batch *b, gpe_c64 *const *psis, int64_t nsteps, double t0)
{
    if (!b || !psis || nsteps < 0) return fail(GPE_ERR_INVALID, "null batch/psis or negative nsteps");
    if (!std::isfinite(t0)) return fail(GPE_ERR_INVALID, "t0 must be finite");
    for (int i = 0; i < b->n; ++i)
        if (!psis[i]) return fail(GPE_ERR_INVALID, "null member wave function");
    if (nsteps == 0) return GPE_OK;
    if (nsteps > (1 << 30)) return fail(GPE_ERR_INVALID, "nsteps too large for one call");
    HIP_OK(hipEventRecord(b->ev_in, b->user));
    HIP_OK(hipStreamWaitEvent(b->work, b->ev_in, 0));
    int rc = bind_psis(b, psis, nsteps);
    if (rc) return rc;
    LAUNCH_OK(launch_set_call_batched(b->d_states, b->n, t0, b->work));
    // LDS-resident groups: all steps in one launch on the side stream
    bool side_used = false;
    HIP_OK(hipEventRecord(b->ev_fork, b->work));
    for (auto &g : b->groups) {
        if (!g.lds) continue;
        if (!side_used) HIP_OK(hipStreamWaitEvent(b->side, b->ev_fork, 0));
        side_used = true;
        // bounded launches (about 2^26 point-steps per member each): a long call is a
        // sequence of kernels of well under a second, not one kernel of minutes
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(1 << 20, (1LL << 26) / ((int64_t)g.nx * g.ny)));
        for (int64_t s0 = 0; s0 < nsteps; s0 += chunk)
            LAUNCH_OK(launch_lds_batched(g.nx, g.ny, g.d_lds, (int)g.members.size(), s0,
                                         (int)std::min<int64_t>(chunk, nsteps - s0), b->side));
    }
    if (side_used) HIP_OK(hipEventRecord(b->ev_side, b->side));
    // multi-pass groups
    if (has_multipass(b)) {
        for (auto &g : b->groups) {
            if (g.lds) continue;
            if (g.adia && (rc = group_row(b, g, ROW_PROBE_REAL, 0, b->work))) return rc;
            if ((rc = group_row(b, g, ROW_ENTRY, 0, b->work))) return rc;
        }
        int64_t mids = nsteps - 1, done = 0;
        // step 0 directly: the first call's launches load the kernels, and a field-ODE
        // member's first column pass treats its overlap history differently
        if ((!b->warmed || b->has_ode) && mids > 0) {
            if ((rc = mid_steps(b, 0, 1, b->work, true))) return rc;
            done = 1;
            b->warmed = true;
        }
        // chunks replayed from the captured graph use steps relative to st->t0,
        // which the graph advances by chunk*dt at its end
        if (mids - done >= b->chunk) {
            if (done > 0) LAUNCH_OK(launch_advance_t0(b->d_states_mp, b->n_mp, done * b->dt, b->work));
            if (!b->graph && (rc = build_graph(b))) return rc;
            while (mids - done >= b->chunk) {
                HIP_OK(hipGraphLaunch(b->graph, b->work));
                done += b->chunk;
            }
            if ((rc = mid_steps(b, 0, (int)(mids - done), b->work))) return rc;
            if ((rc = exit_step(b, (int)(mids - done), false))) return rc;
        } else {
            if ((rc = mid_steps(b, (int)done, (int)(mids - done), b->work, done == 0))) return rc;
            if ((rc = exit_step(b, (int)mids, mids == 0))) return rc;
        }
        for (auto &g : b->groups)
            if (!g.lds && g.ode)
                for (int i : g.members) b->plans[i]->have_theta = true;
    }
    if (side_used) HIP_OK(hipStreamWaitEvent(b->work, b->ev_side, 0));
    HIP_OK(hipEventRecord(b->ev_out, b->work));
    HIP_OK(hipStreamWaitEvent(b->user, b->ev_out, 0));
    return GPE_OK;
}

// Time batched calls of `steps` steps over every member's scratch array (contents
// irrelevant to the timing): all groups at once, the LDS-resident ones on their side
// stream, as a call runs them.  Best of two calls after one that loads kernels and
// captures the step graph; microseconds per step, or 1e30 when a shape cannot launch.
// The members' device states and history flags are restored by the caller.
static double time_batch(gpe_batch *b, int steps)
{
    std::vector<gpe_c64 *> psis(b->n, nullptr);
    for (int i = 0; i < b->n; ++i) psis[i] = (gpe_c64 *)b->plans[i]->scratch;
    drop_graph(b);
    if (gpe_step_batched(b, psis.data(), steps, 0.0) || hipStreamSynchronize(b->work) != hipSuccess) return 1e30;
    double best = 1e30;
    for (int it = 0; it < 2; ++it) {
        auto t = std::chrono::steady_clock::now();
        if (gpe_step_batched(b, psis.data(), steps, 0.0) || hipStreamSynchronize(b->work) != hipSuccess) return 1e30;
        best = std::min(best, std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t).count());
    }
    return best / steps;
}

int gpe_batch_tune(gpe_batch *b, const char *cache_path)
{
    if (!b) return fail(GPE_ERR_INVALID, "null batch");
    hipDeviceProp_t prop;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    const std::string arch = prop.gcnArchName;
    std::vector<std::string> lines;
    if (cache_path && *cache_path) {
        std::ifstream f(cache_path);
        std::string l;
        while (std::getline(f, l)) lines.push_back(l);
    }
    // the timing runs advance the members' cavity states and history flags: keep them and
    // put them back
    std::vector<DevState> saved(b->n);
    std::vector<char> had_theta(b->n);
    HIP_OK(hipStreamSynchronize(b->work));
    for (int i = 0; i < b->n; ++i) {
        HIP_OK(hipMemcpy(&saved[i], b->plans[i]->st, sizeof(DevState), hipMemcpyDeviceToHost));
        had_theta[i] = b->plans[i]->have_theta ? 1 : 0;
    }
    // the shapes interact (the multi-pass groups run one after another beside the LDS
    // groups on the side stream, and share the caches), so they are tuned on whole batched
    // steps, one group at a time with the others held, and cached for this composition
    std::ostringstream comp;
    for (auto &g : b->groups) comp << (g.lds ? " L" : " M") << g.nx << "x" << g.ny << "x" << g.members.size();
    auto key_of = [&](const BGroup &g) {
        std::ostringstream key;
        key << arch << " " << g.nx << " " << g.ny << " " << g.members.size() << " in" << comp.str() << " :";
        return key.str();
    };
    bool all_cached = true;
    for (auto &g : b->groups) {
        if (g.lds) continue;
        bool found = false;
        for (auto &l : lines) {
            if (l.rfind(key_of(g) + " ", 0) == 0) {
                std::istringstream is(l.substr(key_of(g).size()));
                Tuning t;
                double us;
                if (is >> t.radix >> t.row_threads >> t.min_col_tiles >> us) {
                    g.tune = t;
                    g.shape = group_shape(g);
                    found = true;
                }
            }
        }
        all_cached = all_cached && found;
    }
    bool changed = false;
    if (!all_cached) {
        for (int i = 0; i < b->n; ++i)
            (void)hipMemsetAsync(b->plans[i]->scratch, 0, sizeof(float2) * (size_t)b->plans[i]->nx * b->plans[i]->ny,
                                 b->work);
        const int steps = 2 * b->chunk + 8;
        std::vector<double> best_us(b->groups.size(), 1e30);
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            BGroup &g = b->groups[gi];
            if (g.lds) continue;
            Tuning best = g.tune;
            // column tiles per member from whole-line tiles (16 columns of complex64, at
            // 16..64 tiles) to narrow ones that spread a member over more work-groups
            for (int r : {8, 4})
                for (int rt : {64, 128, 256, 512})
                    for (int mt : {16, 32, 64, 128, 256, 512}) {
                        if (g.nx / r > 512 || g.ny / r > 1024 || g.nx > 2048 || g.ny > 2048) continue;
                        g.tune = {r, rt, mt};
                        g.shape = group_shape(g);
                        if (g.shape.row_threads > 512 || g.shape.col_threads > 1024) continue;
                        const double us = time_batch(b, steps);
                        if (us < best_us[gi]) {
                            best_us[gi] = us;
                            best = g.tune;
                        }
                    }
            g.tune = best;
            g.shape = group_shape(g);
        }
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            const BGroup &g = b->groups[gi];
            if (g.lds) continue;
            std::ostringstream l;
            l << key_of(g) << " " << g.tune.radix << " " << g.tune.row_threads << " " << g.tune.min_col_tiles << " "
              << best_us[gi];
            lines.push_back(l.str());
        }
        changed = true;
    }
    HIP_OK(hipStreamSynchronize(b->work));
    HIP_OK(hipStreamSynchronize(b->side));
    for (int i = 0; i < b->n; ++i) {
        HIP_OK(hipMemcpy(b->plans[i]->st, &saved[i], sizeof(DevState), hipMemcpyHostToDevice));
        b->plans[i]->have_theta = had_theta[i] != 0;
    }
    drop_graph(b);
    b->warmed = false;
    if (changed && cache_path && *cache_path) {
        std::ofstream f(cache_path);
        for (auto &l : lines) f << l << "\n";
    }
    HIP_OK(hipStreamSynchronize(b->work));
    return GPE_OK;
}

int gpe_batch_info(gpe_batch *b, int group, int out[8])
{
    if (!b || !out || group < 0 || group >= (int)b->groups.size()) return fail(GPE_ERR_INVALID, "bad group");
    const BGroup &g = b->groups[group];
    out[0] = g.nx;
    out[1] = g.ny;
    out[2] = (int)g.members.size();
    out[3] = g.lds ? 1 : 0;
    out[4] = g.tune.radix;
    out[5] = g.shape.row_threads;
    out[6] = g.shape.col_blocks;
    out[7] = (int)b->groups.size();
    return GPE_OK;
}

int gpe_batch_sync(gpe_batch *b, int *first_bad)
{
    if (!b) return fail(GPE_ERR_INVALID, "null batch");
    if (first_bad) *first_bad = -1;
    HIP_OK(hipStreamSynchronize(b->work));
    HIP_OK(hipStreamSynchronize(b->side));
    std::vector<int> flags((size_t)b->n, 0);
    LAUNCH_OK(launch_gather_flags(b->d_states, b->n, b->d_flags, b->work));
    HIP_OK(hipMemcpyAsync(flags.data(), b->d_flags, sizeof(int) * (size_t)b->n, hipMemcpyDeviceToHost, b->work));
    HIP_OK(hipStreamSynchronize(b->work));
    for (int i = 0; i < b->n; ++i)
        if (flags[i]) {
            if (first_bad) *first_bad = i;
            return fail(GPE_ERR_NONFINITE, "non-finite values in the wave function of batch member " + std::to_string(i));
        }
    return GPE_OK;
}

int gpe_batch_get_cavity(gpe_batch *b, int member, double out[4])
{
    if (!b || !out || member < 0 || member >= b->n) return fail(GPE_ERR_INVALID, "bad member");
    HIP_OK(hipStreamSynchronize(b->work));
    HIP_OK(hipStreamSynchronize(b->side));
    return gpe_get_cavity(b->plans[member], out);
}

// --------------------------------------------------------------------- adjoint


// The batch owns its adjoint workspace (its device buffers are in b->allocs).
static AdjWork *adj_work(gpe_batch *b)
{
    if (!b->adj) b->adj = new AdjWork();
    return b->adj;
}

// Hat weights of the piecewise-linear schedule at time t (same clamping as the device).
static void hat(const gpe_schedule &s, double t, int *i0, double *w0, double *w1)
{
    const int m = s.nknots;
    if (t <= s.t0) { *i0 = 0; *w0 = 1; *w1 = 0; return; }
    if (t >= s.t1) { *i0 = m - 2; *w0 = 0; *w1 = 1; return; }
    double u = (t - s.t0) / (s.t1 - s.t0) * (m - 1);
    int i = (int)std::floor(u);
    if (i >= m - 1) i = m - 2;
    *i0 = i;
    *w1 = u - i;
    *w0 = 1.0 - *w1;
}

static int adj_alloc(gpe_batch *b, AdjWork *w, int nx, int ny, int nb, int64_t nsteps, int slots,
                     int64_t traj_steps = 0)
{
    const size_t npts = (size_t)nx * ny;
    if (w->nx != nx || w->ny != ny || w->nb != nb) {
        if (w->nb) return fail(GPE_ERR_INVALID, "adjoint workspace already sized for another batch shape");
        w->nx = nx;
        w->ny = ny;
        w->nb = nb;
        w->psi.resize(nb);
        w->lam.resize(nb);
        w->kick_grad.resize(nb);
        w->partials.resize(nb);
        w->probe.resize(nb);
        w->aprobe.resize(nb);
        for (int i = 0; i < nb; ++i) {
            int rc;
            if ((rc = balloc(b, (void **)&w->psi[i], sizeof(float2) * npts))) return rc;
            if ((rc = balloc(b, (void **)&w->lam[i], sizeof(float2) * npts))) return rc;
            if ((rc = balloc(b, (void **)&w->partials[i], sizeof(double) * 4096))) return rc;
            if ((rc = balloc(b, (void **)&w->probe[i], sizeof(double) * NPART * 4096))) return rc;
            if ((rc = balloc(b, (void **)&w->aprobe[i], sizeof(double) * NPART * 4096))) return rc;
            w->bytes += 2 * sizeof(float2) * npts;
        }
        int rc;
        if ((rc = balloc(b, (void **)&w->d_adj, sizeof(AdjInst) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_fwd, sizeof(InstDesc) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_pa, sizeof(void *) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_pb, sizeof(void *) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_dst, sizeof(void *) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_coef, sizeof(double2) * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_sums, sizeof(double) * 4 * 64 * nb))) return rc;
        if ((rc = balloc(b, (void **)&w->d_psi, sizeof(void *) * nb))) return rc;
        HIP_OK(hipMemcpy(w->d_psi, w->psi.data(), sizeof(void *) * nb, hipMemcpyHostToDevice));
    }
    if (nsteps + 1 > w->cap_steps) {
        for (int i = 0; i < nb; ++i) {
            bfree(b, w->kick_grad[i]);  // replaced by a longer one
            int rc;
            if ((rc = balloc(b, (void **)&w->kick_grad[i], sizeof(double) * (size_t)(nsteps + 1)))) return rc;
        }
        w->cap_steps = nsteps + 1;
    }
    if (w->ckpt_slots < slots) {
        // every slot of every member in one allocation (a first call pays one hipMalloc, not
        // one per member and slot), replaced by a larger one when a call needs more slots;
        // slots hold nothing from call to call
        const size_t slot_bytes = sizeof(float2) * npts * nb;
        bfree(b, w->ckpt_buf);
        bfree(b, w->d_ckpt);
        w->bytes -= std::min(w->bytes, (size_t)w->ckpt_slots * slot_bytes);
        w->ckpt_buf = nullptr;
        w->d_ckpt = nullptr;
        w->ckpt.clear();
        w->ckpt_slots = 0;
        int rc;
        if ((rc = balloc(b, (void **)&w->ckpt_buf, slot_bytes * slots))) return rc;
        if ((rc = balloc(b, (void **)&w->d_ckpt, sizeof(void *) * (size_t)slots * nb))) {
            bfree(b, w->ckpt_buf);
            w->ckpt_buf = nullptr;
            return rc;
        }
        for (size_t k = 0; k < (size_t)slots * nb; ++k) w->ckpt.push_back(w->ckpt_buf + k * npts);
        HIP_OK(hipMemcpy(w->d_ckpt, w->ckpt.data(), sizeof(void *) * w->ckpt.size(), hipMemcpyHostToDevice));
        w->ckpt_slots = slots;
        w->bytes += slot_bytes * slots;
    }
    if (traj_steps > w->traj_steps) {
        // one buffer per member, replaced (not kept alongside) when a longer run needs more
        for (float2 *p : w->traj) bfree(b, p);
        w->bytes -= std::min(w->bytes, (size_t)w->traj_steps * nb * sizeof(float2) * npts);
        w->traj.assign(nb, nullptr);
        w->traj_steps = 0;
        for (int i = 0; i < nb; ++i) {
            int rc;
            if ((rc = balloc(b, (void **)&w->traj[i], sizeof(float2) * npts * (size_t)traj_steps))) {
                for (float2 *&p : w->traj) {
                    bfree(b, p);
                    p = nullptr;
                }
                return rc;
            }
        }
        w->traj_steps = traj_steps;
        w->bytes += (size_t)traj_steps * nb * sizeof(float2) * npts;
    }
    return GPE_OK;
}

// Host sums of pair_sums partials: {Re <a|b>, Im <a|b>, |a-b|^2, |b|^2} per member.
static int pair_sums(gpe_batch *b, AdjWork *w, const std::vector<const float2 *> &pa,
                     const std::vector<const float2 *> &pb, std::vector<std::array<double, 4>> &out)
{
    const int per = 64, nb = w->nb;
    HIP_OK(hipMemcpyAsync(w->d_pa, pa.data(), sizeof(void *) * nb, hipMemcpyHostToDevice, b->work));
    HIP_OK(hipMemcpyAsync(w->d_pb, pb.data(), sizeof(void *) * nb, hipMemcpyHostToDevice, b->work));
    LAUNCH_OK(launch_pair_sums(w->d_pa, w->d_pb, (size_t)w->nx * w->ny, nb, per, w->d_sums, b->work));
    std::vector<double> h((size_t)4 * per * nb);
    HIP_OK(hipMemcpyAsync(h.data(), w->d_sums, sizeof(double) * h.size(), hipMemcpyDeviceToHost, b->work));
    HIP_OK(hipStreamSynchronize(b->work));
    out.assign(nb, {0, 0, 0, 0});
    for (int i = 0; i < nb; ++i)
        for (int l = 0; l < per; ++l)
            for (int k = 0; k < 4; ++k) out[i][k] += h[((size_t)i * per + l) * 4 + k];
    return GPE_OK;
}

// Forward real-time steps [n0, n1) of every member on the adjoint workspace (batched
// multi-pass kernels, time base st->t0 = t0 + n0 dt).
static int adj_forward(gpe_batch *b, AdjWork *w, const Shape &sh, int radix, double t0, int64_t n0, int64_t n1,
                       bool record = false)
{
    const int nb = w->nb;
    LAUNCH_OK(launch_set_call_batched(b->d_states, b->n, t0 + n0 * b->dt, b->work));
    BatchPassArgs ra{}, ca{};
    ra.inst = w->d_fwd;
    ra.cav = w->any_adia ? 1 : 0;
    ra.traj = record ? 1 : 0;
    ra.blocks_per_inst = sh.row_blocks;
    ra.per_wg = sh.row_lines;
    ca.inst = w->d_fwd;
    ca.blocks_per_inst = sh.col_blocks;
    ca.per_wg = sh.col_cols;
    const int rblocks = sh.row_blocks * nb, cblocks = sh.col_blocks * nb;
    ca.xcd_swizzle = (cblocks % 8 == 0 && cblocks >= 64) ? 1 : 0;
    const int64_t k = n1 - n0;
    ra.n = 0;
    if (w->any_adia)
        LAUNCH_OK(launch_row_batched(w->nx, radix, ROW_PROBE_REAL, ra, rblocks, sh.row_threads, sh.row_shmem, b->work));
    LAUNCH_OK(launch_row_batched(w->nx, radix, ROW_ENTRY, ra, rblocks, sh.row_threads, sh.row_shmem, b->work));
    for (int64_t j = 0; j < k; ++j) {
        LAUNCH_OK(launch_col_batched(w->ny, radix, ca, cblocks, sh.col_threads, sh.col_shmem, b->work));
        ra.n = (int)j;
        if (w->any_adia)
            LAUNCH_OK(launch_row_batched(w->nx, radix, ROW_PROBE_MID, ra, rblocks, sh.row_threads, sh.row_shmem, b->work));
        LAUNCH_OK(launch_row_batched(w->nx, radix, j + 1 < k ? ROW_MID : ROW_EXIT, ra, rblocks, sh.row_threads,
                                     sh.row_shmem, b->work));
    }
    return GPE_OK;
}

// Reverse sweep over steps [n0, n1) (from n1 down to n0): on entry psi holds psi_{n1}
// and lam the adjoint at n1 (real space); on exit psi_{n0} (reconstructed) and lam_{n0}.
// stored: the kick outputs come from the members' trajectories, psi stays psi_{n1}.
static int adj_reverse(gpe_batch *b, AdjWork *w, const Shape &sh, double t0, int64_t n0, int64_t n1,
                       bool stored = false)
{
    const int nb = w->nb;
    LAUNCH_OK(launch_set_call_batched(b->d_states, b->n, t0, b->work));
    AdjPassArgs ra{}, ca{};
    ra.inst = w->d_adj;
    ra.blocks_per_inst = sh.row_blocks;
    ra.per_wg = sh.row_lines;
    ca.inst = w->d_adj;
    ca.blocks_per_inst = sh.col_blocks;
    ca.per_wg = sh.col_cols;
    ca.row_blocks = sh.row_blocks;
    const int rblocks = sh.row_blocks * nb, cblocks = sh.col_blocks * nb;
    ca.xcd_swizzle = (cblocks % 8 == 0 && cblocks >= 64) ? 1 : 0;
    ra.traj = ca.traj = stored ? 1 : 0;
    const int arrays = stored ? 1 : 2;
    const size_t rsh = adj_row_shmem(w->nx, sh.row_lines, 8, arrays), csh = adj_col_shmem(w->ny, sh.col_cols, 8, arrays);
    ra.kick = (int)n1;
    if (w->any_adia)
        LAUNCH_OK(launch_row_adj(w->nx, ADJ_PROBE_FIRST, ra, rblocks, sh.row_threads, rsh, b->work));
    LAUNCH_OK(launch_row_adj(w->nx, ADJ_FIRST, ra, rblocks, sh.row_threads, rsh, b->work));
    int pending = (int)n1;
    for (int64_t n = n1 - 1; n >= n0; --n) {
        ca.tail_kick = pending;
        LAUNCH_OK(launch_col_adj(w->ny, ca, cblocks, sh.col_threads, csh, b->work));
        ra.kick = (int)n;
        if (w->any_adia)
            LAUNCH_OK(launch_row_adj(w->nx, ADJ_PROBE_MID, ra, rblocks, sh.row_threads, rsh, b->work));
        LAUNCH_OK(launch_row_adj(w->nx, n > n0 ? ADJ_MID : ADJ_LAST, ra, rblocks, sh.row_threads, rsh, b->work));
        pending = (int)n;
    }
    LAUNCH_OK(launch_adj_tail(w->d_adj, nb, sh.row_blocks, pending, b->work));
    return GPE_OK;
}

int gpe_adjoint(gpe_batch *b, const gpe_c64 *const *psi0, const gpe_c64 *const *target, int64_t nsteps, double t0,
                const double *knots, int nknots, int control, int loss_kind, int mode, double drift_tol, double *loss,
                double *grad, gpe_c64 *const *psi_final, double *info)
{
    if (control != GPE_CONTROL_X_LATTICE && control != GPE_CONTROL_PUMP)
        return fail(GPE_ERR_INVALID, "control must be GPE_CONTROL_X_LATTICE or GPE_CONTROL_PUMP");
    const bool pump = control == GPE_CONTROL_PUMP;
    if (!b || !psi0 || !loss || nsteps < 1 || !knots) return fail(GPE_ERR_INVALID, "null argument or nsteps < 1");
    const bool loss_only = grad == nullptr;  // forward sweep and loss, no reverse sweep
    if (loss_kind != GPE_LOSS_FIDELITY && loss_kind != GPE_LOSS_ENERGY) return fail(GPE_ERR_INVALID, "bad loss kind");
    const bool energy = loss_kind == GPE_LOSS_ENERGY;
    if (!energy && !target) return fail(GPE_ERR_INVALID, "fidelity loss needs target states");
    if (mode < GPE_ADJ_AUTO || mode > GPE_ADJ_STORE) return fail(GPE_ERR_INVALID, "bad adjoint mode");
    const bool store = mode == GPE_ADJ_STORE && !loss_only;
    if (nsteps > (1 << 28)) return fail(GPE_ERR_INVALID, "nsteps too large");
    const int nb = b->n;
    const int nx = b->plans[0]->nx, ny = b->plans[0]->ny;
    for (int i = 0; i < nb; ++i) {
        gpe_plan *p = b->plans[i];
        if (p->nx != nx || p->ny != ny) return fail(GPE_ERR_INVALID, "adjoint members must share the grid size");
        const Sched &ctl = pump ? p->pot.sy : p->pot.sx;
        if (ctl.kind != GPE_SCHED_KNOTS || ctl.nknots != nknots)
            return fail(GPE_ERR_INVALID, "members need a knot schedule with nknots values on the controlled lattice");
        if (p->pot.cavity == GPE_CAVITY_ODE)
            return fail(GPE_ERR_UNSUPPORTED, "adjoint with the field-ODE cavity (the adiabatic field is supported)");
        if (energy && p->pot.cavity != GPE_CAVITY_OFF)
            return fail(GPE_ERR_UNSUPPORTED, "the energy loss with a cavity (fidelity only there)");
        if (!psi0[i] || (!energy && !target[i])) return fail(GPE_ERR_INVALID, "null member state");
        // the knots replace the controlled schedule's values: the checks gpe_set_potential
        // applies to a schedule apply to them too
        for (int m = 0; m < nknots; ++m) {
            const double k = knots[(size_t)i * nknots + m];
            if (!std::isfinite(k)) return fail(GPE_ERR_INVALID, "knot values must be finite");
            // the interference lattice's sqrt(Vp U0) needs the pump and U0 on one side of
            // zero, and its derivative by Vp is singular at Vp = 0
            if (pump && p->pot.cavity != GPE_CAVITY_OFF && !(k * p->pot.vc > 0))
                return fail(GPE_ERR_INVALID, "pump knots of a cavity member must share the sign of vc and be nonzero");
        }
    }
    if (nx < 64 || ny < 64 || nx > 1024 || ny > 1024) return fail(GPE_ERR_UNSUPPORTED, "adjoint grid sizes 64..1024");
    // launch shape of the adjoint's passes: 256 threads per row work-group and at least
    // 128 column tiles per member, measured best at 16 x 512^2 against row 128/512 and
    // 32..512 tiles; the stored trajectory's passes (the adjoint alone) at least 64, which
    // there took 0.244 s against 0.253 s for 2000 steps, where reconstruction lost 3%
    // (environment GPE_ADJ_ROW_THREADS, GPE_ADJ_MIN_COL_TILES for tuning runs)
    auto env = [](const char *name, int dflt) {
        const char *v = getenv(name);
        return v && *v ? atoi(v) : dflt;
    };
    const int art = env("GPE_ADJ_ROW_THREADS", 256), act = env("GPE_ADJ_MIN_COL_TILES", store ? 64 : 128);
    Shape sh = make_shape_r(nx, ny, 8, xchg_bytes(), art, act);
    if (sh.col_threads > 512) sh = make_shape_r(nx, ny, 8, xchg_bytes(), art, nx / std::max(1, 512 / (ny / 8)));
    if (sh.col_threads > 512) return fail(GPE_ERR_UNSUPPORTED, "column shape");
    // the adjoint column pass holds two exchange areas: narrow the tiles until they fit LDS
    for (int tiles = nx / sh.col_cols * 2; adj_col_shmem(ny, sh.col_cols, 8, 2) > 158 * 1024 && sh.col_cols > 1;
         tiles *= 2)
        sh = make_shape_r(nx, ny, 8, xchg_bytes(), art, tiles);
    if (adj_col_shmem(ny, sh.col_cols, 8, 2) > 158 * 1024 || adj_row_shmem(nx, sh.row_lines, 8, 2) > 158 * 1024)
        return fail(GPE_ERR_UNSUPPORTED, "adjoint passes exceed the LDS of a work-group");
    // the forward sweep takes the batch's own (tuned) shape of this grid size where the
    // group runs the batched passes, at radix 8 for the stored trajectory (whose recording
    // kernels are radix 8 only); else the adjoint's shape
    Shape fsh = sh;
    int fr = 8;
    for (auto &g : b->groups)
        if (!g.lds && g.nx == nx && g.ny == ny && (g.tune.radix == 8 || !store)) {
            fsh = g.shape;
            fr = g.tune.radix;
        }
    AdjWork *w = adj_work(b);
    const int64_t seg = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)nsteps)));
    const int64_t nseg = (nsteps + seg - 1) / seg;
    int rc = adj_alloc(b, w, nx, ny, nb, nsteps,
                       (!loss_only && (mode == GPE_ADJ_AUTO || mode == GPE_ADJ_CHECKPOINT)) ? (int)nseg : 0,
                       store ? nsteps : 0);
    if (rc) return rc;
    const size_t npts = (size_t)nx * ny;
    HIP_OK(hipEventRecord(b->ev_in, b->user));
    HIP_OK(hipStreamWaitEvent(b->work, b->ev_in, 0));
    // controls: the members' knot values of the controlled lattice
    for (int i = 0; i < nb; ++i)
        HIP_OK(hipMemcpyAsync(pump ? b->plans[i]->knots_y : b->plans[i]->knots_x, knots + (size_t)i * nknots,
                              sizeof(double) * nknots, hipMemcpyHostToDevice, b->work));
    std::vector<InstDesc> fwd(nb);
    std::vector<AdjInst> adj(nb);
    w->any_adia = false;
    for (int i = 0; i < nb; ++i) {
        gpe_plan *p = b->plans[i];
        const bool adia = p->pot.cavity == GPE_CAVITY_ADIABATIC;
        float2 *traj = store ? w->traj[i] : nullptr;
        fwd[i] = InstDesc{w->psi[i], p->grid, p->pot, p->st, adia ? w->probe[i] : nullptr, traj};
        adj[i] = AdjInst{w->psi[i], w->lam[i], p->grid, p->pot, p->st, w->partials[i], w->kick_grad[i], pump ? 1 : 0,
                         adia ? w->aprobe[i] : nullptr, traj};
        if (adia) w->any_adia = true;
    }
    HIP_OK(hipMemcpyAsync(w->d_fwd, fwd.data(), sizeof(InstDesc) * nb, hipMemcpyHostToDevice, b->work));
    HIP_OK(hipMemcpyAsync(w->d_adj, adj.data(), sizeof(AdjInst) * nb, hipMemcpyHostToDevice, b->work));

    std::vector<double> terminal(nb, 0.0);  // energy loss: dL/dV0 at T
    auto run = [&](bool checkpoint, double *drift) -> int {
        for (int i = 0; i < nb; ++i) {
            HIP_OK(hipMemcpyAsync(w->psi[i], psi0[i], sizeof(float2) * npts, hipMemcpyDeviceToDevice, b->work));
            HIP_OK(hipMemsetAsync(w->kick_grad[i], 0, sizeof(double) * (size_t)(nsteps + 1), b->work));
        }
        int r;
        if (checkpoint) {
            for (int64_t s = 0; s < nseg; ++s) {
                // every member's psi into slot s: one launch
                LAUNCH_OK(launch_copy_members(w->d_ckpt + (size_t)s * nb, w->d_psi, npts, nb, kCopyBlocks, b->work));
                if ((r = adj_forward(b, w, fsh, fr, t0, s * seg, std::min(nsteps, (s + 1) * seg)))) return r;
            }
        } else if ((r = adj_forward(b, w, fsh, fr, t0, 0, nsteps, store))) {
            return r;
        }
        if (psi_final)
            for (int i = 0; i < nb; ++i)
                if (psi_final[i])
                    HIP_OK(hipMemcpyAsync(psi_final[i], w->psi[i], sizeof(float2) * npts, hipMemcpyDeviceToDevice,
                                          b->work));
        std::vector<const float2 *> pa(nb), pb(nb);
        std::vector<std::array<double, 4>> sums;
        if (energy) {
            // terminal adjoint of L = E(psi(T)): G = 2 dA H psi(T), plus dL/dV0 at T
            const double T = t0 + nsteps * b->dt;
            for (int i = 0; i < nb; ++i)
                if ((r = energy_terminal(b->plans[i], w->psi[i], w->lam[i], T, pump ? 1 : 0, w->partials[i], b->work,
                                         &loss[i], &terminal[i])))
                    return r;
        } else {
            // terminal adjoint: L = 1 - |c|^2, c = <target|psi(T)>, G = -2 c target dA
            for (int i = 0; i < nb; ++i) {
                pa[i] = (const float2 *)target[i];
                pb[i] = w->psi[i];
            }
            if ((r = pair_sums(b, w, pa, pb, sums))) return r;
            std::vector<double2> coef(nb);
            for (int i = 0; i < nb; ++i) {
                const double dA = b->plans[i]->grid.dA;
                const double cr = sums[i][0] * dA, ci = sums[i][1] * dA;
                loss[i] = 1.0 - (cr * cr + ci * ci);
                coef[i] = make_double2(-2.0 * cr * dA, -2.0 * ci * dA);
            }
            HIP_OK(hipMemcpyAsync(w->d_coef, coef.data(), sizeof(double2) * nb, hipMemcpyHostToDevice, b->work));
            std::vector<float2 *> dst(w->lam.begin(), w->lam.end());
            HIP_OK(hipMemcpyAsync(w->d_dst, dst.data(), sizeof(void *) * nb, hipMemcpyHostToDevice, b->work));
            HIP_OK(hipMemcpyAsync(w->d_pa, pa.data(), sizeof(void *) * nb, hipMemcpyHostToDevice, b->work));
            LAUNCH_OK(launch_scaled_copy(w->d_dst, w->d_pa, w->d_coef, npts, nb, 64, b->work));
        }
        *drift = 0;
        if (loss_only) return GPE_OK;
        if (checkpoint) {
            for (int64_t s = nseg - 1; s >= 0; --s) {
                const int64_t e = std::min(nsteps, (s + 1) * seg);
                if (s < nseg - 1)  // restart the state from the stored psi at the segment end
                    LAUNCH_OK(launch_copy_members(w->d_psi, w->d_ckpt + (size_t)(s + 1) * nb, npts, nb, kCopyBlocks,
                                                  b->work));
                if ((r = adj_reverse(b, w, sh, t0, s * seg, e))) return r;
            }
        } else if ((r = adj_reverse(b, w, sh, t0, 0, nsteps, store))) {
            return r;
        }
        *drift = 0;
        if (store) return GPE_OK;  // the state was read back, not rebuilt
        // drift of the state rebuilt at t0 against the input
        for (int i = 0; i < nb; ++i) {
            pa[i] = w->psi[i];
            pb[i] = (const float2 *)psi0[i];
        }
        if ((r = pair_sums(b, w, pa, pb, sums))) return r;
        *drift = 0;
        for (int i = 0; i < nb; ++i) *drift = std::max(*drift, std::sqrt(sums[i][2] / std::max(sums[i][3], 1e-300)));
        return GPE_OK;
    };

    double drift = 0;
    bool ckpt = (mode == GPE_ADJ_CHECKPOINT) && !loss_only;
    if ((rc = run(ckpt, &drift))) return rc;
    if (loss_only) {
        if (info) {
            info[0] = 0;
            info[1] = 0;
            info[2] = (double)w->bytes;
            info[3] = (double)nsteps;
        }
        HIP_OK(hipEventRecord(b->ev_out, b->work));
        HIP_OK(hipStreamWaitEvent(b->user, b->ev_out, 0));
        return GPE_OK;
    }
    int64_t fwd_steps = nsteps;
    if (mode == GPE_ADJ_AUTO && !(drift <= drift_tol)) {
        if ((rc = adj_alloc(b, w, nx, ny, nb, nsteps, (int)nseg))) return rc;
        ckpt = true;
        if ((rc = run(true, &drift))) return rc;
        fwd_steps += nsteps;
    }
    // gradient: dL/dc_m = sum_k w_m(t_k) dL/dV0(t_k)
    std::vector<double> kg((size_t)(nsteps + 1));
    for (int i = 0; i < nb; ++i) {
        HIP_OK(hipMemcpyAsync(kg.data(), w->kick_grad[i], sizeof(double) * kg.size(), hipMemcpyDeviceToHost, b->work));
        HIP_OK(hipStreamSynchronize(b->work));
        gpe_schedule s{};
        const Sched &d = pump ? b->plans[i]->pot.sy : b->plans[i]->pot.sx;
        s.nknots = d.nknots;
        s.t0 = d.t0;
        s.t1 = d.t1;
        double *g = grad + (size_t)i * nknots;
        for (int m = 0; m < nknots; ++m) g[m] = 0;
        for (int64_t k = 0; k <= nsteps; ++k) {
            int i0;
            double w0, w1;
            hat(s, t0 + k * b->dt, &i0, &w0, &w1);
            g[i0] += w0 * (kg[k] + (k == nsteps ? terminal[i] : 0.0));
            g[i0 + 1] += w1 * (kg[k] + (k == nsteps ? terminal[i] : 0.0));
        }
    }
    if (info) {
        info[0] = store ? 3 : ckpt ? 2 : 1;
        info[1] = drift;
        info[2] = (double)w->bytes;
        info[3] = (double)fwd_steps;
    }
    HIP_OK(hipEventRecord(b->ev_out, b->work));
    HIP_OK(hipStreamWaitEvent(b->user, b->ev_out, 0));
    return GPE_OK;
}

}  // extern "C"
