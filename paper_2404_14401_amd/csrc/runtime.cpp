// runtime.cpp -- host side of the C ABI declared in include/gpe.h: plans, tables,
// launch sequences, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>


#include "runtime_internal.h"

static thread_local std::string g_err;

int gpe_fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

hipEvent_t *timing_pair(gpe_plan *p, int kind)
{
    if (p->ev_used + 2 > p->ev_pool.size()) return nullptr;
    p->ev_pairs.push_back({kind, p->ev_used});
    hipEvent_t *e = &p->ev_pool[p->ev_used];
    p->ev_used += 2;
    return e;
}

int dalloc(gpe_plan *p, void **ptr, size_t bytes)
{
    if (p->max_bytes && p->bytes + bytes > p->max_bytes)
        return fail(GPE_ERR_NOMEM, "plan memory cap exceeded");
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // the failure is reported here, not by the next launch check
        *ptr = nullptr;
        return fail(GPE_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p->allocs.push_back(*ptr);
    p->bytes += bytes;
    return GPE_OK;
}

template <typename T> static int upload(gpe_plan *p, T **dst, const std::vector<T> &src)
{
    int rc = dalloc(p, (void **)dst, src.size() * sizeof(T));
    if (rc) return rc;
    HIP_OK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return GPE_OK;
}

static double kval(int j, int n, double len) { return 2.0 * M_PI * (j >= n / 2 ? j - n : j) / len; }

static int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

// Launch shape: threads per line T = n / R.  Rows: lines per work-group so that a
// work-group has about 128 threads (one 1024-point line at radix 8; measured best at
// 1024^2, where more work-groups spread the pass's latency over more CUs).  Columns: tiles of W adjacent columns, W chosen
// so that there are at least 256 tiles (one per CU) when the grid allows it.
Shape make_shape_r(int nx, int ny, int R, size_t eb, int row_threads, int min_col_tiles, int row_r)
{
    Shape s{};
    if (row_r <= 0) row_r = R;
    int sh = 0, shr = 0;
    while ((1 << sh) < R) ++sh;
    while ((1 << shr) < row_r) ++shr;
    const int tr = std::max(1, nx / row_r);
    s.row_lines = std::max(1, row_threads / tr);
    if (s.row_lines > ny) s.row_lines = ny;
    if (s.row_lines * tr > 512) s.row_lines = std::max(1, 512 / tr);
    s.row_threads = s.row_lines * tr;
    s.row_blocks = ny / s.row_lines;
    s.row_shmem = (size_t)s.row_lines * (nx + (nx >> shr)) * eb;
    s.row_shmem = (s.row_shmem + 15) / 16 * 16;
    const int tc = std::max(1, ny / R);
    int w = std::max(1, std::min(nx, 1024 / tc));
    while (w > 1 && nx / w < min_col_tiles) w /= 2;
    s.col_cols = w;
    s.col_threads = w * tc;
    s.col_blocks = nx / w;
    s.col_shmem = ((size_t)ny * w + (ny >> sh) + w) * eb;
    s.col_shmem = (s.col_shmem + 15) / 16 * 16;
    return s;
}

// The three-pass column step (col_split) for columns of ny points: outer passes of
// split_a-point transforms on tiles of up to 16 columns (one 128-byte line of complex64 per
// row), the middle pass of (ny / split_a)-point transforms on tiles of up to 256 threads.
static void set_split(Shape &s, int nx, int ny)
{
    const int r = kernel_radix(), na = col_split_a(), nb = ny / na;
    int sh = 0;
    while ((1 << sh) < r) ++sh;
    const size_t eb = xchg_bytes();
    s.split_a = na;
    s.split_ta = na / r;
    s.split_wa = std::min(nx, std::max(1, 256 / s.split_ta));
    s.split_ba = (nx / s.split_wa) * nb;
    s.split_sha = ((size_t)na * s.split_wa + (na >> sh) + s.split_wa) * eb;
    s.split_sha = (s.split_sha + 15) / 16 * 16;
    s.split_tb = nb / r;
    s.split_wb = std::min(nx, std::max(1, 256 / s.split_tb));
    s.split_bb = (nx / s.split_wb) * na;
    s.split_shb = ((size_t)nb * s.split_wb + (nb >> sh) + s.split_wb) * eb;
    s.split_shb = (s.split_shb + 15) / 16 * 16;
}

static Shape make_shape(int nx, int ny)
{
    // column tiles: at least 256 per grid, and up to 2048-point columns work-groups of at
    // most 512 threads (2048-point columns: two columns per tile rather than four, 87.9
    // against 89.9 us per 2048^2 imaginary step; at 1024 points 512 threads is the 256-tile
    // shape already; longer columns take the three-pass column step)
    // and at short columns no fewer than one wave per column work-group (256^2: two-column
    // tiles, 15.35 -> 14.70 us per imaginary step with the 64 row threads below)
    const int tc = std::max(1, ny / kernel_radix());
    int min_tiles = ny <= 2048 ? std::max(256, (int)std::min<int64_t>((int64_t)nx * tc / 512, nx)) : 256;
    if (tc < 64) min_tiles = std::min(min_tiles, std::max(1, nx * tc / 64));
    // row work-groups of 64 threads where a line takes fewer (several lines per work-group;
    // 512^2 17.72 against 18.05 us per imaginary step with 128): from 1024 points on one line
    // per work-group either way
    Shape s = make_shape_r(nx, ny, kernel_radix(), xchg_bytes(), env_int("GPE_ROW_THREADS", 64),
                           env_int("GPE_MIN_COL_TILES", min_tiles), row_radix(nx));
    const int w = env_int("GPE_COL_W", 0);
    if (w > 0 && w <= nx && (w & (w - 1)) == 0 && w * s.col_threads / s.col_cols <= 1024) {
        Shape t = make_shape_r(nx, ny, kernel_radix(), xchg_bytes(), env_int("GPE_ROW_THREADS", 64), nx / w,
                               row_radix(nx));
        s = t;
    }
    // columns of at least GPE_COL_SPLIT_MIN points take the three-pass column step (built
    // for 4096 and 8192; measured at 8192^2: 2.47 -> 1.65 ms per real-time step, at 4096^2:
    // 0.319 -> 0.304 ms)
    const int split_min = env_int("GPE_COL_SPLIT_MIN", 4096);
    if ((ny == 4096 || ny == 8192) && ny >= split_min) set_split(s, nx, ny);
    return s;
}

// The column step (FFT_y, kinetic factor, IFFT_y) of real or imaginary time: one pass, or
// on long columns the three of col_split; timing events around the whole step.
static hipError_t col_step(const gpe_plan *p, int mode, const ColArgs &ca, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr)
{
    const Shape &sh = p->shape;
    if (!sh.split_a || (mode != COL_KIN_REAL && mode != COL_KIN_IMAG))
        return launch_col(p->ny, mode, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, s, e0, e1);
    ColArgs c = ca;
    c.cols_per_wg = sh.split_wa;
    hipError_t e = launch_col_split(p->ny, 0, mode, c, sh.split_ba, sh.split_wa * sh.split_ta, sh.split_sha, s, e0);
    if (e != hipSuccess) return e;
    c.src = c.dst;  // the later passes work on the first one's output
    c.do_tail = 0;
    c.cols_per_wg = sh.split_wb;
    e = launch_col_split(p->ny, 1, mode, c, sh.split_bb, sh.split_wb * sh.split_tb, sh.split_shb, s);
    if (e != hipSuccess) return e;
    c.cols_per_wg = sh.split_wa;
    return launch_col_split(p->ny, 2, mode, c, sh.split_ba, sh.split_wa * sh.split_ta, sh.split_sha, s, nullptr, e1);
}

static Sched to_sched(const gpe_schedule &s, const double *dev_knots)
{
    Sched d{};
    d.kind = s.kind;
    d.nknots = s.nknots;
    d.v0 = s.v0;
    d.v1 = s.v1;
    d.t0 = s.t0;
    d.t1 = s.t1;
    d.knots = dev_knots;
    return d;
}

static void drop_plan_graphs(gpe_plan *p)
{
    for (int k = 0; k < 2; ++k) {
        if (p->graph[k]) (void)hipGraphExecDestroy(p->graph[k]);
        if (p->graph_def[k]) (void)hipGraphDestroy(p->graph_def[k]);
        p->graph[k] = nullptr;
        p->graph_def[k] = nullptr;
        p->graph_psi[k] = nullptr;
    }
}

// Steps per captured chunk.  A call replays chunks when it records no per-step
// observables, times no passes and is long enough to amortise a capture (a plan
// created with GPE_PLAN_GRAPH=0 in the environment never does).
static constexpr int kChunk = 32;

static bool replay_ok(const gpe_plan *p, int64_t nsteps, const double *obs)
{
    return p->replay && !obs && p->timing_every == 0 && nsteps >= 2 + 2 * kChunk;
}

// Capture kChunk steps issued by `issue` (on the capture stream) as graph k, unless the
// graph for this psi exists.
template <class F> static int capture_chunk(gpe_plan *p, int k, const void *psi, F issue)
{
    if (p->graph[k] && p->graph_psi[k] == psi) return GPE_OK;
    if (p->graph[k]) (void)hipGraphExecDestroy(p->graph[k]);
    if (p->graph_def[k]) (void)hipGraphDestroy(p->graph_def[k]);
    p->graph[k] = nullptr;
    p->graph_def[k] = nullptr;
    p->graph_psi[k] = nullptr;
    if (!p->cap) HIP_OK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    const int rc = issue(p->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : fail(GPE_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(&p->graph[k], g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(g);
        p->graph[k] = nullptr;
        return fail(GPE_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    p->graph_def[k] = g;
    p->graph_psi[k] = psi;
    return GPE_OK;
}

static int check_sched(const gpe_schedule &s, const char *name)
{
    if (s.kind < 0 || s.kind > 3) return fail(GPE_ERR_INVALID, std::string(name) + ": unknown schedule kind");
    if ((s.kind == GPE_SCHED_RAMP || s.kind == GPE_SCHED_PULSE) && !(s.t1 > s.t0))
        return fail(GPE_ERR_INVALID, std::string(name) + ": ramp and pulse need t1 > t0");
    if (s.kind == GPE_SCHED_KNOTS && (s.nknots < 2 || !s.knots || !(s.t1 > s.t0)))
        return fail(GPE_ERR_INVALID, std::string(name) + ": knots need nknots >= 2, a host array and t1 > t0");
    return GPE_OK;
}

static int upload_knots(gpe_plan *p, const gpe_schedule &s, double **dev, int *cap)
{
    if (s.kind != GPE_SCHED_KNOTS) return GPE_OK;
    if (s.nknots > *cap) {
        int rc = dalloc(p, (void **)dev, sizeof(double) * (size_t)s.nknots);
        if (rc) return rc;
        *cap = s.nknots;
    }
    HIP_OK(hipMemcpy(*dev, s.knots, sizeof(double) * (size_t)s.nknots, hipMemcpyHostToDevice));
    return GPE_OK;
}

// Argument checks of a potential description (gpe_set_potential and the allocation-free
// entry point).
int check_potential_desc(const gpe_potential_desc *v)
{
    int rc = check_sched(v->sx, "sx");
    if (rc) return rc;
    if ((rc = check_sched(v->sy, "sy"))) return rc;
    if (v->cavity < 0 || v->cavity > 2) return fail(GPE_ERR_INVALID, "cavity must be 0, 1 (field ODE) or 2 (adiabatic)");
    if (v->cavity) {
        // the interference lattice carries sqrt(Vp U0): pump and cavity lattices share a sign
        auto same_sign = [&](double x) { return x * v->vc >= 0; };
        bool ok = same_sign(v->sy.v0) && (v->sy.kind == GPE_SCHED_CONST || same_sign(v->sy.v1));
        if (v->sy.kind == GPE_SCHED_KNOTS && v->sy.knots)
            for (int i = 0; i < v->sy.nknots; ++i) ok = ok && same_sign(v->sy.knots[i]);
        if (!ok) return fail(GPE_ERR_INVALID, "cavity: the pump depth (y lattice) and vc must not differ in sign");
    }
    if (v->cavity == 2 && !(v->n_atoms >= 0 && std::isfinite(v->n_atoms)))
        return fail(GPE_ERR_INVALID, "cavity: n_atoms must be finite and >= 0");
    if (!std::isfinite(v->probe_omega) || !std::isfinite(v->probe_detuning) || !std::isfinite(v->probe_phase))
        return fail(GPE_ERR_INVALID, "probe parameters must be finite");
    if (v->probe_omega != 0 && v->cavity != 2)
        return fail(GPE_ERR_INVALID, "the cavity probe acts on the adiabatic field only");
    return GPE_OK;
}

// One entry of a per-axis potential table at coordinate x: {1/2 w^2 (x - x0)^2,
// cos^2(k_lat x), cos(kc x), x} (trap, lattice of Sec. 5.2 Eq. 9, cavity mode of Sec. 5.3).
static float4 axis_entry(double w, double x0, double klat, double kc, double x)
{
    const double c = std::cos(klat * x);
    return make_float4((float)(0.5 * w * w * (x - x0) * (x - x0)), (float)(c * c), (float)std::cos(kc * x), (float)x);
}

// Device view of a potential whose tables and knots sit at the given device addresses,
// with the cavity field's one-step propagator e^{lambda dt}, (e^{lambda dt} - 1)/lambda.
void potdev_from_desc(PotDev &d, const gpe_potential_desc *v, double dt, const float4 *tx, const float4 *ty,
                      const double *knots_x, const double *knots_y)
{
    d.tx = tx;
    d.ty = ty;
    d.vuser = v->v_user;
    d.sx = to_sched(v->sx, knots_x);
    d.sy = to_sched(v->sy, knots_y);
    d.cavity = v->cavity;
    d.vc = v->vc;
    d.eta = v->eta;
    d.delta_c = v->delta_c;
    d.kappa = v->kappa;
    d.n_atoms = v->n_atoms;
    d.probe_omega = v->probe_omega;
    d.probe_detuning = v->probe_detuning;
    d.probe_phase = v->probe_phase;
    const std::complex<double> lam(-v->kappa, v->delta_c);
    const std::complex<double> e = std::exp(lam * dt);
    const std::complex<double> phi1 = std::abs(lam) > 0 ? (e - 1.0) / lam : std::complex<double>(dt, 0.0);
    d.ecav_re = e.real();
    d.ecav_im = e.imag();
    d.phi1_re = phi1.real();
    d.phi1_im = phi1.imag();
}

// Device state after a potential is set: field alpha0, no overlap history, no pending scale.
DevState initial_state(const gpe_potential_desc *v)
{
    DevState st{};
    st.alpha_re = v->alpha0_re;
    st.alpha_im = v->alpha0_im;
    st.scale = 1.0;
    return st;
}

int check_plan_desc(const gpe_plan_desc *d)
{
    if (!pow2_in(d->nx, 16, 8192) || !pow2_in(d->ny, 16, 8192))
        return fail(GPE_ERR_INVALID, "nx, ny must be powers of two in [16, 8192]");
    if (!(d->lx > 0) || !(d->ly > 0) || !(d->dt > 0) || !(d->g >= 0) || !std::isfinite(d->dt) ||
        !std::isfinite(d->g) || !std::isfinite(d->lx) || !std::isfinite(d->ly))
        return fail(GPE_ERR_INVALID, "need lx, ly, dt > 0 and g >= 0, all finite");
    return GPE_OK;
}

// Scalars of the grid (the table pointers are filled by the caller).
void griddev_from_desc(GridDev &gd, const gpe_plan_desc *d)
{
    gd = GridDev{};
    gd.nx = d->nx;
    gd.ny = d->ny;
    gd.lx = d->lx;
    gd.ly = d->ly;
    gd.dx = d->lx / d->nx;
    gd.dy = d->ly / d->ny;
    gd.dA = gd.dx * gd.dy;
    gd.dt = d->dt;
    gd.g = d->g;
}

Shape plan_shape(int nx, int ny) { return make_shape(nx, ny); }

// Path, tile order and graph replay as the environment selects them (GPE_PATH, GPE_XCD,
// GPE_PLAN_GRAPH).
void plan_env(gpe_plan *p)
{
    const char *force = getenv("GPE_PATH");
    if (force && !strcmp(force, "multipass")) p->path = 1;
    if (force && !strcmp(force, "lds")) p->path = 2;
    const char *xcd = getenv("GPE_XCD");
    if (xcd && !strcmp(xcd, "0")) p->xcd = 0;
    const char *rep = getenv("GPE_PLAN_GRAPH");
    if (rep && !strcmp(rep, "0")) p->replay = false;
}

extern "C" {

const char *gpe_last_error(void) { return g_err.c_str(); }

int gpe_set_potential(gpe_plan *p, const gpe_potential_desc *v)
{
    if (!p || !v) return fail(GPE_ERR_INVALID, "null plan or potential");
    int rc = check_potential_desc(v);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(p->stream));
    drop_plan_graphs(p);  // the potential is baked into captured kernel arguments
    const int nx = p->nx, ny = p->ny;
    std::vector<float4> tx(nx), ty(ny);
    for (int i = 0; i < nx; ++i) tx[i] = axis_entry(v->wx, v->x0, v->kx_lat, v->kc, -0.5 * p->lx + i * (p->lx / nx));
    for (int j = 0; j < ny; ++j) ty[j] = axis_entry(v->wy, v->y0, v->ky_lat, v->kc, -0.5 * p->ly + j * (p->ly / ny));
    HIP_OK(hipMemcpy(p->tx, tx.data(), sizeof(float4) * nx, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->ty, ty.data(), sizeof(float4) * ny, hipMemcpyHostToDevice));
    if ((rc = upload_knots(p, v->sx, &p->knots_x, &p->knots_cap_x))) return rc;
    if ((rc = upload_knots(p, v->sy, &p->knots_y, &p->knots_cap_y))) return rc;
    potdev_from_desc(p->pot, v, p->dt, p->tx, p->ty, p->knots_x, p->knots_y);
    const DevState st = initial_state(v);
    HIP_OK(hipMemcpy(p->st, &st, sizeof(st), hipMemcpyHostToDevice));
    p->have_theta = false;
    return GPE_OK;
}

int gpe_plan_create(gpe_plan **out, const gpe_plan_desc *d)
{
    if (!out || !d) return fail(GPE_ERR_INVALID, "null argument");
    *out = nullptr;
    int rc0 = check_plan_desc(d);
    if (rc0) return rc0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GPE_ERR_DEVICE, "no HIP device");
    gpe_plan *p = new gpe_plan();
    p->nx = d->nx;
    p->ny = d->ny;
    p->lx = d->lx;
    p->ly = d->ly;
    p->dt = d->dt;
    p->g = d->g;
    p->stream = (hipStream_t)d->stream;
    p->max_bytes = d->max_bytes;
    plan_env(p);
    const int nx = d->nx, ny = d->ny;
    p->shape = make_shape(nx, ny);
    int rc = 0;
    auto cleanup = [&](int code) {
        gpe_plan_destroy(p);
        return code;
    };
    if ((rc = dalloc(p, (void **)&p->st, sizeof(DevState)))) return cleanup(rc);
    if ((rc = dalloc(p, (void **)&p->tx, sizeof(float4) * nx))) return cleanup(rc);
    if ((rc = dalloc(p, (void **)&p->ty, sizeof(float4) * ny))) return cleanup(rc);
    std::vector<double2> kx(nx), ky(ny), twx(nx), twy(ny), khx(nx), khyi(ny), khyo(ny);
    std::vector<double> kmx(nx), kmy(ny), khix(nx), khiyi(ny), khiyo(ny);
    const double inv = 1.0 / ((double)nx * ny);
    for (int i = 0; i < nx; ++i) {
        const double k = kval(i, nx, d->lx), ph = 0.5 * k * k * d->dt;
        kx[i] = make_double2(std::cos(ph), -std::sin(ph));
        khx[i] = make_double2(std::cos(0.5 * ph), -std::sin(0.5 * ph));
        kmx[i] = std::exp(-ph);
        khix[i] = std::exp(-0.5 * ph);
        const double a = -2.0 * M_PI * i / nx;
        twx[i] = make_double2(std::cos(a), std::sin(a));
    }
    for (int j = 0; j < ny; ++j) {
        const double k = kval(j, ny, d->ly), ph = 0.5 * k * k * d->dt;
        ky[j] = make_double2(std::cos(ph) * inv, -std::sin(ph) * inv);
        khyi[j] = make_double2(std::cos(0.5 * ph) * inv, -std::sin(0.5 * ph) * inv);
        khyo[j] = make_double2(std::cos(0.5 * ph), -std::sin(0.5 * ph));
        kmy[j] = std::exp(-ph) * inv;
        khiyi[j] = std::exp(-0.5 * ph) * inv;
        khiyo[j] = std::exp(-0.5 * ph);
        const double a = -2.0 * M_PI * j / ny;
        twy[j] = make_double2(std::cos(a), std::sin(a));
    }
    if ((rc = upload(p, &p->kin_x, kx)) || (rc = upload(p, &p->kin_y, ky)) || (rc = upload(p, &p->kim_x, kmx)) ||
        (rc = upload(p, &p->kim_y, kmy)) || (rc = upload(p, &p->tw_x, twx)) || (rc = upload(p, &p->tw_y, twy)) ||
        (rc = upload(p, &p->kh_x, khx)) || (rc = upload(p, &p->kh_yin, khyi)) || (rc = upload(p, &p->kh_yout, khyo)) ||
        (rc = upload(p, &p->khi_x, khix)) || (rc = upload(p, &p->khi_yin, khiyi)) || (rc = upload(p, &p->khi_yout, khiyo)))
        return cleanup(rc);
    p->npart_max = std::max(std::max(p->shape.row_blocks, p->shape.col_blocks), 256);
    if ((rc = dalloc(p, (void **)&p->partials, sizeof(double) * NPART * p->npart_max))) return cleanup(rc);
    if ((rc = dalloc(p, (void **)&p->partials2, sizeof(double) * NPART * p->npart_max))) return cleanup(rc);
    if ((rc = dalloc(p, (void **)&p->probe, sizeof(double) * NPART * p->npart_max))) return cleanup(rc);
    if ((rc = dalloc(p, (void **)&p->scratch, sizeof(float2) * (size_t)nx * ny))) return cleanup(rc);
    if (hipHostMalloc((void **)&p->hpart, sizeof(double) * NPART * p->npart_max) != hipSuccess) {
        (void)hipGetLastError();
        p->hpart = nullptr;
        return cleanup(fail(GPE_ERR_NOMEM, "hipHostMalloc"));
    }
    GridDev &gd = p->grid;
    griddev_from_desc(gd, d);
    gd.kin_x = p->kin_x;
    gd.kin_y = p->kin_y;
    gd.kim_x = p->kim_x;
    gd.kim_y = p->kim_y;
    gd.tw_x = p->tw_x;
    gd.tw_y = p->tw_y;
    gd.kh_x = p->kh_x;
    gd.kh_yin = p->kh_yin;
    gd.kh_yout = p->kh_yout;
    gd.khi_x = p->khi_x;
    gd.khi_yin = p->khi_yin;
    gd.khi_yout = p->khi_yout;
    gpe_potential_desc pot{};
    pot.wx = pot.wy = 1.0;
    if ((rc = gpe_set_potential(p, &pot))) return cleanup(rc);
    *out = p;
    return GPE_OK;
}

int gpe_plan_destroy(gpe_plan *p)
{
    if (!p) return GPE_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    drop_plan_graphs(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (void *a : p->allocs) (void)hipFree(a);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    if (p->hpart) (void)hipHostFree(p->hpart);
    delete p;
    return GPE_OK;
}

// Whole grid in one work-group's LDS for a single plan: one work-group owns the grid, so
// it pays only while the grid is too small to spread over the chip.  Measured on the
// MI355X (us per step, LDS vs multi-pass): 32^2 6.4 vs 8.3 (real), 7.8 vs 16.2 (imaginary);
// 64^2 9.7 vs 9.2 (real), 12.5 vs 17.0 (imaginary); 128^2 109 vs 11 (real).
static bool use_lds(const gpe_plan *p, bool imag)
{
    if (p->path == 1 || !lds_supported(p->nx, p->ny)) return false;
    if (p->path == 2) return true;
    const int pts = p->nx * p->ny;
    return pts <= 32 * 32 || (imag && pts <= 64 * 64);
}

static RowArgs row_args(gpe_plan *p, float2 *psi)
{
    RowArgs a{};
    a.src = psi;
    a.dst = psi;
    a.grid = p->grid;
    a.pot = p->pot;
    a.st = p->st;
    a.partials = p->partials;
    a.lines_per_wg = p->shape.row_lines;
    return a;
}

static ColArgs col_args(gpe_plan *p, float2 *psi, int mode_tail_unused = 0)
{
    (void)mode_tail_unused;
    ColArgs c{};
    c.src = psi;
    c.dst = psi;
    c.grid = p->grid;
    c.st = p->st;
    c.partials = p->partials2;
    c.cols_per_wg = p->shape.col_cols;
    c.xcd_swizzle = (p->shape.col_blocks % 8 == 0 && p->shape.col_blocks >= 64) ? p->xcd : 0;
    c.pot = p->pot;
    return c;
}


static int run_lds(gpe_plan *p, gpe_c64 *psi, int64_t nsteps, double t, double *obs, bool imag)
{
    LdsArgs a{};
    a.psi = (float2 *)psi;
    a.grid = p->grid;
    a.pot = p->pot;
    a.st = p->st;
    a.obs = obs;
    a.imag = imag ? 1 : 0;
    LAUNCH_OK(launch_set_call(p->st, t, 1, 0, p->stream));
    // the kernel runs all steps; split very long runs so one launch stays short
    const int64_t chunk = 1 << 20;
    for (int64_t s0 = 0; s0 < nsteps; s0 += chunk) {
        a.nsteps = (int)std::min<int64_t>(chunk, nsteps - s0);
        a.obs = obs ? obs + s0 * NOBS : nullptr;
        if (s0 > 0 && !imag) LAUNCH_OK(launch_set_call(p->st, t + s0 * p->dt, 1, 0, p->stream));
        LAUNCH_OK(launch_lds_grid(a, p->stream));
    }
    if (p->pot.cavity && !imag) p->have_theta = true;
    return GPE_OK;
}

}  // extern "C"

// Real time with the adiabatic field (multi-pass): before every kick a probe pass
// reduces the density about to be kicked (norm, Theta, C), and each work-group of
// the kicking row pass turns those sums into alpha at the kick time:
//   probe(psi_0), entry kick at t_0 | per step: columns, probe (IFFT_x), merged kick.
static int step_real_adiabatic(gpe_plan *p, gpe_c64 *psi, int64_t nsteps, double t0, double *obs)
{
    const Shape &sh = p->shape;
    float2 *f = (float2 *)psi;
    LAUNCH_OK(launch_set_call(p->st, t0, 0, 0, p->stream));
    RowArgs pa = row_args(p, f);
    pa.partials = p->probe;
    pa.reduce = 1;
    LAUNCH_OK(launch_row(p->nx, ROW_PROBE_REAL, false, pa, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
    RowArgs ra = row_args(p, f);
    ra.probe = p->probe;
    ra.nprobe = sh.row_blocks;
    ra.n = 0;
    LAUNCH_OK(launch_row(p->nx, ROW_ENTRY, false, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
    ra.reduce = obs ? 1 : 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        ColArgs ca = col_args(p, f);
        TailArgs &ta = ca.tail;
        ta.partials = p->partials;
        ta.npartials = (n >= 1 && obs) ? sh.row_blocks : 0;
        ta.obs = (n >= 1 && obs) ? obs + (n - 1) * NOBS : nullptr;
        ca.do_tail = ta.npartials > 0 ? 1 : 0;
        LAUNCH_OK(col_step(p, COL_KIN_REAL, ca, p->stream));
        pa.n = (int)n;
        LAUNCH_OK(launch_row(p->nx, ROW_PROBE_MID, false, pa, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
        ra.n = (int)n;
        LAUNCH_OK(launch_row(p->nx, n + 1 < nsteps ? ROW_MID : ROW_EXIT, false, ra, sh.row_blocks, sh.row_threads,
                             sh.row_shmem, p->stream));
    }
    if (obs) {
        TailArgs ta{};
        ta.partials = p->partials;
        ta.npartials = sh.row_blocks;
        ta.obs = obs + (nsteps - 1) * NOBS;
        LAUNCH_OK(launch_tail(ta, p->grid, p->pot, p->st, p->stream));
    }
    return GPE_OK;
}

// Terminal adjoint of the energy loss L = E_kin + E_pot + E_int (the energy functional
// of Sec. 5.1, not divided by the norm): G = 2 dA (T + V + g|psi|^2) psi in the
// real-gradient convention, T psi formed spectrally (FFT_x, FFT_y, |k|^2/2, IFFT_y,
// IFFT_x).
int energy_terminal(gpe_plan *p, const float2 *psi, float2 *lam, double t, int axis, double *rpart, hipStream_t s,
                    double *loss, double *lat)
{
    const Shape &sh = p->shape;
    LAUNCH_OK(launch_set_call(p->st, t, 0, 0, s));
    RowArgs ra = row_args(p, lam);
    ra.src = psi;
    ra.reduce = 1;
    LAUNCH_OK(launch_row(p->nx, ROW_FWD, false, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, s));
    ColArgs ca = col_args(p, lam);
    ca.do_tail = 0;
    LAUNCH_OK(launch_col(p->ny, COL_KIN_APPLY, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, s));
    RowArgs ri = row_args(p, lam);
    ri.partials = nullptr;
    LAUNCH_OK(launch_row(p->nx, ROW_INV, false, ri, sh.row_blocks, sh.row_threads, sh.row_shmem, s));
    LAUNCH_OK(launch_energy_grad(psi, lam, p->grid, p->pot, p->st, axis, rpart, s));
    std::vector<double> rp((size_t)sh.row_blocks * NPART), cp((size_t)sh.col_blocks * NPART), lp((size_t)p->ny);
    HIP_OK(hipMemcpyAsync(rp.data(), p->partials, rp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(cp.data(), p->partials2, cp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(lp.data(), rpart, lp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double ep = 0, ei = 0, ek = 0, l = 0;
    for (int b = 0; b < sh.row_blocks; ++b) {
        ep += rp[b * NPART + 1];
        ei += rp[b * NPART + 2];
    }
    for (int b = 0; b < sh.col_blocks; ++b) ek += cp[b * NPART + 0];
    for (int j = 0; j < p->ny; ++j) l += lp[j];
    const double dA = p->grid.dA;
    *loss = ek * dA / ((double)p->nx * p->ny) + ep * dA + 0.5 * p->g * ei * dA;
    *lat = l;
    return GPE_OK;
}

extern "C" {

int gpe_step_real(gpe_plan *p, gpe_c64 *psi, int64_t nsteps, double t0, double *obs)
{
    if (!p || !psi || nsteps < 0) return fail(GPE_ERR_INVALID, "null plan/psi or negative nsteps");
    if (!std::isfinite(t0)) return fail(GPE_ERR_INVALID, "t0 must be finite");
    if (nsteps == 0) return GPE_OK;
    if (use_lds(p, false)) return run_lds(p, psi, nsteps, t0, obs, false);
    if (p->pot.cavity == 2) return step_real_adiabatic(p, psi, nsteps, t0, obs);
    const Shape &sh = p->shape;
    float2 *f = (float2 *)psi;
    const bool cav = p->pot.cavity != 0;
    const bool first_theta = cav && !p->have_theta;
    const bool red = cav || obs != nullptr;
    LAUNCH_OK(launch_set_call(p->st, t0, 0, 0, p->stream));
    RowArgs ra = row_args(p, f);
    ra.n = 0;
    ra.reduce = first_theta ? 2 : 0;
    LAUNCH_OK(launch_row(p->nx, ROW_ENTRY, false, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
    // step n of the call: column pass, then the row pass whose kick sits at st->t0 +
    // (rel + 1) dt (rel = n unless replayed chunks have moved st->t0 on)
    auto step = [&](int64_t n, int64_t rel, hipStream_t s) -> int {
        ColArgs ca = col_args(p, f);
        TailArgs &ta = ca.tail;
        ta.partials = p->partials;
        ta.npartials = (n == 0) ? (first_theta ? sh.row_blocks : 0) : (red ? sh.row_blocks : 0);
        ta.first_theta = (n == 0 && first_theta) ? 1 : 0;
        ta.obs = (n >= 1 && obs) ? obs + (n - 1) * NOBS : nullptr;
        ta.theta_only = (n == 0 || !obs) ? 1 : 0;  // matches the row pass's reduce mode 2
        ta.imag = 0;
        ta.advance_alpha = cav ? 1 : 0;
        ca.do_tail = (ta.npartials > 0 || ta.advance_alpha) ? 1 : 0;
        // the last step of every window of timing_every steps (never a call's first or
        // last step, whose row passes are the entry and exit kicks)
        const bool timed = p->timing_every > 0 && (n + 1) % p->timing_every == 0 && n + 1 < nsteps;
        hipEvent_t *ec = timed ? timing_pair(p, 0) : nullptr;
        LAUNCH_OK(col_step(p, COL_KIN_REAL, ca, s, ec ? ec[0] : nullptr, ec ? ec[1] : nullptr));
        RowArgs rb = ra;
        rb.n = (int)rel;
        rb.reduce = red ? (obs ? 1 : 2) : 0;
        hipEvent_t *er = timed ? timing_pair(p, 1) : nullptr;
        LAUNCH_OK(launch_row(p->nx, n + 1 < nsteps ? ROW_MID : ROW_EXIT, false, rb, sh.row_blocks, sh.row_threads,
                             sh.row_shmem, s, er ? er[0] : nullptr, er ? er[1] : nullptr));
        return GPE_OK;
    };
    int rc;
    if (!replay_ok(p, nsteps, obs)) {
        for (int64_t n = 0; n < nsteps; ++n)
            if ((rc = step(n, n, p->stream))) return rc;
    } else {
        // step 0 (it may start the overlap history), then the middle steps 1 .. nsteps-2
        // from replayed chunks of kChunk steps counted from st->t0 = t0 + dt, which each
        // chunk moves on by kChunk dt, then the rest and the exit step directly
        if ((rc = step(0, 0, p->stream))) return rc;
        LAUNCH_OK(launch_advance_one(p->st, p->dt, p->stream));
        if ((rc = capture_chunk(p, 0, f, [&](hipStream_t s) -> int {
                 for (int j = 0; j < kChunk; ++j) {
                     int r = step(1, j, s);
                     if (r) return r;
                 }
                 LAUNCH_OK(launch_advance_one(p->st, kChunk * p->dt, s));
                 return GPE_OK;
             })))
            return rc;
        const int64_t mids = nsteps - 2;
        int64_t done = 0;
        for (; mids - done >= kChunk; done += kChunk) HIP_OK(hipGraphLaunch(p->graph[0], p->stream));
        for (int64_t r = 0; r < mids - done; ++r)
            if ((rc = step(1 + done + r, r, p->stream))) return rc;
        if ((rc = step(nsteps - 1, mids - done, p->stream))) return rc;
    }
    if (red) {
        TailArgs ta{};
        ta.partials = p->partials;
        ta.npartials = sh.row_blocks;
        ta.obs = obs ? obs + (nsteps - 1) * NOBS : nullptr;
        ta.theta_only = obs ? 0 : 1;
        LAUNCH_OK(launch_tail(ta, p->grid, p->pot, p->st, p->stream));
    }
    if (cav) p->have_theta = true;
    return GPE_OK;
}

int gpe_step_real_k(gpe_plan *p, gpe_c64 *psik, int64_t nsteps, double t0, double *obs)
{
    if (!p || !psik || nsteps < 0) return fail(GPE_ERR_INVALID, "null plan/psi or negative nsteps");
    if (!std::isfinite(t0)) return fail(GPE_ERR_INVALID, "t0 must be finite");
    if (p->pot.cavity) return fail(GPE_ERR_UNSUPPORTED, "the Fourier-space ordering runs without the cavity");
    if (nsteps == 0) return GPE_OK;
    const Shape &sh = p->shape;
    float2 *f = (float2 *)psik;
    LAUNCH_OK(launch_set_call(p->st, t0, 0, 0, p->stream));
    ColArgs ca = col_args(p, f);
    ca.do_tail = 0;
    LAUNCH_OK(launch_col(p->ny, COL_KHALF_INV, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, p->stream));
    RowArgs ra = row_args(p, f);
    ra.t_shift = -0.5 * p->dt;  // kick at the step midpoint
    ra.reduce = obs ? 1 : 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        ra.n = (int)n;
        LAUNCH_OK(launch_row(p->nx, ROW_MID, false, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
        ColArgs cb = col_args(p, f);
        TailArgs &ta = cb.tail;
        ta.partials = p->partials;
        ta.npartials = obs ? sh.row_blocks : 0;
        ta.obs = obs ? obs + n * NOBS : nullptr;
        cb.do_tail = obs ? 1 : 0;
        LAUNCH_OK(col_step(p, n + 1 < nsteps ? COL_KIN_REAL : COL_FWD_KHALF, cb, p->stream));
    }
    return GPE_OK;
}

int gpe_step_imag_k(gpe_plan *p, gpe_c64 *psik, int64_t nsteps, double t, double *obs)
{
    if (!p || !psik || nsteps < 0) return fail(GPE_ERR_INVALID, "null plan/psi or negative nsteps");
    if (!std::isfinite(t)) return fail(GPE_ERR_INVALID, "t must be finite");
    if (p->pot.cavity) return fail(GPE_ERR_UNSUPPORTED, "the Fourier-space ordering runs without the cavity");
    if (nsteps == 0) return GPE_OK;
    const Shape &sh = p->shape;
    float2 *f = (float2 *)psik;
    LAUNCH_OK(launch_set_call(p->st, t, 1, 0, p->stream));
    RowArgs ra = row_args(p, f);
    for (int64_t n = 0; n < nsteps; ++n) {
        ColArgs ca = col_args(p, f);
        ca.do_tail = 0;
        LAUNCH_OK(launch_col(p->ny, COL_KHALF_INV_IM, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, p->stream));
        ra.n = (int)n;
        LAUNCH_OK(launch_row(p->nx, ROW_MID, true, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
        LAUNCH_OK(launch_col(p->ny, COL_FWD_KHALF_IM, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, p->stream));
        TailArgs ta{};
        ta.partials = p->partials2;
        ta.npartials = sh.col_blocks;
        ta.imag = 1;
        ta.obs = obs ? obs + n * NOBS : nullptr;
        LAUNCH_OK(launch_tail(ta, p->grid, p->pot, p->st, p->stream));
    }
    LAUNCH_OK(launch_scale(f, (size_t)p->nx * p->ny, p->st, p->stream));
    LAUNCH_OK(launch_set_call(p->st, t, 1, 0, p->stream));
    return GPE_OK;
}

int gpe_step_imag(gpe_plan *p, gpe_c64 *psi, int64_t nsteps, double t, double *obs)
{
    if (!p || !psi || nsteps < 0) return fail(GPE_ERR_INVALID, "null plan/psi or negative nsteps");
    if (!std::isfinite(t)) return fail(GPE_ERR_INVALID, "t must be finite");
    if (nsteps == 0) return GPE_OK;
    if (use_lds(p, true)) return run_lds(p, psi, nsteps, t, obs, true);
    const Shape &sh = p->shape;
    float2 *f = (float2 *)psi;
    LAUNCH_OK(launch_set_call(p->st, t, 1, 0, p->stream));
    const bool adia = p->pot.cavity == 2;
    if (adia) {
        // the adiabatic field of psi_0 drives the first step
        RowArgs pa = row_args(p, f);
        pa.partials = p->probe;
        pa.reduce = 1;
        LAUNCH_OK(launch_row(p->nx, ROW_PROBE_REAL, false, pa, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
        TailArgs ta{};
        ta.partials = p->probe;
        ta.npartials = sh.row_blocks;
        ta.alpha_from_partials = 1;
        LAUNCH_OK(launch_tail(ta, p->grid, p->pot, p->st, p->stream));
    }
    RowArgs ra = row_args(p, f);
    // one step: entry kick (with the pending scale), columns, exit kick with the norm
    // partials, tail (renormalisation scale, field); the potential is frozen at t, so
    // every step without observables is the same launch sequence.  Without observables
    // or the adiabatic field, and with at most GPE_FOLD_ROWS (2048) row work-groups, the
    // tail between steps is left out: every work-group of the next entry kick forms the
    // scale from the exit partials itself, and one tail after the last step leaves the
    // scale for the final renormalisation.  (Each entry work-group reads every partial, so
    // the reads grow with the square of the row work-groups: measured, per step, 128^2
    // 17.1 -> 14.7 us, 1024^2 37.1 -> 36.1 us, 2048^2 91.7 -> 90.0 us, but 4096^2 323.5 ->
    // 332.8 us and 8192^2 1992 -> 2085 us.)
    const int fold_rows = env_int("GPE_FOLD_ROWS", 2048);
    const bool fold = !obs && !adia && sh.row_blocks <= fold_rows;
    auto tail = [&](int64_t n, hipStream_t s) -> int {
        TailArgs ta{};
        ta.partials = p->partials;
        ta.npartials = sh.row_blocks;
        ta.imag = 1;
        ta.alpha_from_partials = adia ? 1 : 0;
        ta.obs = obs ? obs + n * NOBS : nullptr;
        LAUNCH_OK(launch_tail(ta, p->grid, p->pot, p->st, s));
        return GPE_OK;
    };
    auto step = [&](int64_t n, hipStream_t s, bool after_step) -> int {
        ra.n = (int)n;
        ra.reduce = 0;
        ra.scale_partials = (fold && after_step) ? p->partials : nullptr;
        ra.nscale = sh.row_blocks;
        LAUNCH_OK(launch_row(p->nx, ROW_ENTRY, true, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, s));
        ra.scale_partials = nullptr;
        ColArgs ca = col_args(p, f);
        ca.do_tail = 0;
        LAUNCH_OK(col_step(p, COL_KIN_IMAG, ca, s));
        ra.reduce = 1;
        LAUNCH_OK(launch_row(p->nx, ROW_EXIT, true, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, s));
        return fold ? GPE_OK : tail(n, s);
    };
    int rc;
    int64_t done = 0;
    if (replay_ok(p, nsteps, obs)) {
        // the first step directly (its launches set up the kernels), then chunks
        if ((rc = step(0, p->stream, false))) return rc;
        done = 1;
        if ((rc = capture_chunk(p, 1, f, [&](hipStream_t s) -> int {
                 for (int j = 0; j < kChunk; ++j) {
                     int r = step(0, s, true);
                     if (r) return r;
                 }
                 return GPE_OK;
             })))
            return rc;
        for (; nsteps - done >= kChunk; done += kChunk) HIP_OK(hipGraphLaunch(p->graph[1], p->stream));
    }
    for (int64_t n = done; n < nsteps; ++n)
        if ((rc = step(n, p->stream, n > 0))) return rc;
    if (fold && (rc = tail(nsteps - 1, p->stream))) return rc;
    LAUNCH_OK(launch_scale(f, (size_t)p->nx * p->ny, p->st, p->stream));
    LAUNCH_OK(launch_set_call(p->st, t, 1, 0, p->stream));
    return GPE_OK;
}

static int read_state(gpe_plan *p, DevState *out)
{
    HIP_OK(hipMemcpyAsync(out, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    return GPE_OK;
}

int gpe_sync(gpe_plan *p)
{
    if (!p) return fail(GPE_ERR_INVALID, "null plan");
    DevState st;
    int rc = read_state(p, &st);
    if (rc) return rc;
    if (st.nonfinite) return fail(GPE_ERR_NONFINITE, "non-finite values in psi");
    return GPE_OK;
}

int gpe_norm(gpe_plan *p, const gpe_c64 *psi, double *out)
{
    if (!p || !psi || !out) return fail(GPE_ERR_INVALID, "null argument");
    const int blocks = 256;
    LAUNCH_OK(launch_norm((const float2 *)psi, (size_t)p->nx * p->ny, p->partials, blocks, p->stream));
    HIP_OK(hipMemcpyAsync(p->hpart, p->partials, sizeof(double) * blocks, hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    double s = 0;
    for (int i = 0; i < blocks; ++i) s += p->hpart[i];
    *out = s * p->grid.dA;
    if (!std::isfinite(s)) return fail(GPE_ERR_NONFINITE, "non-finite values in psi");
    return GPE_OK;
}

int gpe_momentum_orders(gpe_plan *p, const gpe_c64 *psik, int axis, int order_step, int nmax, double *out)
{
    if (!p || !psik || !out) return fail(GPE_ERR_INVALID, "null argument");
    if (axis != 0 && axis != 1) return fail(GPE_ERR_INVALID, "axis must be 0 (x) or 1 (y)");
    const int n = axis == 0 ? p->nx : p->ny;
    if (order_step < 1 || order_step > n) return fail(GPE_ERR_INVALID, "order_step must be in [1, grid points on the axis]");
    if (nmax < 0 || (2LL * nmax + 1) * order_step > n)
        return fail(GPE_ERR_INVALID, "nmax < 0 or the orders' windows exceed the grid");
    double *marg = (double *)p->scratch;  // n doubles fit in the nx*ny*8-byte scratch grid
    LAUNCH_OK(launch_marginal((const float2 *)psik, p->nx, p->ny, axis, marg, p->stream));
    std::vector<double> h((size_t)n);
    HIP_OK(hipMemcpyAsync(h.data(), marg, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    std::vector<double> pop((size_t)(2 * nmax + 1), 0.0);
    double tot = 0.0;
    for (int j = 0; j < n; ++j) {
        const int js = j >= n / 2 ? j - n : j;  // signed bin
        const int a = js + order_step / 2;
        const int ord = a >= 0 ? a / order_step : -((-a + order_step - 1) / order_step);
        tot += h[j];
        if (ord >= -nmax && ord <= nmax) pop[ord + nmax] += h[j];
    }
    if (!std::isfinite(tot)) return fail(GPE_ERR_NONFINITE, "non-finite momentum distribution");
    for (int q = 0; q <= 2 * nmax; ++q) out[q] = tot > 0 ? pop[q] / tot : 0.0;
    out[2 * nmax + 1] = tot * p->grid.dA / ((double)p->nx * p->ny);
    return GPE_OK;
}

int gpe_energy(gpe_plan *p, const gpe_c64 *psi, double t, double out[6])
{
    if (!p || !psi || !out) return fail(GPE_ERR_INVALID, "null argument");
    if (!std::isfinite(t)) return fail(GPE_ERR_INVALID, "t must be finite");
    const Shape &sh = p->shape;
    LAUNCH_OK(launch_set_call(p->st, t, 0, 0, p->stream));
    RowArgs ra = row_args(p, p->scratch);
    ra.src = (const float2 *)psi;
    ra.dst = p->scratch;
    ra.reduce = 1;
    LAUNCH_OK(launch_row(p->nx, ROW_FWD, false, ra, sh.row_blocks, sh.row_threads, sh.row_shmem, p->stream));
    ColArgs ca = col_args(p, p->scratch);
    ca.do_tail = 0;
    LAUNCH_OK(launch_col(p->ny, COL_EKIN, ca, sh.col_blocks, sh.col_threads, sh.col_shmem, p->stream));
    std::vector<double> rp((size_t)sh.row_blocks * NPART), cp((size_t)sh.col_blocks * NPART);
    HIP_OK(hipMemcpyAsync(rp.data(), p->partials, rp.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipMemcpyAsync(cp.data(), p->partials2, cp.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    double nrm = 0, ep = 0, ei = 0, ek = 0;
    for (int b = 0; b < sh.row_blocks; ++b) {
        nrm += rp[b * NPART + 0];
        ep += rp[b * NPART + 1];
        ei += rp[b * NPART + 2];
    }
    for (int b = 0; b < sh.col_blocks; ++b) ek += cp[b * NPART + 0];
    const double dA = p->grid.dA;
    nrm *= dA;
    ep *= dA;
    ei *= 0.5 * p->g * dA;
    ek *= dA / ((double)p->nx * p->ny);
    out[0] = ek / nrm;
    out[1] = ep / nrm;
    out[2] = ei / nrm;
    out[3] = (ek + ep + ei) / nrm;
    out[4] = (ek + ep + 2 * ei) / nrm;
    out[5] = nrm;
    if (!std::isfinite(nrm) || !std::isfinite(ek) || !std::isfinite(ep) || !std::isfinite(ei))
        return fail(GPE_ERR_NONFINITE, "non-finite values in psi");
    return GPE_OK;
}

int gpe_set_timing(gpe_plan *p, int every)
{
    if (!p || every < 0) return fail(GPE_ERR_INVALID, "null plan or negative interval");
    HIP_OK(hipStreamSynchronize(p->stream));
    p->ev_pairs.clear();
    p->ev_used = 0;
    p->timing_every = every;
    if (every > 0 && p->ev_pool.empty()) {
        p->ev_pool.resize(8192);
        for (auto &e : p->ev_pool) HIP_OK(hipEventCreate(&e));
    }
    return GPE_OK;
}

int gpe_get_timing(gpe_plan *p, double out[4])
{
    if (!p || !out) return fail(GPE_ERR_INVALID, "null argument");
    HIP_OK(hipStreamSynchronize(p->stream));
    double sum[2] = {0, 0};
    int cnt[2] = {0, 0};
    for (auto &pr : p->ev_pairs) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, p->ev_pool[pr.second], p->ev_pool[pr.second + 1]));
        sum[pr.first] += ms;
        cnt[pr.first] += 1;
    }
    out[0] = cnt[0] ? sum[0] / cnt[0] : 0.0;
    out[1] = cnt[0];
    out[2] = cnt[1] ? sum[1] / cnt[1] : 0.0;
    out[3] = cnt[1];
    return GPE_OK;
}

int gpe_get_cavity(gpe_plan *p, double out[4])
{
    if (!p || !out) return fail(GPE_ERR_INVALID, "null argument");
    DevState st;
    int rc = read_state(p, &st);
    if (rc) return rc;
    out[0] = st.alpha_re;
    out[1] = st.alpha_im;
    out[2] = st.theta;
    out[3] = st.theta_prev;
    if (st.nonfinite) return fail(GPE_ERR_NONFINITE, "non-finite values in psi");
    return GPE_OK;
}

int gpe_set_cavity(gpe_plan *p, const double s[4], int have_history)
{
    if (!p || !s) return fail(GPE_ERR_INVALID, "null argument");
    DevState st;
    int rc = read_state(p, &st);
    if (rc) return rc;
    st.alpha_re = s[0];
    st.alpha_im = s[1];
    st.theta = s[2];
    st.theta_prev = s[3];
    st.have_theta = have_history ? 1 : 0;
    HIP_OK(hipMemcpyAsync(p->st, &st, sizeof(st), hipMemcpyHostToDevice, p->stream));
    HIP_OK(hipStreamSynchronize(p->stream));
    p->have_theta = have_history != 0;
    return GPE_OK;
}

}  // extern "C"
