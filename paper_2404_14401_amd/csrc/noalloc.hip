// noalloc.hip -- gpe_step_real_noalloc: real-time split steps without a plan and without
// any allocation, for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Everything gpe_step_real keeps in a plan -- the per-axis potential tables, twiddles,
// kinetic factors, lattice knots, the per-work-group partial sums and the device state
// (cavity field, overlap history, call time, non-finite flag) -- lives here in one
// file-scope device array, `scratch`, of kScratchBytes.  Each call rebuilds the tables
// there with kernels (no host-to-device copies), so a call is a sequence of kernel
// launches on the caller's stream and nothing else.  Each device holds its own copy of
// the array until the process ends; calls on one device share it, so calls that overlap
// on one device (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "runtime_internal.h"

// Largest grid: 8192 x 8192 needs 6 tables of 8192 16-byte entries (768 KiB), two knot
// arrays and three partial buffers of 8192 work-groups x NPART doubles (960 KiB).
static constexpr size_t kScratchBytes = size_t(2) << 20;

// Host code never uses this name as an address: it stands for the array only in
// hipGetSymbolAddress; kernels get the per-device address that call returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxKnots = 256;     // per lattice schedule
constexpr int kKnotChunk = 128;    // knots carried by one launch's arguments
constexpr int kMaxDevices = 64;

std::mutex g_mu;
unsigned char *g_base[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device.
int scratch_base(unsigned char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GPE_ERR_DEVICE, "no HIP device");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(GPE_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_base[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(GPE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_base[dev] = (unsigned char *)ptr;
    }
    *out = g_base[dev];
    return GPE_OK;
}

constexpr size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets of the pieces inside the scratch array.
struct Layout {
    size_t st, tx, ty, twx, twy, kinx, kiny, knx, kny, part, part2, probe, total;
};

Layout layout(int nx, int ny, int npart)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += up256(bytes);
        return at;
    };
    L.st = take(sizeof(DevState));
    L.tx = take(sizeof(float4) * nx);
    L.ty = take(sizeof(float4) * ny);
    L.twx = take(sizeof(double2) * nx);
    L.twy = take(sizeof(double2) * ny);
    L.kinx = take(sizeof(double2) * nx);
    L.kiny = take(sizeof(double2) * ny);
    L.knx = take(sizeof(double) * kMaxKnots);
    L.kny = take(sizeof(double) * kMaxKnots);
    L.part = take(sizeof(double) * NPART * npart);
    L.part2 = take(sizeof(double) * NPART * npart);
    L.probe = take(sizeof(double) * NPART * npart);
    L.total = o;
    return L;
}

struct TableArgs {
    float4 *tx, *ty;
    double2 *twx, *twy, *kinx, *kiny;
    DevState *st;
    DevState init;
    int nx, ny;
    double lx, ly, dt;
    double wx, wy, x0, y0, kx_lat, ky_lat, kc;
};

__device__ float4 axis_entry_dev(double w, double x0, double klat, double kc, double x)
{
    const double c = cos(klat * x);
    return make_float4((float)(0.5 * w * w * (x - x0) * (x - x0)), (float)(c * c), (float)cos(kc * x), (float)x);
}

// The plan's tables for real time, built on the device: potential axis tables (trap,
// lattice cos^2, cavity cos, coordinate), twiddles W_N^m = e^{-2 pi i m / N}, kinetic
// factors e^{-i k^2 dt/2} (the y table carrying the 1/(nx ny) of the round trip), k in
// FFT order; thread 0 also resets the device state.
__global__ void noalloc_tables(TableArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double inv = 1.0 / ((double)a.nx * a.ny);
    if (i < a.nx) {
        const double x = -0.5 * a.lx + i * (a.lx / a.nx);
        a.tx[i] = axis_entry_dev(a.wx, a.x0, a.kx_lat, a.kc, x);
        const double ang = -2.0 * M_PI * i / a.nx;
        a.twx[i] = make_double2(cos(ang), sin(ang));
        const double k = 2.0 * M_PI * (i >= a.nx / 2 ? i - a.nx : i) / a.lx, ph = 0.5 * k * k * a.dt;
        a.kinx[i] = make_double2(cos(ph), -sin(ph));
    }
    if (i < a.ny) {
        const double y = -0.5 * a.ly + i * (a.ly / a.ny);
        a.ty[i] = axis_entry_dev(a.wy, a.y0, a.ky_lat, a.kc, y);
        const double ang = -2.0 * M_PI * i / a.ny;
        a.twy[i] = make_double2(cos(ang), sin(ang));
        const double k = 2.0 * M_PI * (i >= a.ny / 2 ? i - a.ny : i) / a.ly, ph = 0.5 * k * k * a.dt;
        a.kiny[i] = make_double2(cos(ph) * inv, -sin(ph) * inv);
    }
    if (i == 0) *a.st = a.init;
}

struct KnotArgs {
    double *dst;
    int n;
    double v[kKnotChunk];
};

__global__ void noalloc_knots(KnotArgs a)
{
    if ((int)threadIdx.x < a.n) a.dst[threadIdx.x] = a.v[threadIdx.x];
}

__global__ void noalloc_flag(const DevState *st, int *out)
{
    if (threadIdx.x == 0) *out = st->nonfinite;
}

int copy_knots(const gpe_schedule &s, double *dst, hipStream_t stream)
{
    if (s.kind != GPE_SCHED_KNOTS) return GPE_OK;
    for (int off = 0; off < s.nknots; off += kKnotChunk) {
        KnotArgs k{};
        k.dst = dst + off;
        k.n = std::min(kKnotChunk, s.nknots - off);
        for (int i = 0; i < k.n; ++i) k.v[i] = s.knots[off + i];
        hipLaunchKernelGGL(noalloc_knots, dim3(1), dim3(kKnotChunk), 0, stream, k);
        LAUNCH_OK(hipGetLastError());
    }
    return GPE_OK;
}

}  // namespace

extern "C" int gpe_step_real_noalloc(const gpe_plan_desc *d, const gpe_potential_desc *v, gpe_c64 *psi,
                                     int64_t nsteps, double t0, int *nonfinite)
{
    if (!d || !v || !psi || nsteps < 0) return fail(GPE_ERR_INVALID, "null descriptor/psi or negative nsteps");
    if (!std::isfinite(t0)) return fail(GPE_ERR_INVALID, "t0 must be finite");
    int rc = check_plan_desc(d);
    if (rc) return rc;
    if ((rc = check_potential_desc(v))) return rc;
    for (const gpe_schedule *s : {&v->sx, &v->sy})
        if (s->kind == GPE_SCHED_KNOTS && s->nknots > kMaxKnots)
            return fail(GPE_ERR_INVALID, "gpe_step_real_noalloc: more than 256 knots in a schedule");
    const int nx = d->nx, ny = d->ny;
    const Shape sh = plan_shape(nx, ny);
    const int npart = std::max(std::max(sh.row_blocks, sh.col_blocks), 256);
    const Layout L = layout(nx, ny, npart);
    if (L.total > kScratchBytes)
        return fail(GPE_ERR_INVALID, "gpe_step_real_noalloc: the grid's tables exceed the 2 MiB static scratch");
    unsigned char *base = nullptr;
    if ((rc = scratch_base(&base))) return rc;
    if (nsteps == 0) return GPE_OK;

    // a plan on the stack whose every buffer is a piece of the scratch array
    gpe_plan p;
    p.nx = nx;
    p.ny = ny;
    p.lx = d->lx;
    p.ly = d->ly;
    p.dt = d->dt;
    p.g = d->g;
    p.stream = (hipStream_t)d->stream;
    plan_env(&p);
    p.replay = false;  // a captured chunk would be a graph the library allocates
    p.shape = sh;
    p.st = (DevState *)(base + L.st);
    p.tx = (float4 *)(base + L.tx);
    p.ty = (float4 *)(base + L.ty);
    p.tw_x = (double2 *)(base + L.twx);
    p.tw_y = (double2 *)(base + L.twy);
    p.kin_x = (double2 *)(base + L.kinx);
    p.kin_y = (double2 *)(base + L.kiny);
    p.knots_x = (double *)(base + L.knx);
    p.knots_y = (double *)(base + L.kny);
    p.partials = (double *)(base + L.part);
    p.partials2 = (double *)(base + L.part2);
    p.probe = (double *)(base + L.probe);
    p.npart_max = npart;
    griddev_from_desc(p.grid, d);
    p.grid.kin_x = p.kin_x;
    p.grid.kin_y = p.kin_y;
    p.grid.tw_x = p.tw_x;
    p.grid.tw_y = p.tw_y;
    potdev_from_desc(p.pot, v, d->dt, p.tx, p.ty, p.knots_x, p.knots_y);
    p.have_theta = false;

    TableArgs ta{};
    ta.tx = p.tx;
    ta.ty = p.ty;
    ta.twx = p.tw_x;
    ta.twy = p.tw_y;
    ta.kinx = p.kin_x;
    ta.kiny = p.kin_y;
    ta.st = p.st;
    ta.init = initial_state(v);
    ta.nx = nx;
    ta.ny = ny;
    ta.lx = d->lx;
    ta.ly = d->ly;
    ta.dt = d->dt;
    ta.wx = v->wx;
    ta.wy = v->wy;
    ta.x0 = v->x0;
    ta.y0 = v->y0;
    ta.kx_lat = v->kx_lat;
    ta.ky_lat = v->ky_lat;
    ta.kc = v->kc;
    const int nmax = std::max(nx, ny);
    hipLaunchKernelGGL(noalloc_tables, dim3((nmax + 255) / 256), dim3(256), 0, p.stream, ta);
    LAUNCH_OK(hipGetLastError());
    if ((rc = copy_knots(v->sx, p.knots_x, p.stream))) return rc;
    if ((rc = copy_knots(v->sy, p.knots_y, p.stream))) return rc;

    if ((rc = gpe_step_real(&p, psi, nsteps, t0, nullptr))) return rc;
    if (nonfinite) {
        hipLaunchKernelGGL(noalloc_flag, dim3(1), dim3(64), 0, p.stream, p.st, nonfinite);
        LAUNCH_OK(hipGetLastError());
    }
    return GPE_OK;
}
