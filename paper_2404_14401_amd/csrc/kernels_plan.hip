// kernels_plan.hip -- launchers of a plan's passes (row, column, LDS-resident grid)
// and the small bookkeeping kernels; host-side shape helpers.
#include "kernels.h"

namespace gpe {

int kernel_radix() { return kRadix; }
int row_radix(int n) { return n >= 8192 ? kRowRadix<8192> : kRadix; }
size_t xchg_bytes() { return sizeof(XchgT); }
// extra LDS bytes per work-group for the staged tables (twiddles + one axis table)

// LDS of the adjoint passes: exchange areas for `arrays` lines (state and adjoint, or the
// adjoint alone) plus the tables
size_t adj_row_shmem(int n, int lines, int r, int arrays)
{
    const size_t words = (size_t)n + (n >> ilog2(r));
    return align16(arrays * lines * words * sizeof(XchgT)) + (size_t)n * (sizeof(double2) + sizeof(float4));
}
size_t adj_col_shmem(int n, int w, int r, int arrays)
{
    const size_t words = (size_t)n * w + (n >> ilog2(r)) + w;
    return align16(arrays * words * sizeof(XchgT)) + (size_t)n * 2 * sizeof(double2);
}

// --------------------------------------------------------------- small kernels
__global__ void __launch_bounds__(256) tail_kernel(TailArgs ta, GridDev gd, PotDev pot, DevState *st)
{
    __shared__ double red[4 * NPART];
    run_tail(ta, gd, pot, st, red);
}

// psi <- psi * st->scale (final renormalisation in imaginary time)
__global__ void __launch_bounds__(256) scale_kernel(float2 *psi, size_t n, const DevState *st)
{
    const double sc = st->scale;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float2 p = psi[i];
        psi[i] = make_float2((float)(p.x * sc), (float)(p.y * sc));
    }
}

// Start of a call: record its first time; imaginary time starts unscaled.
__global__ void set_call_kernel(DevState *st, double t0, int reset_scale, int clear_history)
{
    if (threadIdx.x == 0) {
        st->t0 = t0;
        if (reset_scale) st->scale = 1.0;
        if (clear_history) st->have_theta = 0;
    }
}

// sum |psi|^2 per work-group (norm)
__global__ void __launch_bounds__(256) norm_kernel(const float2 *psi, size_t n, double *partials)
{
    __shared__ double red[4 * 1];
    double s[1] = {0.0};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float2 p = psi[i];
        s[0] += (double)p.x * p.x + (double)p.y * p.y;
    }
    block_sum<1>(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// Marginals of |psi|^2: axis 1 sums every row (out[j], one work-group per row), axis 0
// every column (out[i]; a work-group owns 64 columns, its four waves take every fourth
// row and are combined in a fixed order).  Fixed summation order throughout.
__global__ void __launch_bounds__(256) marginal_kernel(const float2 *psi, int nx, int ny, int axis, double *out)
{
    __shared__ double red[4 * 64];
    if (axis == 1) {
        const float2 *row = psi + (size_t)blockIdx.x * nx;
        double s[1] = {0.0};
        for (int i = threadIdx.x; i < nx; i += blockDim.x) s[0] += (double)row[i].x * row[i].x + (double)row[i].y * row[i].y;
        block_sum<1>(s, red);
        if (threadIdx.x == 0) out[blockIdx.x] = s[0];
        return;
    }
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (col < nx)
        for (int j = q; j < ny; j += 4) {
            const float2 p = psi[(size_t)j * nx + col];
            s += (double)p.x * p.x + (double)p.y * p.y;
        }
    red[q * 64 + lane] = s;
    __syncthreads();
    if (q == 0 && col < nx) out[col] = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
}

// Terminal adjoint of the energy loss (one work-group per row): with lam = T psi on
// entry, lam <- 2 dA (T psi + (V(t) + g|psi|^2) psi), the gradient of E_kin + E_pot +
// E_int; partials[row] = dA sum_x w(x) |psi|^2, the loss's derivative by the depth of
// the controlled lattice (w = cos^2 along x, or along y for axis 1).
__global__ void __launch_bounds__(256) energy_grad_kernel(const float2 *psi, float2 *lam, GridDev gd, PotDev pot,
                                                          const DevState *st, int axis, double *partials)
{
    __shared__ double red[4];
    const int row = blockIdx.x, nx = gd.nx;
    const VLine vl = vline_cav(pot, row, st->t0, st->alpha_re, st->alpha_im);
    const float4 ty = pot.ty[row];
    const float *vu = pot.vuser ? pot.vuser + (size_t)row * nx : nullptr;
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const size_t q = (size_t)row * nx + i;
        const float4 tx = pot.tx[i];
        const float2 p = psi[q], l = lam[q];
        const double d = (double)p.x * p.x + (double)p.y * p.y;
        double V = vpoint(vl, tx);
        if (vu) V += (double)vu[i];
        const double f = V + gd.g * d;
        lam[q] = make_float2((float)(2.0 * gd.dA * ((double)l.x + f * p.x)), (float)(2.0 * gd.dA * ((double)l.y + f * p.y)));
        s[0] += (axis ? (double)ty.y : (double)tx.y) * d;
    }
    block_sum<1>(s, red);
    if (threadIdx.x == 0) partials[row] = s[0] * gd.dA;
}


// ------------------------------------------------------------------- launchers
// With e0/e1, the launch records the kernel's own start and end in those events
// (hipExtLaunchKernel), which times the kernel without extra queue markers.
template <int N> static hipError_t row_dispatch(int mode, bool imag, const RowArgs &a, int blocks, int threads,
                                                size_t shmem, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
#define GPE_ROW(M, I)                                                                              \
    do {                                                                                           \
        static bool attr_ = false;                                                                 \
        if (!attr_) {                                                                              \
            hipError_t e_ = hipFuncSetAttribute((const void *)row_pass<N, M, I>,                   \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024); \
            if (e_ != hipSuccess) return e_;                                                       \
            attr_ = true;                                                                          \
        }                                                                                          \
        if (e0)                                                                                    \
            hipExtLaunchKernelGGL((row_pass<N, M, I>), dim3(blocks), dim3(threads), (uint32_t)shmem, s, e0, e1, 0, a); \
        else                                                                                       \
            hipLaunchKernelGGL((row_pass<N, M, I>), dim3(blocks), dim3(threads), shmem, s, a);     \
    } while (0)
    if (imag) {
        if (mode == ROW_ENTRY) GPE_ROW(ROW_ENTRY, true);
        else if (mode == ROW_EXIT) GPE_ROW(ROW_EXIT, true);
        else if (mode == ROW_MID) GPE_ROW(ROW_MID, true);
        else return hipErrorInvalidValue;
    } else {
        if (mode == ROW_ENTRY) GPE_ROW(ROW_ENTRY, false);
        else if (mode == ROW_MID) GPE_ROW(ROW_MID, false);
        else if (mode == ROW_EXIT) GPE_ROW(ROW_EXIT, false);
        else if (mode == ROW_FWD) GPE_ROW(ROW_FWD, false);
        else if (mode == ROW_PROBE_REAL) GPE_ROW(ROW_PROBE_REAL, false);
        else if (mode == ROW_PROBE_MID) GPE_ROW(ROW_PROBE_MID, false);
        else if (mode == ROW_INV) GPE_ROW(ROW_INV, false);
        else return hipErrorInvalidValue;
    }
#undef GPE_ROW
    return hipGetLastError();
}

hipError_t launch_row(int n, int mode, bool imag, const RowArgs &a, int blocks, int threads, size_t shmem,
                      hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (n) {
    case 16: return row_dispatch<16>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 32: return row_dispatch<32>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 64: return row_dispatch<64>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 128: return row_dispatch<128>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 256: return row_dispatch<256>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 512: return row_dispatch<512>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 1024: return row_dispatch<1024>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 2048: return row_dispatch<2048>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 4096: return row_dispatch<4096>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    case 8192: return row_dispatch<8192>(mode, imag, a, blocks, threads, shmem, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <int N> static hipError_t col_dispatch(int mode, const ColArgs &a, int blocks, int threads, size_t shmem,
                                                hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
#define GPE_COL(M)                                                                                 \
    do {                                                                                           \
        static bool attr_ = false;                                                                 \
        if (!attr_) {                                                                              \
            hipError_t e_ = hipFuncSetAttribute((const void *)col_pass<N, M>,                      \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024); \
            if (e_ != hipSuccess) return e_;                                                       \
            attr_ = true;                                                                          \
        }                                                                                          \
        if (e0)                                                                                    \
            hipExtLaunchKernelGGL((col_pass<N, M>), dim3(blocks), dim3(threads), (uint32_t)shmem, s, e0, e1, 0, a); \
        else                                                                                       \
            hipLaunchKernelGGL((col_pass<N, M>), dim3(blocks), dim3(threads), shmem, s, a);        \
    } while (0)
    if (mode == COL_KIN_REAL) GPE_COL(COL_KIN_REAL);
    else if (mode == COL_KIN_IMAG) GPE_COL(COL_KIN_IMAG);
    else if (mode == COL_EKIN) GPE_COL(COL_EKIN);
    else if (mode == COL_KHALF_INV) GPE_COL(COL_KHALF_INV);
    else if (mode == COL_FWD_KHALF) GPE_COL(COL_FWD_KHALF);
    else if (mode == COL_KHALF_INV_IM) GPE_COL(COL_KHALF_INV_IM);
    else if (mode == COL_FWD_KHALF_IM) GPE_COL(COL_FWD_KHALF_IM);
    else if (mode == COL_KIN_APPLY) GPE_COL(COL_KIN_APPLY);
    else return hipErrorInvalidValue;
#undef GPE_COL
    return hipGetLastError();
}

hipError_t launch_col(int n, int mode, const ColArgs &a, int blocks, int threads, size_t shmem, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1)
{
    switch (n) {
    case 16: return col_dispatch<16>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 32: return col_dispatch<32>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 64: return col_dispatch<64>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 128: return col_dispatch<128>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 256: return col_dispatch<256>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 512: return col_dispatch<512>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 1024: return col_dispatch<1024>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 2048: return col_dispatch<2048>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 4096: return col_dispatch<4096>(mode, a, blocks, threads, shmem, s, e0, e1);
    case 8192: return col_dispatch<8192>(mode, a, blocks, threads, shmem, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <int NY> static hipError_t split_dispatch(int phase, int mode, const ColArgs &a, int blocks, int threads,
                                                   size_t shmem, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
#define GPE_SPLIT(P, M)                                                                            \
    do {                                                                                           \
        if (e0 || e1)                                                                              \
            hipExtLaunchKernelGGL((col_split<NY, P, M>), dim3(blocks), dim3(threads), (uint32_t)shmem, s, e0, e1, 0, \
                                  a);                                                              \
        else                                                                                       \
            hipLaunchKernelGGL((col_split<NY, P, M>), dim3(blocks), dim3(threads), shmem, s, a);   \
    } while (0)
#define GPE_SPLIT_MODE(M)                                                                          \
    do {                                                                                           \
        if (phase == 0) GPE_SPLIT(0, M);                                                           \
        else if (phase == 1) GPE_SPLIT(1, M);                                                      \
        else GPE_SPLIT(2, M);                                                                      \
    } while (0)
    if (phase < 0 || phase > 2) return hipErrorInvalidValue;
    if (mode == COL_KIN_REAL) GPE_SPLIT_MODE(COL_KIN_REAL);
    else if (mode == COL_KIN_IMAG) GPE_SPLIT_MODE(COL_KIN_IMAG);
    else return hipErrorInvalidValue;
#undef GPE_SPLIT_MODE
#undef GPE_SPLIT
    return hipGetLastError();
}

int col_split_a() { return kSplitA; }

hipError_t launch_col_split(int ny, int phase, int mode, const ColArgs &a, int blocks, int threads, size_t shmem,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (ny) {
    case 4096: return split_dispatch<4096>(phase, mode, a, blocks, threads, shmem, s, e0, e1);
    case 8192: return split_dispatch<8192>(phase, mode, a, blocks, threads, shmem, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tail(const TailArgs &ta, const GridDev &gd, const PotDev &pot, DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(tail_kernel, dim3(1), dim3(256), 0, s, ta, gd, pot, st);
    return hipGetLastError();
}

hipError_t launch_scale(float2 *psi, size_t n, const DevState *st, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_kernel, dim3(blocks), dim3(256), 0, s, psi, n, st);
    return hipGetLastError();
}

hipError_t launch_set_call(DevState *st, double t0, int reset_scale, int clear_history, hipStream_t s)
{
    hipLaunchKernelGGL(set_call_kernel, dim3(1), dim3(64), 0, s, st, t0, reset_scale, clear_history);
    return hipGetLastError();
}

hipError_t launch_norm(const float2 *psi, size_t n, double *partials, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(norm_kernel, dim3(blocks), dim3(256), 0, s, psi, n, partials);
    return hipGetLastError();
}

hipError_t launch_energy_grad(const float2 *psi, float2 *lam, const GridDev &gd, const PotDev &pot,
                              const DevState *st, int axis, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(energy_grad_kernel, dim3(gd.ny), dim3(256), 0, s, psi, lam, gd, pot, st, axis, partials);
    return hipGetLastError();
}

hipError_t launch_marginal(const float2 *psi, int nx, int ny, int axis, double *out, hipStream_t s)
{
    const int blocks = axis == 1 ? ny : (nx + 63) / 64;
    hipLaunchKernelGGL(marginal_kernel, dim3(blocks), dim3(256), 0, s, psi, nx, ny, axis, out);
    return hipGetLastError();
}

template <int NX, int NY> static hipError_t lds_launch(const LdsArgs &a, int threads, hipStream_t s)
{
    const size_t shmem = (size_t)(NX + 1) * NY * sizeof(float2);
    hipError_t e = hipFuncSetAttribute((const void *)lds_grid<NX, NY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lds_grid<NX, NY>), dim3(1), dim3(threads), shmem, s, a);
    return hipGetLastError();
}

bool lds_supported(int nx, int ny)
{
    return nx >= 16 && ny >= 16 && nx <= 128 && ny <= 128 && (size_t)(nx + 1) * ny * 8 <= 160 * 1024;
}

int lds_threads(int nx, int ny)
{
    const int n = nx * ny / kLdsRadix;
    return n < 1024 ? n : 1024;
}

hipError_t launch_lds_grid(const LdsArgs &a, hipStream_t s)
{
    const int nx = a.grid.nx, ny = a.grid.ny, th = lds_threads(nx, ny);
#define GPE_LDS_Y(X)                                              \
    switch (ny) {                                                 \
    case 16: return lds_launch<X, 16>(a, th, s);                  \
    case 32: return lds_launch<X, 32>(a, th, s);                  \
    case 64: return lds_launch<X, 64>(a, th, s);                  \
    case 128: return lds_launch<X, 128>(a, th, s);                \
    default: return hipErrorInvalidValue;                         \
    }
    switch (nx) {
    case 16: GPE_LDS_Y(16)
    case 32: GPE_LDS_Y(32)
    case 64: GPE_LDS_Y(64)
    case 128: GPE_LDS_Y(128)
    default: return hipErrorInvalidValue;
    }
#undef GPE_LDS_Y
}

}  // namespace gpe
