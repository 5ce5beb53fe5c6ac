// kernels_batch.hip -- launchers of the batched passes (every member of a size group
// in one launch per pass) and the batch's bookkeeping kernels.
#include "kernels.h"

namespace gpe {

// ------------------------------------------------------------ batched launchers
template <int N, int R> static hipError_t rowb_dispatch(int mode, const BatchPassArgs &a, int blocks, int threads,
                                                        size_t shmem, hipStream_t s)
{
#define GPE_ROWB_T(M, A, TJ)                                                                       \
    do {                                                                                           \
        static bool attr_ = false;                                                                 \
        if (!attr_) {                                                                              \
            hipError_t e_ = hipFuncSetAttribute((const void *)row_pass_b<N, R, M, A, TJ>,          \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024); \
            if (e_ != hipSuccess) return e_;                                                       \
            attr_ = true;                                                                          \
        }                                                                                          \
        hipLaunchKernelGGL((row_pass_b<N, R, M, A, TJ>), dim3(blocks), dim3(threads), shmem, s, a); \
    } while (0)
#define GPE_ROWB(M, A) GPE_ROWB_T(M, A, false)
    if (a.traj) {
        // the adjoint's recording forward sweep (radix 8 only): entry and merged kicks
        if constexpr (R == 8) {
            if (a.cav) {
                if (mode == ROW_ENTRY) GPE_ROWB_T(ROW_ENTRY, true, true);
                else if (mode == ROW_MID) GPE_ROWB_T(ROW_MID, true, true);
                else if (mode == ROW_EXIT) GPE_ROWB(ROW_EXIT, true);
                else if (mode == ROW_PROBE_REAL) GPE_ROWB(ROW_PROBE_REAL, true);
                else if (mode == ROW_PROBE_MID) GPE_ROWB(ROW_PROBE_MID, true);
                else return hipErrorInvalidValue;
            } else {
                if (mode == ROW_ENTRY) GPE_ROWB_T(ROW_ENTRY, false, true);
                else if (mode == ROW_MID) GPE_ROWB_T(ROW_MID, false, true);
                else if (mode == ROW_EXIT) GPE_ROWB(ROW_EXIT, false);
                else return hipErrorInvalidValue;
            }
        } else {
            return hipErrorInvalidValue;
        }
    } else if (a.cav) {
        if (mode == ROW_ENTRY) GPE_ROWB(ROW_ENTRY, true);
        else if (mode == ROW_MID) GPE_ROWB(ROW_MID, true);
        else if (mode == ROW_EXIT) GPE_ROWB(ROW_EXIT, true);
        else if (mode == ROW_PROBE_REAL) GPE_ROWB(ROW_PROBE_REAL, true);
        else if (mode == ROW_PROBE_MID) GPE_ROWB(ROW_PROBE_MID, true);
        else return hipErrorInvalidValue;
    } else {
        if (mode == ROW_ENTRY) GPE_ROWB(ROW_ENTRY, false);
        else if (mode == ROW_MID) GPE_ROWB(ROW_MID, false);
        else if (mode == ROW_EXIT) GPE_ROWB(ROW_EXIT, false);
        else return hipErrorInvalidValue;
    }
#undef GPE_ROWB
#undef GPE_ROWB_T
    return hipGetLastError();
}

template <int N, int R, bool ODE> static hipError_t colb_launch(const BatchPassArgs &a, int blocks, int threads,
                                                                size_t shmem, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)col_pass_b<N, R, ODE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((col_pass_b<N, R, ODE>), dim3(blocks), dim3(threads), shmem, s, a);
    return hipGetLastError();
}

template <int N, int R> static hipError_t colb_dispatch(const BatchPassArgs &a, int blocks, int threads, size_t shmem,
                                                        hipStream_t s)
{
    return a.ode ? colb_launch<N, R, true>(a, blocks, threads, shmem, s)
                 : colb_launch<N, R, false>(a, blocks, threads, shmem, s);
}

#define GPE_SIZES(F, ...)                                                                          \
    switch (n) {                                                                                   \
    case 64: return F<64, RR>(__VA_ARGS__);                                                        \
    case 128: return F<128, RR>(__VA_ARGS__);                                                      \
    case 256: return F<256, RR>(__VA_ARGS__);                                                      \
    case 512: return F<512, RR>(__VA_ARGS__);                                                      \
    case 1024: return F<1024, RR>(__VA_ARGS__);                                                    \
    case 2048: return F<2048, RR>(__VA_ARGS__);                                                    \
    default: return hipErrorInvalidValue;                                                          \
    }

hipError_t launch_row_batched(int n, int r, int mode, const BatchPassArgs &a, int blocks, int threads, size_t shmem,
                              hipStream_t s)
{
    if (r == 8) {
        constexpr int RR = 8;
        GPE_SIZES(rowb_dispatch, mode, a, blocks, threads, shmem, s)
    } else if (r == 4) {
        constexpr int RR = 4;
        GPE_SIZES(rowb_dispatch, mode, a, blocks, threads, shmem, s)
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col_batched(int n, int r, const BatchPassArgs &a, int blocks, int threads, size_t shmem,
                              hipStream_t s)
{
    if (r == 8) {
        constexpr int RR = 8;
        GPE_SIZES(colb_dispatch, a, blocks, threads, shmem, s)
    } else if (r == 4) {
        constexpr int RR = 4;
        GPE_SIZES(colb_dispatch, a, blocks, threads, shmem, s)
    }
    return hipErrorInvalidValue;
}
#undef GPE_SIZES

template <int NX, int NY>
static hipError_t ldsb_launch(const LdsArgs *arr, int count, int threads, int64_t s0, int nsteps, hipStream_t s)
{
    const size_t shmem = (size_t)(NX + 1) * NY * sizeof(float2);
    hipError_t e = hipFuncSetAttribute((const void *)lds_grid_b<NX, NY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lds_grid_b<NX, NY>), dim3(count), dim3(threads), shmem, s, arr, s0, nsteps);
    return hipGetLastError();
}

hipError_t launch_lds_batched(int nx, int ny, const LdsArgs *arr, int count, int64_t s0, int nsteps, hipStream_t s)
{
    const int th = lds_threads(nx, ny);
#define GPE_LDSB_Y(X)                                                                              \
    switch (ny) {                                                                                  \
    case 16: return ldsb_launch<X, 16>(arr, count, th, s0, nsteps, s);                                         \
    case 32: return ldsb_launch<X, 32>(arr, count, th, s0, nsteps, s);                                         \
    case 64: return ldsb_launch<X, 64>(arr, count, th, s0, nsteps, s);                                         \
    case 128: return ldsb_launch<X, 128>(arr, count, th, s0, nsteps, s);                                       \
    default: return hipErrorInvalidValue;                                                          \
    }
    switch (nx) {
    case 16: GPE_LDSB_Y(16)
    case 32: GPE_LDSB_Y(32)
    case 64: GPE_LDSB_Y(64)
    case 128: GPE_LDSB_Y(128)
    default: return hipErrorInvalidValue;
    }
#undef GPE_LDSB_Y
}

// Start of a batched call: every member's state records the call's first time.

__global__ void set_call_batched_kernel(DevState *const *st, int n, double t0)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        st[i]->t0 = t0;
        st[i]->scale = 1.0;
    }
}

// After a replayed chunk of steps: advance every member's first time.
__global__ void advance_t0_kernel(DevState *const *st, int n, double dt_total)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) st[i]->t0 += dt_total;
}

hipError_t launch_set_call_batched(DevState *const *st, int n, double t0, hipStream_t s)
{
    hipLaunchKernelGGL(set_call_batched_kernel, dim3(1), dim3(256), 0, s, st, n, t0);
    return hipGetLastError();
}

// One plan's time base moves on by dt_total (after a replayed chunk of steps).
__global__ void advance_one_kernel(DevState *st, double dt_total)
{
    if (threadIdx.x == 0) st->t0 += dt_total;
}

hipError_t launch_advance_one(DevState *st, double dt_total, hipStream_t s)
{
    hipLaunchKernelGGL(advance_one_kernel, dim3(1), dim3(64), 0, s, st, dt_total);
    return hipGetLastError();
}

// Non-finite flags of every member, gathered for one copy to the host.
__global__ void gather_flags_kernel(DevState *const *st, int n, int *out)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = st[i]->nonfinite;
}

hipError_t launch_gather_flags(DevState *const *st, int n, int *out, hipStream_t s)
{
    hipLaunchKernelGGL(gather_flags_kernel, dim3(1), dim3(256), 0, s, st, n, out);
    return hipGetLastError();
}

hipError_t launch_advance_t0(DevState *const *st, int n, double dt_total, hipStream_t s)
{
    hipLaunchKernelGGL(advance_t0_kernel, dim3(1), dim3(256), 0, s, st, n, dt_total);
    return hipGetLastError();
}

}  // namespace gpe
