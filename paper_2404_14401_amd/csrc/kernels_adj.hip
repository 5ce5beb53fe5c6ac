// kernels_adj.hip -- the discrete adjoint's kernels and launchers.
#include "kernels.h"

namespace gpe {

__global__ void __launch_bounds__(256) tail_batched_kernel(const InstDesc *inst, int nrow)
{
    __shared__ double red[4 * NPART];
    const InstDesc &I = inst[blockIdx.x];
    if (!I.partials) return;
    TailArgs ta{};
    ta.partials = I.partials;
    ta.npartials = nrow;
    ta.theta_only = 1;
    run_tail(ta, I.grid, I.pot, I.st, red);
}

hipError_t launch_tail_batched(const InstDesc *inst, int count, int nrow, hipStream_t s)
{
    hipLaunchKernelGGL(tail_batched_kernel, dim3(count), dim3(256), 0, s, inst, nrow);
    return hipGetLastError();
}

// The last kick's sums: one work-group per member.
__global__ void __launch_bounds__(256) adj_tail_kernel(const AdjInst *inst, int nrow, int k)
{
    __shared__ double red[4];
    adj_tail(inst[blockIdx.x], nrow, k, red);
}

// Per work-group partial sums over one member's points: {Re, Im} of sum conj(a) b, and
// sum |a - b|^2, sum |b|^2.  Work-group b serves member b / per_inst.
__global__ void __launch_bounds__(256) pair_sums_kernel(const float2 *const *a, const float2 *const *b, size_t npts,
                                                        int per_inst, double *out)
{
    __shared__ double red[4 * 4];
    const int inst = blockIdx.x / per_inst, lb = blockIdx.x % per_inst;
    const float2 *pa = a[inst], *pb = b[inst];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)lb * blockDim.x + threadIdx.x; i < npts; i += (size_t)per_inst * blockDim.x) {
        const float2 x = pa[i], y = pb[i];
        s[0] += (double)x.x * y.x + (double)x.y * y.y;
        s[1] += (double)x.x * y.y - (double)x.y * y.x;
        const double dx = (double)x.x - y.x, dy = (double)x.y - y.y;
        s[2] += dx * dx + dy * dy;
        s[3] += (double)y.x * y.x + (double)y.y * y.y;
    }
    block_sum<4>(s, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[blockIdx.x * 4 + k] = s[k];
}

// lam_i = coef_i * src_i (terminal adjoint of the fidelity loss).
__global__ void __launch_bounds__(256) scaled_copy_kernel(float2 *const *dst, const float2 *const *src,
                                                          const double2 *coef, size_t npts, int per_inst)
{
    const int inst = blockIdx.x / per_inst, lb = blockIdx.x % per_inst;
    const double2 c = coef[inst];
    float2 *d = dst[inst];
    const float2 *s = src[inst];
    for (size_t i = (size_t)lb * blockDim.x + threadIdx.x; i < npts; i += (size_t)per_inst * blockDim.x) {
        const float2 x = s[i];
        d[i] = make_float2((float)(c.x * x.x - c.y * x.y), (float)(c.x * x.y + c.y * x.x));
    }
}

// dst_i = src_i for every member, npts points each (checkpoint save and restore).
__global__ void __launch_bounds__(256) copy_members_kernel(float2 *const *dst, const float2 *const *src, size_t npts,
                                                           int per_inst)
{
    const int inst = blockIdx.x / per_inst, lb = blockIdx.x % per_inst;
    float4 *d = reinterpret_cast<float4 *>(dst[inst]);
    const float4 *s = reinterpret_cast<const float4 *>(src[inst]);
    const size_t n4 = npts / 2;
    for (size_t i = (size_t)lb * blockDim.x + threadIdx.x; i < n4; i += (size_t)per_inst * blockDim.x) d[i] = s[i];
    if ((npts & 1) && lb == 0 && threadIdx.x == 0) dst[inst][npts - 1] = src[inst][npts - 1];
}

template <int N, int R, bool TRAJ> static hipError_t rowadj_mode(int mode, const AdjPassArgs &a, int blocks,
                                                                 int threads, size_t shmem, hipStream_t s)
{
#define GPE_RADJ(M)                                                                                \
    do {                                                                                           \
        static bool attr_ = false;                                                                 \
        if (!attr_) {                                                                              \
            hipError_t e_ = hipFuncSetAttribute((const void *)row_adj_b<N, R, M, TRAJ>,            \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024); \
            if (e_ != hipSuccess) return e_;                                                       \
            attr_ = true;                                                                          \
        }                                                                                          \
        hipLaunchKernelGGL((row_adj_b<N, R, M, TRAJ>), dim3(blocks), dim3(threads), shmem, s, a);  \
    } while (0)
    if (mode == ADJ_FIRST) GPE_RADJ(ADJ_FIRST);
    else if (mode == ADJ_MID) GPE_RADJ(ADJ_MID);
    else if (mode == ADJ_LAST) GPE_RADJ(ADJ_LAST);
    else if (mode == ADJ_PROBE_FIRST) GPE_RADJ(ADJ_PROBE_FIRST);
    else if (mode == ADJ_PROBE_MID) GPE_RADJ(ADJ_PROBE_MID);
    else return hipErrorInvalidValue;
#undef GPE_RADJ
    return hipGetLastError();
}

template <int N, int R> static hipError_t rowadj_dispatch(int mode, const AdjPassArgs &a, int blocks, int threads,
                                                          size_t shmem, hipStream_t s)
{
    return a.traj ? rowadj_mode<N, R, true>(mode, a, blocks, threads, shmem, s)
                  : rowadj_mode<N, R, false>(mode, a, blocks, threads, shmem, s);
}

template <int N, int R, bool TRAJ> static hipError_t coladj_launch(const AdjPassArgs &a, int blocks, int threads,
                                                                   size_t shmem, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)col_adj_b<N, R, TRAJ>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((col_adj_b<N, R, TRAJ>), dim3(blocks), dim3(threads), shmem, s, a);
    return hipGetLastError();
}

template <int N, int R> static hipError_t coladj_dispatch(const AdjPassArgs &a, int blocks, int threads, size_t shmem,
                                                          hipStream_t s)
{
    return a.traj ? coladj_launch<N, R, true>(a, blocks, threads, shmem, s)
                  : coladj_launch<N, R, false>(a, blocks, threads, shmem, s);
}

#define GPE_ADJ_SIZES(F, ...)                                                                      \
    switch (n) {                                                                                   \
    case 64: return F<64, 8>(__VA_ARGS__);                                                         \
    case 128: return F<128, 8>(__VA_ARGS__);                                                       \
    case 256: return F<256, 8>(__VA_ARGS__);                                                       \
    case 512: return F<512, 8>(__VA_ARGS__);                                                       \
    case 1024: return F<1024, 8>(__VA_ARGS__);                                                     \
    default: return hipErrorInvalidValue;                                                          \
    }

hipError_t launch_row_adj(int n, int mode, const AdjPassArgs &a, int blocks, int threads, size_t shmem, hipStream_t s)
{
    GPE_ADJ_SIZES(rowadj_dispatch, mode, a, blocks, threads, shmem, s)
}

hipError_t launch_col_adj(int n, const AdjPassArgs &a, int blocks, int threads, size_t shmem, hipStream_t s)
{
    GPE_ADJ_SIZES(coladj_dispatch, a, blocks, threads, shmem, s)
}
#undef GPE_ADJ_SIZES

hipError_t launch_adj_tail(const AdjInst *inst, int count, int nrow, int k, hipStream_t s)
{
    hipLaunchKernelGGL(adj_tail_kernel, dim3(count), dim3(256), 0, s, inst, nrow, k);
    return hipGetLastError();
}

hipError_t launch_pair_sums(const float2 *const *a, const float2 *const *b, size_t npts, int count, int per_inst,
                            double *out, hipStream_t s)
{
    hipLaunchKernelGGL(pair_sums_kernel, dim3(count * per_inst), dim3(256), 0, s, a, b, npts, per_inst, out);
    return hipGetLastError();
}

hipError_t launch_scaled_copy(float2 *const *dst, const float2 *const *src, const double2 *coef, size_t npts,
                              int count, int per_inst, hipStream_t s)
{
    hipLaunchKernelGGL(scaled_copy_kernel, dim3(count * per_inst), dim3(256), 0, s, dst, src, coef, npts, per_inst);
    return hipGetLastError();
}

hipError_t launch_copy_members(float2 *const *dst, const float2 *const *src, size_t npts, int count, int per_inst,
                               hipStream_t s)
{
    hipLaunchKernelGGL(copy_members_kernel, dim3(count * per_inst), dim3(256), 0, s, dst, src, npts, per_inst);
    return hipGetLastError();
}

}  // namespace gpe

