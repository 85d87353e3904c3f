// Deterministic reductions and small vector helpers.  Every sum is taken in
// double with a fixed assignment of elements to threads and a fixed
// combination tree, so repeated runs give bit-identical results.
#include "common.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int kReduceBlocks = 1024;

int reduce_partials_cap() { return kReduceBlocks; }

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double* __restrict__ partials, int count,
                                                              double* __restrict__ out) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) s += partials[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) *out = t;
}

hipError_t launch_sum_partials(const double* partials, int count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, partials, count, out);
    return hipGetLastError();
}

// one workgroup per image: rn[k] = sum of the image's partials, fixed order
__global__ __launch_bounds__(kBlock) void sum_partials_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                      const double* __restrict__ partials,
                                                                      const int* __restrict__ pcount, int k) {
    __shared__ double red[kBlock / 64];
    const BatchImage& I = imgs[blockIdx.x];
    const double* p = partials + I.pbase;
    const int count = pcount[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) s += p[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) I.rn[k] = t;
}

hipError_t launch_sum_partials_batched(const BatchImage* imgs, const double* partials, const int* pcount, int count,
                                       int k, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(sum_partials_batched_kernel, dim3(count), dim3(kBlock), 0, s, imgs, partials, pcount, k);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void dot_partials_kernel(const float* __restrict__ a,
                                                              const float* __restrict__ b, size_t count,
                                                              double* __restrict__ partials) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        s += (double)a[i] * (double)b[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

hipError_t launch_dot_partials(const float* a, const float* b, size_t count, double* partials, int* n_partials,
                               hipStream_t s) {
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > (size_t)kReduceBlocks) blocks = kReduceBlocks;
    if (blocks == 0) blocks = 1;
    *n_partials = (int)blocks;
    hipLaunchKernelGGL(dot_partials_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, b, count, partials);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void scale_kernel(float* __restrict__ x, size_t count,
                                                       const double* __restrict__ nrm2, float factor) {
    const float f = nrm2 ? (float)((double)factor / sqrt(*nrm2)) : factor;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        x[i] *= f;
}

hipError_t launch_scale(float* x, size_t count, const double* nrm2, float factor, hipStream_t s) {
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, count, nrm2, factor);
    return hipGetLastError();
}

// A counter-based hash (64-bit SplitMix finaliser) mapped to [-1, 1).
__device__ __forceinline__ float hash_unit(unsigned long long i, unsigned seed) {
    unsigned long long z = i + 0x9E3779B97F4A7C15ull * (unsigned long long)(seed + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0);
}

__global__ __launch_bounds__(kBlock) void fill_hash_kernel(float* __restrict__ x, size_t count, unsigned seed) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        x[i] = hash_unit(i, seed);
}

hipError_t launch_fill_hash(float* x, size_t count, unsigned seed, hipStream_t s) {
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_hash_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, count, seed);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void fill_kernel(float* __restrict__ x, size_t count, float value) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        x[i] = value;
}

hipError_t launch_fill(float* x, size_t count, float value, hipStream_t s) {
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, count, value);
    return hipGetLastError();
}

// ---- preconditioned CG of Algorithm 2 (device scalars, no host round trip) ----
// The CG state lives in device doubles st[]: st[0], st[1] the two rho slots,
// st[2] = d^T q, st[3] = rho_0, st[4] = 1 while the CG is running (0 once it
// has stopped: every later update is skipped, so the result is that of the
// stopped CG), and hist[] the step count of each outer iteration.

// rho_0 = st[0]: the CG runs unless the right-hand side is zero
__global__ void pcg_begin_kernel(double* __restrict__ st, int* __restrict__ hist) {
    st[3] = st[0];
    st[4] = st[0] > 0.0 ? 1.0 : 0.0;
    *hist = 0;
}

// after step j with rho_j = *rn: count the step, stop at the first
// sqrt(rho_j / rho_0) <= tol or at the step cap
__global__ void pcg_check_kernel(double* __restrict__ st, const double* __restrict__ rn, int j, int max_steps,
                                 double tol, int* __restrict__ hist) {
    if (st[4] == 0.0) return;
    *hist = j;
    if (sqrt(*rn / st[3]) <= tol || j == max_steps) st[4] = 0.0;
}

// pcg_begin after summing the np partials of rho_0 (fixed order) into st[0]
__global__ __launch_bounds__(kBlock) void pcg_begin_sum_kernel(double* __restrict__ st,
                                                               const double* __restrict__ part, int np,
                                                               int* __restrict__ hist) {
    __shared__ double red[kBlock / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) acc += part[i];
    const double total = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    st[0] = total;
    st[3] = total;
    st[4] = total > 0.0 ? 1.0 : 0.0;
    *hist = 0;
}

// pcg_check after summing the np partials of rho_j (fixed order) into *rn
__global__ __launch_bounds__(kBlock) void pcg_check_sum_kernel(double* __restrict__ st,
                                                               const double* __restrict__ part, int np,
                                                               double* __restrict__ rn, int j, int max_steps,
                                                               double tol, int* __restrict__ hist) {
    __shared__ double red[kBlock / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) acc += part[i];
    const double total = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    *rn = total;
    if (st[4] == 0.0) return;
    *hist = j;
    if (sqrt(total / st[3]) <= tol || j == max_steps) st[4] = 0.0;
}

// t += a d, res -= a q with a = rho / pq (both device doubles); nothing once
// the CG has stopped (*act == 0)
__global__ __launch_bounds__(kBlock) void pcg_update_kernel(float* __restrict__ t, float* __restrict__ res,
                                                            const float* __restrict__ d, const float* __restrict__ q,
                                                            size_t count, const double* __restrict__ rho,
                                                            const double* __restrict__ pq,
                                                            const double* __restrict__ act) {
    if (*act == 0.0) return;
    const float a = (float)(*rho / *pq);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock) {
        t[i] = fmaf(a, d[i], t[i]);
        res[i] = fmaf(-a, q[i], res[i]);
    }
}

// d = z + (rho_new / rho) d; nothing once the CG has stopped
__global__ __launch_bounds__(kBlock) void pcg_dir_kernel(float* __restrict__ d, const float* __restrict__ z,
                                                         size_t count, const double* __restrict__ rho_new,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ act) {
    if (*act == 0.0) return;
    const float b = (float)(*rho_new / *rho);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        d[i] = fmaf(b, d[i], z[i]);
}

// y += a x
__global__ __launch_bounds__(kBlock) void axpy_kernel(float* __restrict__ y, const float* __restrict__ x, size_t count,
                                                      float a) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        y[i] = fmaf(a, x[i], y[i]);
}

// One Lanczos three-term update: w -= alpha_k v + beta_k vprev, with alpha_k =
// ab[0] and beta_k^2 = *beta2 (device doubles; vprev and beta2 null at the
// first step), and the partial sums of the new w^2 per workgroup.
__global__ __launch_bounds__(kBlock) void lanczos_step_kernel(float* __restrict__ w, const float* __restrict__ v,
                                                              const float* __restrict__ vprev, size_t count,
                                                              const double* __restrict__ ab,
                                                              const double* __restrict__ beta2,
                                                              double* __restrict__ partials) {
    __shared__ double red[kBlock / 64];
    const float a = (float)ab[0];
    const float b = vprev ? (float)sqrt(*beta2) : 0.0f;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock) {
        float x = fmaf(-a, v[i], w[i]);
        if (vprev) x = fmaf(-b, vprev[i], x);
        w[i] = x;
        s += (double)x * (double)x;
    }
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

hipError_t launch_lanczos_step(float* w, const float* v, const float* vprev, size_t count, const double* ab,
                               const double* beta2, double* partials, int* n_partials, hipStream_t s) {
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > (size_t)kReduceBlocks) blocks = kReduceBlocks;
    if (blocks == 0) blocks = 1;
    *n_partials = (int)blocks;
    hipLaunchKernelGGL(lanczos_step_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, w, v, vprev, count, ab,
                       beta2, partials);
    return hipGetLastError();
}

static unsigned elementwise_blocks(size_t count) {
    size_t b = (count + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    return (unsigned)(b ? b : 1);
}

hipError_t launch_pcg_update(float* t, float* res, const float* d, const float* q, size_t count, const double* rho,
                             const double* pq, const double* act, hipStream_t s) {
    hipLaunchKernelGGL(pcg_update_kernel, dim3(elementwise_blocks(count)), dim3(kBlock), 0, s, t, res, d, q, count,
                       rho, pq, act);
    return hipGetLastError();
}

hipError_t launch_pcg_dir(float* d, const float* z, size_t count, const double* rho_new, const double* rho,
                          const double* act, hipStream_t s) {
    hipLaunchKernelGGL(pcg_dir_kernel, dim3(elementwise_blocks(count)), dim3(kBlock), 0, s, d, z, count, rho_new,
                       rho, act);
    return hipGetLastError();
}

hipError_t launch_pcg_begin(double* st, int* hist, hipStream_t s) {
    hipLaunchKernelGGL(pcg_begin_kernel, dim3(1), dim3(1), 0, s, st, hist);
    return hipGetLastError();
}

hipError_t launch_pcg_check(double* st, const double* rn, int j, int max_steps, double tol, int* hist,
                            hipStream_t s) {
    hipLaunchKernelGGL(pcg_check_kernel, dim3(1), dim3(1), 0, s, st, rn, j, max_steps, tol, hist);
    return hipGetLastError();
}

hipError_t launch_pcg_begin_sum(double* st, const double* part, int np, int* hist, hipStream_t s) {
    hipLaunchKernelGGL(pcg_begin_sum_kernel, dim3(1), dim3(kBlock), 0, s, st, part, np, hist);
    return hipGetLastError();
}

hipError_t launch_pcg_check_sum(double* st, const double* part, int np, double* rn, int j, int max_steps,
                                double tol, int* hist, hipStream_t s) {
    hipLaunchKernelGGL(pcg_check_sum_kernel, dim3(1), dim3(kBlock), 0, s, st, part, np, rn, j, max_steps, tol, hist);
    return hipGetLastError();
}

hipError_t launch_axpy(float* y, const float* x, size_t count, float a, hipStream_t s) {
    hipLaunchKernelGGL(axpy_kernel, dim3(elementwise_blocks(count)), dim3(kBlock), 0, s, y, x, count, a);
    return hipGetLastError();
}

}  // namespace mlba
