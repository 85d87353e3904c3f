// Antireflective-transform preconditioner (paper sections 2.2 and 4.3):
// Algorithm 3 with antireflective boundary conditions,
//   P r = T (Lambda^2 + alpha)^-1 T^-1 r        (T along both axes)
// where T is the antireflective transform of length n, N = n - 1:
//   columns t_0[k] = 1 - k/N, t_N[k] = k/N (the two linear functions) and
//   t_j[k] = sin(pi j k / N), 0 < j < N (the sine basis),
// and Lambda the eigenvalues of the antireflective blur of the symmetrised
// PSF H~:
//   lambda[ky][kx] = sum_{a,b} H~[a][b] cos(w_ky (a-c)) cos(w_kx (b-c)),
//   w_j = pi j / N for the sines, 0 for the two linear functions.
//
// T^-1 of one sequence v: the linear coefficients are v[0] and v[N]; the
// sine coefficients are (2/N) DST-I of v minus its linear interpolant.  T of
// coefficients c: the linear interpolant of c_0, c_N plus the DST-I of the
// sine coefficients.  Both sine transforms are read off one complex FFT of
// length 2N: the odd extension x[k] = g[k], x[2N-k] = -g[k], x[0] = x[N] = 0
// of two real sequences a, b packed as a + i b has FFT X with
//   Re X[j] = 2 sum_k b[k] sin(pi j k / N),  Im X[j] = -2 sum_k a[k] sin(pi j k / N).
//
// Three passes over the n x n image, as for the DFT and DCT preconditioners:
//   1. rows: two image rows per sequence, T^-1 along x, written transposed
//      (Tr[jx][y]);
//   2. columns (rows of Tr): T^-1 along y, multiply by 1/(lambda^2 + alpha)
//      (times lambda for Algorithm 4), T along y, all in LDS;
//   3. rows: gather transposed, T along x, write the image rows.
// The transform length 2N is any length fft_length_supported accepts
// (2^a 3^b 5^c up to FFT_MAX_ELEMS, other lengths in the Bluestein form).
#include "artrans.hpp"
#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"

namespace mlba {

template <int NT>
__global__ __launch_bounds__(kBlock) void ar_rows_fwd_kernel(const float* __restrict__ src, int n,
                                                             float* __restrict__ Tr, int ts, FftDesc fd,
                                                             const float2* __restrict__ tw, int G, int seq_shift) {
    extern __shared__ float2 buf[];
    ar_rows_fwd_body<NT>(src, n, Tr, ts, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
}

// red_out (optional): workgroup 0 first sums red_count partials of the
// previous launch (the residual's) into *red_out.
template <int NT>
__global__ __launch_bounds__(kBlock) void ar_cols_filter_kernel(float* __restrict__ Tr, int n, int ts,
                                                                const float* __restrict__ spec, float alpha,
                                                                const float* __restrict__ lamr, FftDesc fd,
                                                                const float2* __restrict__ tw, int CP,
                                                                int seq_shift, const double* __restrict__ red_in,
                                                                int red_count, double* __restrict__ red_out) {
    extern __shared__ float2 buf[];
    __shared__ float2 lin[2 * kArMaxBatch];
    if (red_out && blockIdx.x == 0) {
        __shared__ double red[kBlock / 64];
        const double acc = strided_sum(red_in, red_count);
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) *red_out = t;
    }
    ar_cols_filter_body<NT>(Tr, n, ts, spec, alpha, lamr, fd, tw, CP, seq_shift, blockIdx.x, buf, lin);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void ar_rows_inv_kernel(const float* __restrict__ Tr, int n, int ts,
                                                             float* __restrict__ dst, FftDesc fd,
                                                             const float2* __restrict__ tw, int G, int seq_shift,
                                                             int accum) {
    extern __shared__ float2 buf[];
    ar_rows_inv_body<NT>(Tr, n, ts, dst, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf, accum);
}

// ---- launch helpers --------------------------------------------------------

static int ar_shift_for(int batch) {
    int sh = 8;  // log2(kBlock)
    while (batch > 1) {
        batch >>= 1;
        --sh;
    }
    return sh;
}

// sequences per workgroup: a power of two within the LDS budget, keeping at
// least 256 workgroups when the image allows it
static int ar_batch(int n) {
    const int L = 2 * (n - 1), pairs = (n + 1) / 2;
    int G = 1;
    if (!smooth235(L)) return 1;  // Bluestein: one sequence per workgroup
    while (G * 2 <= kArMaxBatch && (G * 2) * L <= FFT_MAX_ELEMS && pairs / (G * 2) >= 256) G *= 2;
    return G;
}

bool ar_transform_supported(int n) { return n >= 4 && fft_length_supported(2 * (n - 1)); }

int ar_workspace_stride(int n) { return ((n + 1 + 15) / 16) * 16 + 16; }

// the compiled fixed-size transform when the length is kFixedN with one
// sequence per workgroup (n = 1025), the run-time plan otherwise
hipError_t launch_ar_rows_fwd(const float* src, int n, float* Tr, int ts, const FftDesc& fd, const float2* tw,
                              hipStream_t s) {
    const int G = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + G - 1) / G);
    const size_t lds = lds_bytes(fft_lds_elems(G * L, L), L);
    if (L == kFixedN && G == 1)
        hipLaunchKernelGGL(ar_rows_fwd_kernel<kFixedN>, grid, dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw, 1,
                           ar_shift_for(1));
    else if (fd.m > 0)
        hipLaunchKernelGGL(ar_rows_fwd_kernel<kAnyLen>, grid, dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw, G,
                           ar_shift_for(G));
    else
        hipLaunchKernelGGL(ar_rows_fwd_kernel<0>, grid, dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw, G,
                           ar_shift_for(G));
    return hipGetLastError();
}

hipError_t launch_ar_cols_filter(float* Tr, int n, int ts, const float* spec, float alpha, const float* lamr,
                                 const FftDesc& fd, const float2* tw, hipStream_t s, const double* red_in,
                                 int red_count, double* red_out) {
    const int CP = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + CP - 1) / CP);
    const size_t lds = lds_bytes(fft_lds_elems(CP * L, L), L);
    if (L == kFixedN && CP == 1)
        hipLaunchKernelGGL(ar_cols_filter_kernel<kFixedN>, grid, dim3(kBlock), lds, s, Tr, n, ts, spec, alpha, lamr,
                           fd, tw, 1, ar_shift_for(1), red_in, red_count, red_out);
    else if (fd.m > 0)
        hipLaunchKernelGGL(ar_cols_filter_kernel<kAnyLen>, grid, dim3(kBlock), lds, s, Tr, n, ts, spec, alpha, lamr, fd,
                           tw, CP, ar_shift_for(CP), red_in, red_count, red_out);
    else
        hipLaunchKernelGGL(ar_cols_filter_kernel<0>, grid, dim3(kBlock), lds, s, Tr, n, ts, spec, alpha, lamr, fd,
                           tw, CP, ar_shift_for(CP), red_in, red_count, red_out);
    return hipGetLastError();
}

hipError_t launch_ar_rows_inv(const float* Tr, int n, int ts, float* dst, const FftDesc& fd, const float2* tw,
                              hipStream_t s, int accum) {
    const int G = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + G - 1) / G);
    const size_t lds = lds_bytes(fft_lds_elems(G * L, L), L);
    if (L == kFixedN && G == 1)
        hipLaunchKernelGGL(ar_rows_inv_kernel<kFixedN>, grid, dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw, 1,
                           ar_shift_for(1), accum);
    else if (fd.m > 0)
        hipLaunchKernelGGL(ar_rows_inv_kernel<kAnyLen>, grid, dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw, G,
                           ar_shift_for(G), accum);
    else
        hipLaunchKernelGGL(ar_rows_inv_kernel<0>, grid, dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw, G,
                           ar_shift_for(G), accum);
    return hipGetLastError();
}

}  // namespace mlba
