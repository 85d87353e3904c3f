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
// The transform length 2N must be 2^a 3^b 5^c and at most FFT_MAX_ELEMS.
#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int kArMaxBatch = 8;  // sequences per workgroup at most

// Value k (0 <= k < 2N) of the odd extension of the detrended sequence
// v[0..N] read through `at` (positions 0 and N are zero).
template <typename At>
__device__ __forceinline__ float ar_odd_detrended(At at, int k, int N, float invN) {
    if (k == 0 || k == N) return 0.0f;
    const int kk = k < N ? k : 2 * N - k;
    const float v0 = at(0), vN = at(N);
    const float g = at(kk) - v0 - (vN - v0) * ((float)kk * invN);
    return k < N ? g : -g;
}

// G row pairs per workgroup -> Tr[j][y] (row stride ts >= n + 1, j = 0..N)
template <int NT>
__device__ __forceinline__ void ar_rows_fwd_body(const float* __restrict__ src, int n, float* __restrict__ Tr,
                                                 int ts, const FftDesc& fd, const float2* __restrict__ tw, int G,
                                                 int seq_shift, int blk, float2* buf) {
    const int N = n - 1, L = 2 * N;
    const float invN = 1.0f / (float)N;
    const int row0 = blk * 2 * G;
    for (int idx = threadIdx.x; idx < G * L; idx += kBlock) {
        const int g = idx / L;
        const int k = idx - g * L;
        const int ya = row0 + 2 * g;
        float2 v = make_float2(0.0f, 0.0f);
        if (ya < n) {
            const float* ra = src + (size_t)ya * n;
            v.x = ar_odd_detrended([&](int q) { return ra[q]; }, k, N, invN);
            if (ya + 1 < n) v.y = ar_odd_detrended([&](int q) { return ra[n + q]; }, k, N, invN);
        }
        buf[lds_slot(idx)] = v;
    }
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw);
    for (int idx = threadIdx.x; idx < G * n; idx += kBlock) {
        const int j = idx / G;
        const int g = idx - j * G;
        const int ya = row0 + 2 * g;
        if (ya >= n) continue;
        float2 c;
        if (j == 0 || j == N) {
            c.x = src[(size_t)ya * n + j];
            c.y = ya + 1 < n ? src[(size_t)(ya + 1) * n + j] : 0.0f;
        } else {
            const float2 X = buf[lds_slot(g * L + j)];
            c = make_float2(-X.y * invN, X.x * invN);  // (2/N) DST-I
        }
        *reinterpret_cast<float2*>(Tr + (size_t)j * ts + ya) = c;
    }
}

// CP pairs of Tr rows per workgroup: T^-1 along the row, filter, T back.
// filter[j] = 1 / (spec + alpha), times lamr for Algorithm 4 (dense [n][n],
// spec[jx][jy]).
template <int NT>
__device__ __forceinline__ void ar_cols_filter_body(float* __restrict__ Tr, int n, int ts,
                                                    const float* __restrict__ spec, float alpha,
                                                    const float* __restrict__ lamr, const FftDesc& fd,
                                                    const float2* __restrict__ tw, int CP, int seq_shift, int blk,
                                                    float2* buf, float2* lin /* [CP][2] */) {
    const int N = n - 1, L = 2 * N;
    const float invN = 1.0f / (float)N;
    const int pairs = (n + 1) / 2;
    const int p0 = blk * CP;
    const int cp = min(CP, pairs - p0);
    for (int idx = threadIdx.x; idx < cp * L; idx += kBlock) {
        const int q = idx / L;
        const int k = idx - q * L;
        const int ja = 2 * (p0 + q);
        const float* ra = Tr + (size_t)ja * ts;
        float2 v;
        v.x = ar_odd_detrended([&](int i) { return ra[i]; }, k, N, invN);
        v.y = ja + 1 < n ? ar_odd_detrended([&](int i) { return ra[ts + i]; }, k, N, invN) : 0.0f;
        buf[lds_slot(idx)] = v;
    }
    // the filtered linear coefficients of every sequence
    if (threadIdx.x < 2 * cp) {
        const int q = threadIdx.x >> 1;
        const int j = (threadIdx.x & 1) ? N : 0;
        const int ja = 2 * (p0 + q);
        const size_t sa = (size_t)ja * n + j;
        float fa = 1.0f / (spec[sa] + alpha);
        if (lamr) fa *= lamr[sa];
        float2 c = make_float2(Tr[(size_t)ja * ts + j] * fa, 0.0f);
        if (ja + 1 < n) {
            float fb = 1.0f / (spec[sa + n] + alpha);
            if (lamr) fb *= lamr[sa + n];
            c.y = Tr[(size_t)(ja + 1) * ts + j] * fb;
        }
        lin[2 * q + (threadIdx.x & 1)] = c;
    }
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, cp, seq_shift, tw);

    // filtered sine coefficients j = 1..N-1, held in registers while the
    // sequence is rebuilt as their odd extension
    constexpr int KEEP = FFT_MAX_ELEMS / 2 / kBlock;
    const int tot = cp * (N - 1);
    float2 keep[KEEP];
#pragma unroll
    for (int i = 0; i < KEEP; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < tot) {
            const int q = idx / (N - 1);
            const int j = 1 + idx - q * (N - 1);
            const int ja = 2 * (p0 + q);
            const float2 X = buf[lds_slot(q * L + j)];
            const size_t sa = (size_t)ja * n + j;
            float fa = 1.0f / (spec[sa] + alpha);
            if (lamr) fa *= lamr[sa];
            float fb = 0.0f;
            if (ja + 1 < n) {
                fb = 1.0f / (spec[sa + n] + alpha);
                if (lamr) fb *= lamr[sa + n];
            }
            keep[i] = make_float2(-X.y * invN * fa, X.x * invN * fb);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KEEP; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < tot) {
            const int q = idx / (N - 1);
            const int j = 1 + idx - q * (N - 1);
            buf[lds_slot(q * L + j)] = keep[i];
            buf[lds_slot(q * L + L - j)] = make_float2(-keep[i].x, -keep[i].y);
        }
    }
    if (threadIdx.x < 2 * cp) {
        const int q = threadIdx.x >> 1;
        buf[lds_slot(q * L + ((threadIdx.x & 1) ? N : 0))] = make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, cp, seq_shift, tw);
    for (int idx = threadIdx.x; idx < cp * n; idx += kBlock) {
        const int q = idx / n;
        const int k = idx - q * n;
        const int ja = 2 * (p0 + q);
        const float2 X = buf[lds_slot(q * L + k)];
        const float2 c0 = lin[2 * q], cN = lin[2 * q + 1];
        const float t = (float)k * invN;
        float* ra = Tr + (size_t)ja * ts;
        ra[k] = c0.x + (cN.x - c0.x) * t - 0.5f * X.y;
        if (ja + 1 < n) ra[ts + k] = c0.y + (cN.y - c0.y) * t + 0.5f * X.x;
    }
}

template <int NT>
__device__ __forceinline__ void ar_rows_inv_body(const float* __restrict__ Tr, int n, int ts,
                                                 float* __restrict__ dst, const FftDesc& fd,
                                                 const float2* __restrict__ tw, int G, int seq_shift, int blk,
                                                 float2* buf, int accum) {
    const int N = n - 1, L = 2 * N;
    const float invN = 1.0f / (float)N;
    const int row0 = blk * 2 * G;
    for (int idx = threadIdx.x; idx < G * L; idx += kBlock) {
        const int k = idx / G;
        const int g = idx - k * G;
        const int ya = row0 + 2 * g;
        float2 v = make_float2(0.0f, 0.0f);
        if (ya < n && k != 0 && k != N) {
            const int kk = k < N ? k : L - k;
            v = *reinterpret_cast<const float2*>(Tr + (size_t)kk * ts + ya);
            if (k > N) v = make_float2(-v.x, -v.y);
        }
        buf[lds_slot(g * L + k)] = v;
    }
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw);
    for (int idx = threadIdx.x; idx < G * n; idx += kBlock) {
        const int g = idx / n;
        const int x = idx - g * n;
        const int ya = row0 + 2 * g;
        if (ya >= n) continue;
        const float2 X = buf[lds_slot(g * L + x)];
        const float2 c0 = *reinterpret_cast<const float2*>(Tr + ya);
        const float2 cN = *reinterpret_cast<const float2*>(Tr + (size_t)N * ts + ya);
        const float t = (float)x * invN;
        const float va = c0.x + (cN.x - c0.x) * t - 0.5f * X.y;
        const float vb = c0.y + (cN.y - c0.y) * t + 0.5f * X.x;
        const size_t oa = (size_t)ya * n + x;
        if (accum) {
            dst[oa] += va;
            if (ya + 1 < n) dst[oa + n] += vb;
        } else {
            dst[oa] = va;
            if (ya + 1 < n) dst[oa + n] = vb;
        }
    }
}

template <int NT>
__global__ __launch_bounds__(kBlock) void ar_rows_fwd_kernel(const float* __restrict__ src, int n,
                                                             float* __restrict__ Tr, int ts, FftDesc fd,
                                                             const float2* __restrict__ tw, int G, int seq_shift) {
    extern __shared__ float2 buf[];
    ar_rows_fwd_body<NT>(src, n, Tr, ts, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void ar_cols_filter_kernel(float* __restrict__ Tr, int n, int ts,
                                                                const float* __restrict__ spec, float alpha,
                                                                const float* __restrict__ lamr, FftDesc fd,
                                                                const float2* __restrict__ tw, int CP,
                                                                int seq_shift) {
    extern __shared__ float2 buf[];
    __shared__ float2 lin[2 * kArMaxBatch];
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
    while (G * 2 <= kArMaxBatch && (G * 2) * L <= FFT_MAX_ELEMS && pairs / (G * 2) >= 256) G *= 2;
    return G;
}

bool ar_transform_supported(int n) {
    if (n < 4) return false;
    int m = 2 * (n - 1);
    if (m > FFT_MAX_ELEMS) return false;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    while (m % 5 == 0) m /= 5;
    return m == 1;
}

int ar_workspace_stride(int n) { return ((n + 1 + 15) / 16) * 16 + 16; }

// the compiled fixed-size transform when the length is kFixedN with one
// sequence per workgroup (n = 1025), the run-time plan otherwise
hipError_t launch_ar_rows_fwd(const float* src, int n, float* Tr, int ts, const FftDesc& fd, const float2* tw,
                              hipStream_t s) {
    const int G = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + G - 1) / G);
    const size_t lds = lds_bytes(G * L, L);
    if (L == kFixedN && G == 1)
        hipLaunchKernelGGL(ar_rows_fwd_kernel<kFixedN>, grid, dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw, 1,
                           ar_shift_for(1));
    else
        hipLaunchKernelGGL(ar_rows_fwd_kernel<0>, grid, dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw, G,
                           ar_shift_for(G));
    return hipGetLastError();
}

hipError_t launch_ar_cols_filter(float* Tr, int n, int ts, const float* spec, float alpha, const float* lamr,
                                 const FftDesc& fd, const float2* tw, hipStream_t s) {
    const int CP = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + CP - 1) / CP);
    const size_t lds = lds_bytes(CP * L, L);
    if (L == kFixedN && CP == 1)
        hipLaunchKernelGGL(ar_cols_filter_kernel<kFixedN>, grid, dim3(kBlock), lds, s, Tr, n, ts, spec, alpha, lamr,
                           fd, tw, 1, ar_shift_for(1));
    else
        hipLaunchKernelGGL(ar_cols_filter_kernel<0>, grid, dim3(kBlock), lds, s, Tr, n, ts, spec, alpha, lamr, fd,
                           tw, CP, ar_shift_for(CP));
    return hipGetLastError();
}

hipError_t launch_ar_rows_inv(const float* Tr, int n, int ts, float* dst, const FftDesc& fd, const float2* tw,
                              hipStream_t s, int accum) {
    const int G = ar_batch(n), L = 2 * (n - 1), pairs = (n + 1) / 2;
    const dim3 grid((pairs + G - 1) / G);
    const size_t lds = lds_bytes(G * L, L);
    if (L == kFixedN && G == 1)
        hipLaunchKernelGGL(ar_rows_inv_kernel<kFixedN>, grid, dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw, 1,
                           ar_shift_for(1), accum);
    else
        hipLaunchKernelGGL(ar_rows_inv_kernel<0>, grid, dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw, G,
                           ar_shift_for(G), accum);
    return hipGetLastError();
}

}  // namespace mlba
