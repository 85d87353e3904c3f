// Direct LDS-tiled convolution for the blur A and its transpose A^T
// (paper section 2: A f is the valid part of the 2-D convolution of the
// extended image with the PSF; A^T y is the full correlation of y with the
// PSF, followed for imposed boundaries by the transpose of the padding).
//
// One workgroup computes a (32 RY) x 64 output tile.  The (32 RY + p - 1) x
// (64 + p - 1) input window is staged once in LDS under the requested
// boundary extension; every thread then owns an RY x 8 block of outputs and
// walks the p + RY - 1 input rows that feed it: each row segment (8 + p - 1
// values) is loaded into registers once and applied to every output row it
// contributes to (RY = 2 halves the LDS reads per FMA).  PSF taps are
// wavefront-uniform and are read through the scalar cache.  The PSF side is a template
// parameter for the odd sizes 1..33 (fully unrolled tap loops); larger PSFs
// use a generic kernel.
#include "common.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int CONV_TX = 64;  // output columns per workgroup (eight per thread)
constexpr int CONV_RX = 8;
// output rows per workgroup: 32 * RY with RY output rows per thread
template <int RY>
constexpr int conv_ty() { return 32 * RY; }

__host__ __device__ constexpr int conv_stride(int w) { return ((w + 7) / 8) * 8 + 1; }

template <int P, bool FLIP>
__device__ __forceinline__ float conv_tap(const float* __restrict__ psf, int a, int b) {
    return FLIP ? psf[(P - 1 - a) * P + (P - 1 - b)] : psf[a * P + b];
}

template <int P, bool FLIP, int RY>
__global__ __launch_bounds__(kBlock) void conv_kernel(const float* __restrict__ src, int S, int ext,
                                                      int org, float* __restrict__ dst, int D,
                                                      const float* __restrict__ g,
                                                      const float* __restrict__ psf,
                                                      double* __restrict__ partials) {
    constexpr int CONV_TY = conv_ty<RY>();
    constexpr int TH = CONV_TY + P - 1;
    constexpr int TW = CONV_TX + P - 1;
    constexpr int LS = conv_stride(TW);  // 8k+1 row stride: rows start on distinct banks
    __shared__ float tile[TH * LS];
    __shared__ double red[kBlock / 64];

    const int oy0 = blockIdx.y * CONV_TY;
    const int ox0 = blockIdx.x * CONV_TX;
    for (int i = threadIdx.x; i < TH * TW; i += kBlock) {
        const int ly = i / TW;
        const int lx = i - ly * TW;
        tile[ly * LS + lx] = fetch_ext(src, S, oy0 + org + ly, ox0 + org + lx, ext);
    }
    __syncthreads();

    // thread: output rows RY*ty .. RY*ty+RY-1, columns tx0 .. tx0+7; input
    // row RY*ty + q feeds output row RY*ty + h with kernel row q - h
    const int ty = threadIdx.x >> 3;
    const int tx0 = (threadIdx.x & 7) * CONV_RX;
    float acc[RY][CONV_RX];
#pragma unroll
    for (int h = 0; h < RY; ++h)
#pragma unroll
        for (int r = 0; r < CONV_RX; ++r) acc[h][r] = 0.0f;
    for (int q = 0; q < P + RY - 1; ++q) {
        const float* row = tile + (RY * ty + q) * LS + tx0;
        float seg[CONV_RX + P - 1];
#pragma unroll
        for (int k = 0; k < CONV_RX + P - 1; ++k) seg[k] = row[k];
#pragma unroll
        for (int h = 0; h < RY; ++h) {
            const int a = q - h;
            if (a >= 0 && a < P) {
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const float t = conv_tap<P, FLIP>(psf, a, b);
#pragma unroll
                    for (int r = 0; r < CONV_RX; ++r) acc[h][r] = fmaf(t, seg[r + b], acc[h][r]);
                }
            }
        }
    }

    double ss = 0.0;
#pragma unroll
    for (int h = 0; h < RY; ++h) {
        const int y = oy0 + RY * ty + h;
        if (y < D) {
#pragma unroll
            for (int r = 0; r < CONV_RX; ++r) {
                const int x = ox0 + tx0 + r;
                if (x < D) {
                    float v = acc[h][r];
                    if (g) {
                        v = g[(size_t)y * D + x] - v;
                        ss += (double)v * (double)v;
                    }
                    dst[(size_t)y * D + x] = v;
                }
            }
        }
    }
    if (partials) {
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// Generic PSF size (runtime p), same tiling, taps read from LDS.
__global__ __launch_bounds__(kBlock) void conv_kernel_generic(const float* __restrict__ src, int S,
                                                              int ext, int org, float* __restrict__ dst,
                                                              int D, const float* __restrict__ g,
                                                              const float* __restrict__ psf, int P,
                                                              int flip, double* __restrict__ partials) {
    extern __shared__ float smem[];
    __shared__ double red[kBlock / 64];
    constexpr int CONV_TY = conv_ty<2>();
    const int TH = CONV_TY + P - 1;
    const int TW = CONV_TX + P - 1;
    const int LS = conv_stride(TW);
    float* tile = smem;
    float* kern = smem + TH * LS;
    const int oy0 = blockIdx.y * CONV_TY;
    const int ox0 = blockIdx.x * CONV_TX;
    for (int i = threadIdx.x; i < TH * TW; i += kBlock) {
        const int ly = i / TW;
        const int lx = i - ly * TW;
        tile[ly * LS + lx] = fetch_ext(src, S, oy0 + org + ly, ox0 + org + lx, ext);
    }
    for (int i = threadIdx.x; i < P * P; i += kBlock) kern[i] = flip ? psf[P * P - 1 - i] : psf[i];
    __syncthreads();
    const int ty = threadIdx.x >> 3;
    const int tx0 = (threadIdx.x & 7) * CONV_RX;
    double ss = 0.0;
    for (int h = 0; h < 2; ++h) {
        float acc[CONV_RX];
#pragma unroll
        for (int r = 0; r < CONV_RX; ++r) acc[r] = 0.0f;
        for (int a = 0; a < P; ++a) {
            const float* row = tile + (2 * ty + h + a) * LS + tx0;
            for (int b = 0; b < P; ++b) {
                const float k = kern[a * P + b];
#pragma unroll
                for (int r = 0; r < CONV_RX; ++r) acc[r] = fmaf(k, row[r + b], acc[r]);
            }
        }
        const int y = oy0 + 2 * ty + h;
        if (y < D) {
            for (int r = 0; r < CONV_RX; ++r) {
                const int x = ox0 + tx0 + r;
                if (x < D) {
                    float v = acc[r];
                    if (g) {
                        v = g[(size_t)y * D + x] - v;
                        ss += (double)v * (double)v;
                    }
                    dst[(size_t)y * D + x] = v;
                }
            }
        }
    }
    if (partials) {
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// Output-tile height: two rows per thread (fewer LDS reads per FMA) unless
// the 64-row tiling leaves a nearly empty second round of workgroups, in
// which case one row per thread (32-row tiles) balances better.
static int conv_rows_per_thread(int D, int p) {
    const long t2 = (long)((D + CONV_TX - 1) / CONV_TX) * ((D + 63) / 64);
    const int lds2 = (64 + p - 1) * conv_stride(CONV_TX + p - 1) * 4;
    const long slots = 256L * (160 * 1024 / lds2);
    const long rounds = (t2 + slots - 1) / slots;
    const double fill = (double)t2 / (double)(rounds * slots);
    return fill >= 0.75 ? 2 : 1;
}

int conv_partials_count(int D) {
    // upper bound over both tilings
    return ((D + CONV_TX - 1) / CONV_TX) * ((D + 31) / 32);
}

template <int P, int RY>
static hipError_t launch_fixed_ry(const float* src, int S, int ext, int org, float* dst, int D, const float* g,
                                  const float* psf, int flip, double* partials, int* n_partials, hipStream_t s) {
    dim3 grid((D + CONV_TX - 1) / CONV_TX, (D + conv_ty<RY>() - 1) / conv_ty<RY>());
    if (n_partials) *n_partials = (int)(grid.x * grid.y);
    if (flip)
        hipLaunchKernelGGL((conv_kernel<P, true, RY>), grid, dim3(kBlock), 0, s, src, S, ext, org, dst, D, g,
                           psf, partials);
    else
        hipLaunchKernelGGL((conv_kernel<P, false, RY>), grid, dim3(kBlock), 0, s, src, S, ext, org, dst, D, g,
                           psf, partials);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_fixed(const float* src, int S, int ext, int org, float* dst, int D, const float* g,
                               const float* psf, int flip, double* partials, int* n_partials, hipStream_t s) {
    if (conv_rows_per_thread(D, P) == 2)
        return launch_fixed_ry<P, 2>(src, S, ext, org, dst, D, g, psf, flip, partials, n_partials, s);
    return launch_fixed_ry<P, 1>(src, S, ext, org, dst, D, g, psf, flip, partials, n_partials, s);
}

hipError_t launch_conv(const float* src, int S, int ext, int org, float* dst, int D, const float* g,
                       const float* psf, int p, int flip, double* partials, int* n_partials,
                       hipStream_t s) {
    switch (p) {
#define MLBA_CONV_CASE(PP) \
    case PP:               \
        return launch_fixed<PP>(src, S, ext, org, dst, D, g, psf, flip, partials, n_partials, s);
        MLBA_CONV_CASE(1)
        MLBA_CONV_CASE(3)
        MLBA_CONV_CASE(5)
        MLBA_CONV_CASE(7)
        MLBA_CONV_CASE(9)
        MLBA_CONV_CASE(11)
        MLBA_CONV_CASE(13)
        MLBA_CONV_CASE(15)
        MLBA_CONV_CASE(17)
        MLBA_CONV_CASE(19)
        MLBA_CONV_CASE(21)
        MLBA_CONV_CASE(23)
        MLBA_CONV_CASE(25)
        MLBA_CONV_CASE(27)
        MLBA_CONV_CASE(29)
        MLBA_CONV_CASE(31)
        MLBA_CONV_CASE(33)
#undef MLBA_CONV_CASE
        default: {
            constexpr int TY = conv_ty<2>();
            dim3 grid((D + CONV_TX - 1) / CONV_TX, (D + TY - 1) / TY);
            if (n_partials) *n_partials = (int)(grid.x * grid.y);
            const int TH = TY + p - 1;
            const int LS = conv_stride(CONV_TX + p - 1);
            const size_t lds = (size_t)(TH * LS + p * p) * sizeof(float);
            if (lds > 64 * 1024) return hipErrorInvalidValue;
            hipLaunchKernelGGL(conv_kernel_generic, grid, dim3(kBlock), lds, s, src, S, ext, org, dst, D, g,
                               psf, p, flip, partials);
            return hipGetLastError();
        }
    }
}

// Transpose of the half-sample reflective padding by c pixels.  A pixel k of
// the n-point axis is copied to padded positions k + c, c - 1 - k (when
// k < c) and 2n - 1 - k + c (when k >= n - c); p <= n keeps these distinct.
__device__ __forceinline__ int pad_preimages(int k, int n, int c, int* pre) {
    int cnt = 0;
    pre[cnt++] = k + c;
    if (k < c) pre[cnt++] = c - 1 - k;
    if (k >= n - c) pre[cnt++] = 2 * n - 1 - k + c;
    return cnt;
}

__global__ __launch_bounds__(kBlock) void fold_reflect_kernel(const float* __restrict__ wext, int m,
                                                              float* __restrict__ w, int n, int c) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= n) return;
    int py[3], px[3];
    const int cy = pad_preimages(y, n, c, py);
    const int cx = pad_preimages(x, n, c, px);
    float acc = 0.0f;
    for (int i = 0; i < cy; ++i)
        for (int j = 0; j < cx; ++j) acc += wext[(size_t)py[i] * m + px[j]];
    w[(size_t)y * n + x] = acc;
}

hipError_t launch_fold_reflect(const float* wext, int m, float* w, int n, int c, hipStream_t s) {
    dim3 grid((n + kBlock - 1) / kBlock, n);
    hipLaunchKernelGGL(fold_reflect_kernel, grid, dim3(kBlock), 0, s, wext, m, w, n, c);
    return hipGetLastError();
}

}  // namespace mlba
