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
// wavefront-uniform and are read through the scalar cache.  The PSF side is a
// template parameter for the odd sizes 1..33 (fully unrolled tap loops);
// larger PSFs use a generic body.
//
// The tile bodies are device functions shared by the single-image kernels and
// the batched kernel (one launch covering the tiles of many images), so both
// paths perform the same arithmetic in the same order.
#include "common.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int CONV_TX = 64;  // output columns per workgroup (eight per thread)
constexpr int CONV_RX = 8;

template <int RY>
constexpr int conv_ty() { return 32 * RY; }

__host__ __device__ constexpr int conv_stride(int w) { return ((w + 7) / 8) * 8 + 1; }

__host__ __device__ constexpr int conv_lds_floats(int p, int ry) {
    return (32 * ry + p - 1) * conv_stride(CONV_TX + p - 1);
}

int conv_tiles(int D, int ry) { return ((D + CONV_TX - 1) / CONV_TX) * ((D + 32 * ry - 1) / (32 * ry)); }

template <int P, bool FLIP>
__device__ __forceinline__ float conv_tap(const float* __restrict__ psf, int a, int b) {
    return FLIP ? psf[(P - 1 - a) * P + (P - 1 - b)] : psf[a * P + b];
}

__device__ __forceinline__ void conv_stage_window(const ConvJob& j, int P, int TY, int oy0, int ox0,
                                                  float* tile) {
    const int TH = TY + P - 1;
    const int TW = CONV_TX + P - 1;
    const int LS = conv_stride(TW);
    for (int i = threadIdx.x; i < TH * TW; i += kBlock) {
        const int ly = i / TW;
        const int lx = i - ly * TW;
        tile[ly * LS + lx] = fetch_ext(j.src, j.S, oy0 + j.org + ly, ox0 + j.org + lx, j.ext);
    }
}

// Writes (g - s) or s for the thread's outputs; returns its sum of squares of
// the written residuals (0 without g).
template <int RY>
__device__ __forceinline__ double conv_store(const ConvJob& j, int oy0, int ox0, int ty, int tx0,
                                             const float (*acc)[CONV_RX]) {
    double ss = 0.0;
#pragma unroll
    for (int h = 0; h < RY; ++h) {
        const int y = oy0 + RY * ty + h;
        if (y < j.D) {
#pragma unroll
            for (int r = 0; r < CONV_RX; ++r) {
                const int x = ox0 + tx0 + r;
                if (x < j.D) {
                    float v = acc[h][r];
                    if (j.g) {
                        v = j.g[(size_t)y * j.D + x] - v;
                        ss += (double)v * (double)v;
                    } else if (j.acc) {
                        v = j.dst[(size_t)y * j.D + x] + v;
                    }
                    j.dst[(size_t)y * j.D + x] = v;
                }
            }
        }
    }
    return ss;
}

// One output tile at tile coordinates (bx, by); `tile` is the LDS window.
template <int P, bool FLIP, int RY>
__device__ __forceinline__ double conv_tile(const ConvJob& j, int bx, int by, float* tile) {
    constexpr int TW = CONV_TX + P - 1;
    constexpr int LS = conv_stride(TW);  // 8k+1 row stride: rows start on distinct banks
    const int oy0 = by * conv_ty<RY>();
    const int ox0 = bx * CONV_TX;
    conv_stage_window(j, P, conv_ty<RY>(), oy0, ox0, tile);
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
#pragma unroll 1
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
                    const float t = conv_tap<P, FLIP>(j.psf, a, b);
#pragma unroll
                    for (int r = 0; r < CONV_RX; ++r) acc[h][r] = fmaf(t, seg[r + b], acc[h][r]);
                }
            }
        }
    }
    return conv_store<RY>(j, oy0, ox0, ty, tx0, acc);
}

// Runtime PSF side, 64-row tile, taps read from LDS after the window.
__device__ __forceinline__ double conv_tile_generic(const ConvJob& j, int P, int flip, int bx, int by,
                                                    float* smem) {
    constexpr int RY = 2;
    const int TY = conv_ty<RY>();
    const int LS = conv_stride(CONV_TX + P - 1);
    float* tile = smem;
    float* kern = smem + (TY + P - 1) * LS;
    const int oy0 = by * TY;
    const int ox0 = bx * CONV_TX;
    conv_stage_window(j, P, TY, oy0, ox0, tile);
    for (int i = threadIdx.x; i < P * P; i += kBlock) kern[i] = flip ? j.psf[P * P - 1 - i] : j.psf[i];
    __syncthreads();
    const int ty = threadIdx.x >> 3;
    const int tx0 = (threadIdx.x & 7) * CONV_RX;
    float acc[RY][CONV_RX];
    for (int h = 0; h < RY; ++h) {
#pragma unroll
        for (int r = 0; r < CONV_RX; ++r) acc[h][r] = 0.0f;
        for (int a = 0; a < P; ++a) {
            const float* row = tile + (RY * ty + h + a) * LS + tx0;
            for (int b = 0; b < P; ++b) {
                const float k = kern[a * P + b];
#pragma unroll
                for (int r = 0; r < CONV_RX; ++r) acc[h][r] = fmaf(k, row[r + b], acc[h][r]);
            }
        }
    }
    return conv_store<RY>(j, oy0, ox0, ty, tx0, acc);
}

__device__ __forceinline__ void conv_partial(double ss, double* red, double* out) {
    const double t = block_sum(ss, red);
    if (threadIdx.x == 0) *out = t;
}

// ---- single-image kernels -----------------------------------------------

template <int P, bool FLIP, int RY>
__global__ __launch_bounds__(kBlock) void conv_kernel(ConvJob j, double* __restrict__ partials) {
    __shared__ float tile[conv_lds_floats(P, RY)];
    __shared__ double red[kBlock / 64];
    int bx, by;
    xcd_tile(&bx, &by);
    const double ss = conv_tile<P, FLIP, RY>(j, bx, by, tile);
    if (partials) conv_partial(ss, red, partials + blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void conv_kernel_generic(ConvJob j, int P, int flip,
                                                              double* __restrict__ partials) {
    extern __shared__ float smem[];
    __shared__ double red[kBlock / 64];
    int bx, by;
    xcd_tile(&bx, &by);
    const double ss = conv_tile_generic(j, P, flip, bx, by, smem);
    if (partials) conv_partial(ss, red, partials + blockIdx.y * gridDim.x + blockIdx.x);
}

// Output-tile height: two rows per thread (fewer LDS reads per FMA) unless
// the 64-row tiling leaves a nearly empty second round of workgroups, in
// which case one row per thread (32-row tiles) balances better.
int conv_default_rows(int D, int p) {
    const long t2 = conv_tiles(D, 2);
    const int lds2 = conv_lds_floats(p, 2) * 4;
    const long slots = 256L * (160 * 1024 / lds2);
    const long rounds = (t2 + slots - 1) / slots;
    const double fill = (double)t2 / (double)(rounds * slots);
    return fill >= 0.75 ? 2 : 1;
}

int conv_partials_count(int D) { return conv_tiles(D, 1); }  // upper bound over both tilings

template <int P, int RY>
static hipError_t launch_fixed_ry(const ConvJob& j, int flip, double* partials, int* n_partials, hipStream_t s) {
    dim3 grid((j.D + CONV_TX - 1) / CONV_TX, (j.D + conv_ty<RY>() - 1) / conv_ty<RY>());
    if (n_partials) *n_partials = (int)(grid.x * grid.y);
    if (flip)
        hipLaunchKernelGGL((conv_kernel<P, true, RY>), grid, dim3(kBlock), 0, s, j, partials);
    else
        hipLaunchKernelGGL((conv_kernel<P, false, RY>), grid, dim3(kBlock), 0, s, j, partials);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_fixed(const ConvJob& j, int flip, int ry, double* partials, int* n_partials,
                               hipStream_t s) {
    if (ry != 1 && ry != 2) ry = conv_default_rows(j.D, P);
    if (ry == 2) return launch_fixed_ry<P, 2>(j, flip, partials, n_partials, s);
    return launch_fixed_ry<P, 1>(j, flip, partials, n_partials, s);
}

static size_t conv_generic_lds(int p) { return (size_t)(conv_lds_floats(p, 2) + p * p) * sizeof(float); }

hipError_t launch_conv_job(const ConvJob& j, int p, int flip, int ry, double* partials, int* n_partials,
                           hipStream_t s) {
    switch (p) {
#define MLBA_CONV_CASE(PP) \
    case PP:               \
        return launch_fixed<PP>(j, flip, ry, partials, n_partials, s);
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
            dim3 grid((j.D + CONV_TX - 1) / CONV_TX, (j.D + TY - 1) / TY);
            if (n_partials) *n_partials = (int)(grid.x * grid.y);
            const size_t lds = conv_generic_lds(p);
            if (lds > 64 * 1024) return hipErrorInvalidValue;
            hipLaunchKernelGGL(conv_kernel_generic, grid, dim3(kBlock), lds, s, j, p, flip, partials);
            return hipGetLastError();
        }
    }
}

// ---- batched kernel: tiles of many images in one launch ------------------
// Workgroup b serves image bmap[b], local tile b - bfirst[image].  Images with
// p <= 33 use one-row-per-thread tiles, larger PSFs the generic 64-row body.
// FLIP: r = g - A u with the residual-norm partial of the tile written to
// partials[pbase + local tile]; otherwise the A^T correlation.

template <bool FLIP, int RY>
__device__ __forceinline__ double conv_tile_dispatch(const ConvJob& j, int p, int bx, int by, float* lds) {
    switch (p) {
#define MLBA_CONV_DISPATCH(PP) \
    case PP:                   \
        return conv_tile<PP, FLIP, RY>(j, bx, by, lds);
        MLBA_CONV_DISPATCH(1)
        MLBA_CONV_DISPATCH(3)
        MLBA_CONV_DISPATCH(5)
        MLBA_CONV_DISPATCH(7)
        MLBA_CONV_DISPATCH(9)
        MLBA_CONV_DISPATCH(11)
        MLBA_CONV_DISPATCH(13)
        MLBA_CONV_DISPATCH(15)
        MLBA_CONV_DISPATCH(17)
        MLBA_CONV_DISPATCH(19)
        MLBA_CONV_DISPATCH(21)
        MLBA_CONV_DISPATCH(23)
        MLBA_CONV_DISPATCH(25)
        MLBA_CONV_DISPATCH(27)
        MLBA_CONV_DISPATCH(29)
        MLBA_CONV_DISPATCH(31)
        MLBA_CONV_DISPATCH(33)
#undef MLBA_CONV_DISPATCH
        default:
            return conv_tile_generic(j, p, FLIP ? 1 : 0, bx, by, lds);
    }
}

// rows per thread of an image's tiles: the launch's choice, or the generic
// body's 64-row tiles for p > 33
static int batched_rows(int p, int ry) { return p > 33 ? 2 : ry; }

template <bool FLIP, int RY>
__global__ __launch_bounds__(kBlock) void conv_batched_kernel(const BatchImage* __restrict__ imgs,
                                                              const int* __restrict__ bmap,
                                                              const int* __restrict__ bfirst,
                                                              double* __restrict__ partials) {
    extern __shared__ float smem[];
    __shared__ double red[kBlock / 64];
    const int im = bmap[blockIdx.x];
    const BatchImage& I = imgs[im];
    const ConvJob j = FLIP ? blur_job(I) : blurT_job(I);
    const int local = blockIdx.x - bfirst[im];
    const int gx = (j.D + CONV_TX - 1) / CONV_TX;
    const int by = local / gx;
    const int bx = local - by * gx;
    const double ss = conv_tile_dispatch<FLIP, RY>(j, I.p, bx, by, smem);
    if (FLIP && partials) conv_partial(ss, red, partials + I.pbase + local);
}

int conv_batched_tiles(const BatchImage& I, int flip, int ry) {
    const ConvJob j = flip ? blur_job(I) : blurT_job(I);
    return conv_tiles(j.D, batched_rows(I.p, ry));
}

static size_t conv_batched_lds(int pmax, int ry) {
    const size_t fixed = (size_t)conv_lds_floats(pmax < 33 ? pmax : 33, ry) * sizeof(float);
    if (pmax <= 33) return fixed;
    const size_t gen = conv_generic_lds(pmax);
    return gen > fixed ? gen : fixed;
}

template <bool FLIP, int RY>
static hipError_t launch_cb(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int pmax,
                            double* partials, hipStream_t s) {
    const size_t lds = conv_batched_lds(pmax, RY);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv_batched_kernel<FLIP, RY>), dim3(nblocks), dim3(kBlock), lds, s, imgs, bmap, bfirst,
                       partials);
    return hipGetLastError();
}

hipError_t launch_conv_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int flip,
                               int pmax, double* partials, hipStream_t s, int ry) {
    if (nblocks <= 0) return hipSuccess;
    if (flip) return ry == 2 ? launch_cb<true, 2>(imgs, bmap, bfirst, nblocks, pmax, partials, s)
                             : launch_cb<true, 1>(imgs, bmap, bfirst, nblocks, pmax, partials, s);
    return ry == 2 ? launch_cb<false, 2>(imgs, bmap, bfirst, nblocks, pmax, nullptr, s)
                   : launch_cb<false, 1>(imgs, bmap, bfirst, nblocks, pmax, nullptr, s);
}

// ---- transpose of the reflective padding ---------------------------------
// A pixel k of the n-point axis is copied to padded positions k + c, c - 1 - k
// (when k < c) and 2n - 1 - k + c (when k >= n - c); p <= n keeps these
// distinct.
__device__ __forceinline__ int pad_preimages(int k, int n, int c, int* pre) {
    int cnt = 0;
    pre[cnt++] = k + c;
    if (k < c) pre[cnt++] = c - 1 - k;
    if (k >= n - c) pre[cnt++] = 2 * n - 1 - k + c;
    return cnt;
}

__device__ __forceinline__ void fold_pixel(const float* __restrict__ wext, int m, float* __restrict__ w, int n,
                                           int c, int y, int x, int accum = 0) {
    int py[3], px[3];
    const int cy = pad_preimages(y, n, c, py);
    const int cx = pad_preimages(x, n, c, px);
    float acc = 0.0f;
    for (int i = 0; i < cy; ++i)
        for (int k = 0; k < cx; ++k) acc += wext[(size_t)py[i] * m + px[k]];
    w[(size_t)y * n + x] = accum ? w[(size_t)y * n + x] + acc : acc;
}

__global__ __launch_bounds__(kBlock) void fold_reflect_kernel(const float* __restrict__ wext, int m,
                                                              float* __restrict__ w, int n, int c, int accum) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x < n) fold_pixel(wext, m, w, n, c, blockIdx.y, x, accum);
}

hipError_t launch_fold_reflect(const float* wext, int m, float* w, int n, int c, hipStream_t s, int accum) {
    dim3 grid((n + kBlock - 1) / kBlock, n);
    hipLaunchKernelGGL(fold_reflect_kernel, grid, dim3(kBlock), 0, s, wext, m, w, n, c, accum);
    return hipGetLastError();
}

// batched fold: workgroup b covers row (b - bfirst[img]) of image bmap[b]
__global__ __launch_bounds__(kBlock) void fold_batched_kernel(const BatchImage* __restrict__ imgs,
                                                              const int* __restrict__ bmap,
                                                              const int* __restrict__ bfirst) {
    const int im = bmap[blockIdx.x];
    const BatchImage& I = imgs[im];
    const int y = blockIdx.x - bfirst[im];
    const int m = I.n + I.p - 1;
    for (int x = threadIdx.x; x < I.n; x += kBlock) fold_pixel(I.wext, m, I.w, I.n, I.c, y, x, I.blur_acc);
}

hipError_t launch_fold_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                               hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(fold_batched_kernel, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst);
    return hipGetLastError();
}

}  // namespace mlba
