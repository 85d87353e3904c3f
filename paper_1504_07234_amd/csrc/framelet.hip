// Undecimated linear B-spline framelet, one level per launch (paper section
// 6.1).  Masks at offsets (-d, 0, +d):
//   b0 = (1/4, 1/2, 1/4),  b1 = (-sqrt2/4, 0, sqrt2/4),  b2 = (-1/4, 1/2, -1/4)
// (b1 oriented as the rows of the matrix printed in section 6.1).  Band (i,j)
// applies b_i along x and b_j along y under half-sample reflective extension.
//
// Analysis + Bregman update: one thread per column and 8-row strip, no LDS;
// the x-direction taps at x-d and x+d are read from memory (cache hits) and
// every old coefficient of the strip is loaded before the first store.
// Synthesis: one thread per column of an 8-row strip; a workgroup covers 256
// - 2d output columns plus a d-column halo on each side.  Every thread
// streams its column of each of the 9 inputs (8 + 2d rows, coalesced across
// the wavefront) through registers, applies the y-direction transposes there,
// parks the three partial sums in LDS and, after one barrier, applies the
// x-direction transposes for the interior columns.
//
// The transpose (synthesis) uses the fact that for a symmetric mask the
// reflective operator's transpose is the mirrored mask applied to the
// symmetrically extended input, while for the antisymmetric mask b1 the
// input must be extended antisymmetrically (its mirrored copies change
// sign).  The soft threshold of eq. (soft) is applied to each coefficient as
// it is loaded.
#include "common.hpp"
#include "framelet.hpp"
#include "kernels.hpp"

namespace mlba {

// Analysis of one level: one thread per column, AN_TY rows per thread.  The
// x-direction filters read the two neighbouring columns straight from memory
// (cache hits); every old coefficient of the strip is loaded before the first
// store so that 9 * AN_TY independent loads are in flight per thread.

// x-direction filters h_i at column x on the rows y0-D .. y0+TY-1+D
template <int D, int TY = AN_TY>
__device__ __forceinline__ void analysis_xfilter(const float* __restrict__ v, int N, int x, int y0,
                                                 float* h0, float* h1, float* h2) {
    const int xl = reflect_index(x - D, N), xr = reflect_index(x + D, N);
#pragma unroll
    for (int q = 0; q < TY + 2 * D; ++q) {
        const float* row = v + (size_t)reflect_index(y0 - D + q, N) * N;
        const float a = row[xl], b = row[x], e = row[xr];
        h0[q] = fmaf(0.25f, a + e, 0.5f * b);
        h1[q] = kB1 * (e - a);
        h2[q] = fmaf(-0.25f, a + e, 0.5f * b);
    }
}

// y-direction filters of strip row r: the eight bands (slot pair_slot(i, j))
// and the low-pass (slot 8)
template <int D>
__device__ __forceinline__ void analysis_yfilter(const float* h0, const float* h1, const float* h2, int r,
                                                 float* out) {
    const float* hh[3] = {h0, h1, h2};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float a = hh[i][r], b = hh[i][r + D], e = hh[i][r + 2 * D];
        const float y0v = fmaf(0.25f, a + e, 0.5f * b);
        const float y1v = kB1 * (e - a);
        const float y2v = fmaf(-0.25f, a + e, 0.5f * b);
        if (i == 0) out[8] = y0v; else out[pair_slot(i, 0)] = y0v;
        out[pair_slot(i, 1)] = y1v;
        out[pair_slot(i, 2)] = y2v;
    }
}

// Old coefficients come from zin_lev / low_in (the same arrays as zlev / low
// for an in-place update; a new state slot otherwise).
template <int D>
__device__ __forceinline__ void analysis_tile(const float* __restrict__ v, int N, const float* zin_lev,
                                              const float* low_in, float* zlev, float* low, int accum_bands,
                                              int accum_low, int bx, int by) {
    const int x = bx * kBlock + threadIdx.x;
    const int y0 = by * AN_TY;
    if (x >= N) return;
    const size_t NN = (size_t)N * N;
    const int rows = min(AN_TY, N - y0);

    // old values of the 8 bands and the low-pass output for this strip
    float old[AN_TY][9];
    if (accum_bands) {
#pragma unroll
        for (int r = 0; r < AN_TY; ++r) {
            if (r < rows) {
                const size_t o = (size_t)(y0 + r) * N + x;
#pragma unroll
                for (int q = 0; q < 8; ++q) old[r][q] = zin_lev[q * NN + o];
                old[r][8] = accum_low ? low_in[o] : 0.0f;
            }
        }
    }

    float h0[AN_TY + 2 * D], h1[AN_TY + 2 * D], h2[AN_TY + 2 * D];
    analysis_xfilter<D>(v, N, x, y0, h0, h1, h2);

#pragma unroll
    for (int r = 0; r < AN_TY; ++r) {
        if (r >= rows) break;
        const size_t o = (size_t)(y0 + r) * N + x;
        float out[9];
        analysis_yfilter<D>(h0, h1, h2, r, out);
        if (accum_bands) {
#pragma unroll
            for (int q = 0; q < 9; ++q) out[q] += old[r][q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) zlev[q * NN + o] = out[q];
        low[o] = out[8];
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void analysis_level_kernel(const float* __restrict__ v, int N,
                                                                float* __restrict__ zlev,
                                                                float* __restrict__ low,
                                                                int accum_bands, int accum_low) {
    int bx, by;
    xcd_tile(&bx, &by);  // row halos of adjacent strips in one L2
    analysis_tile<D>(v, N, zlev, low, zlev, low, accum_bands, accum_low, bx, by);
}

// Reverse-sweep level: the filters of analysis_tile, and for every band value
// v the cotangent update under the active set of the forward state zk (the
// a.e. derivative of the soft threshold: 1{|zk| > mu}, 0 at the kink).  psum
// collects the thread's contribution to the threshold gradient per slot.
// A wave covers 64 columns x ADJ_TY rows and a workgroup four such strips
// stacked in y; the forward state and the old cotangent of the strip are
// loaded before the first store.
constexpr int ADJ_TY = 4;
constexpr int ADJ_TX = 64;

template <int D>
__device__ __forceinline__ void analysis_adjoint_tile(const float* __restrict__ v, int N,
                                                      const float* __restrict__ zk_lev,
                                                      float* __restrict__ zb_lev,
                                                      const float* __restrict__ zk_low,
                                                      float* __restrict__ zb_low,
                                                      float* __restrict__ low_out, const LevelMu& mu,
                                                      float delta, int init, int bx, int by, float* psum) {
#pragma unroll
    for (int q = 0; q < 9; ++q) psum[q] = 0.0f;
    const int x = bx * ADJ_TX + (threadIdx.x & (ADJ_TX - 1));
    const int y0 = (by * (kBlock / ADJ_TX) + (threadIdx.x / ADJ_TX)) * ADJ_TY;
    if (x >= N || y0 >= N) return;
    const size_t NN = (size_t)N * N;
    const int rows = min(ADJ_TY, N - y0);
    const bool last = zk_low != nullptr;
    const float sd = init ? delta : -delta;  // change of zbar per unit of v where active

    float zkv[ADJ_TY][9], zbv[ADJ_TY][9];
#pragma unroll
    for (int r = 0; r < ADJ_TY; ++r) {
        if (r < rows) {
            const size_t o = (size_t)(y0 + r) * N + x;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                zkv[r][q] = zk_lev[q * NN + o];
                zbv[r][q] = init ? 0.0f : zb_lev[q * NN + o];
            }
            zkv[r][8] = last ? zk_low[o] : 0.0f;
            zbv[r][8] = (last && !init) ? zb_low[o] : 0.0f;
        }
    }
    float h0[ADJ_TY + 2 * D], h1[ADJ_TY + 2 * D], h2[ADJ_TY + 2 * D];
    analysis_xfilter<D, ADJ_TY>(v, N, x, y0, h0, h1, h2);

#pragma unroll
    for (int r = 0; r < ADJ_TY; ++r) {
        if (r >= rows) break;
        const size_t o = (size_t)(y0 + r) * N + x;
        float out[9];
        analysis_yfilter<D>(h0, h1, h2, r, out);
        if (!last) low_out[o] = out[8];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            if (q == 8 && !last) continue;
            const float m = q < 8 ? mu.band[q] : mu.low;
            const bool act = fabsf(zkv[r][q]) > m;
            const float nv = act ? fmaf(sd, out[q], zbv[r][q]) : zbv[r][q];
            if (q < 8) zb_lev[q * NN + o] = nv;
            else zb_low[o] = nv;
            if (act) psum[q] -= sd * (zkv[r][q] > 0.0f ? out[q] : -out[q]);
        }
    }
}

template <int D>
__device__ __forceinline__ void synthesis_tile(const float* __restrict__ zlev, const float* __restrict__ low,
                                               int N, float* __restrict__ out, const LevelMu& mu, float delta,
                                               int thr_low, int thr_bands, int bx, int by,
                                               float (*ys)[FR_TY][kBlock]) {
    constexpr int IW = kBlock - 2 * D;
    const int x0 = bx * IW;
    const int y0 = by * FR_TY;
    const int c = threadIdx.x;
    bool fx;
    const int gx = reflect_index(x0 - D + c, N, &fx);
    const size_t NN = (size_t)N * N;

    // rows of the strip with halo, and whether each is a mirrored copy
    int rowi[FR_TY + 2 * D];
    bool rowf[FR_TY + 2 * D];
#pragma unroll
    for (int q = 0; q < FR_TY + 2 * D; ++q) {
        bool f;
        rowi[q] = reflect_index(y0 - D + q, N, &f);
        rowf[q] = f;
    }

    float acc[3][FR_TY];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < FR_TY; ++r) acc[i][r] = 0.0f;

#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const bool is_low = (i == 0 && j == 0);
            const float* src = is_low ? low : zlev + pair_slot(i, j) * NN;
            const bool thr = is_low ? (thr_low != 0) : (thr_bands != 0);
            const float m = is_low ? mu.low : mu.band[pair_slot(i, j)];
            const float sx = (i == 1 && fx) ? -1.0f : 1.0f;
            // issue the whole column's loads before using any of them
            float col[FR_TY + 2 * D];
#pragma unroll
            for (int q = 0; q < FR_TY + 2 * D; ++q) col[q] = src[(size_t)rowi[q] * N + gx];
#pragma unroll
            for (int q = 0; q < FR_TY + 2 * D; ++q) {
                float val = col[q];
                if (thr) val = shrink(val, m, delta);
                const float sy = (j == 1 && rowf[q]) ? -1.0f : 1.0f;
                col[q] = sx * sy * val;
            }
            // transpose along y: sum_k b_j[k] w~[y - k d]
#pragma unroll
            for (int r = 0; r < FR_TY; ++r) {
                const float wm = col[r], w0 = col[r + D], wp = col[r + 2 * D];  // y-d, y, y+d
                if (j == 0) acc[i][r] += fmaf(0.25f, wp + wm, 0.5f * w0);
                else if (j == 1) acc[i][r] = fmaf(kB1, wm - wp, acc[i][r]);
                else acc[i][r] += fmaf(-0.25f, wp + wm, 0.5f * w0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < FR_TY; ++r) ys[i][r][c] = acc[i][r];
    __syncthreads();

    if (c < D || c >= kBlock - D) return;
    const int x = x0 + c - D;
    if (x >= N) return;
    for (int r = 0; r < FR_TY; ++r) {
        const int y = y0 + r;
        if (y >= N) break;
        // transpose along x: sum_i sum_k b_i[k] Y_i[x - k d]
        float s = 0.0f;
        {
            const float l = ys[0][r][c - D], m = ys[0][r][c], rr = ys[0][r][c + D];
            s += fmaf(0.25f, rr + l, 0.5f * m);
        }
        {
            const float l = ys[1][r][c - D], rr = ys[1][r][c + D];
            s = fmaf(kB1, l - rr, s);
        }
        {
            const float l = ys[2][r][c - D], m = ys[2][r][c], rr = ys[2][r][c + D];
            s += fmaf(-0.25f, rr + l, 0.5f * m);
        }
        out[(size_t)y * N + x] = s;
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void synthesis_level_kernel(const float* __restrict__ zlev,
                                                                 const float* __restrict__ low, int N,
                                                                 float* __restrict__ out, LevelMu mu,
                                                                 float delta, int thr_low, int thr_bands) {
    __shared__ float ys[3][FR_TY][kBlock];
    int bx, by;
    xcd_tile(&bx, &by);  // row halos of adjacent strips in one L2
    synthesis_tile<D>(zlev, low, N, out, mu, delta, thr_low, thr_bands, bx, by, ys);
}

template <int D>
static hipError_t launch_an(const float* v, int N, float* zlev, float* low, int ab, int al, hipStream_t s) {
    dim3 grid((N + kBlock - 1) / kBlock, (N + AN_TY - 1) / AN_TY);
    hipLaunchKernelGGL((analysis_level_kernel<D>), grid, dim3(kBlock), 0, s, v, N, zlev, low, ab, al);
    return hipGetLastError();
}

hipError_t launch_analysis_level(const float* v, int N, int d, float* zlev, float* low, int accum_bands,
                                 int accum_low, hipStream_t s) {
    switch (d) {
        case 1: return launch_an<1>(v, N, zlev, low, accum_bands, accum_low, s);
        case 2: return launch_an<2>(v, N, zlev, low, accum_bands, accum_low, s);
        case 4: return launch_an<4>(v, N, zlev, low, accum_bands, accum_low, s);
        case 8: return launch_an<8>(v, N, zlev, low, accum_bands, accum_low, s);
        default: return hipErrorInvalidValue;
    }
}

template <int D>
static hipError_t launch_syn(const float* zlev, const float* low, int N, float* out, LevelMu mu, float delta,
                             int tl, int tb, hipStream_t s) {
    constexpr int IW = kBlock - 2 * D;
    dim3 grid((N + IW - 1) / IW, (N + FR_TY - 1) / FR_TY);
    hipLaunchKernelGGL((synthesis_level_kernel<D>), grid, dim3(kBlock), 0, s, zlev, low, N, out, mu, delta,
                       tl, tb);
    return hipGetLastError();
}

hipError_t launch_synthesis_level(const float* zlev, const float* low, int N, int d, float* out, LevelMu mu,
                                  float delta, int thr_low, int thr_bands, hipStream_t s) {
    switch (d) {
        case 1: return launch_syn<1>(zlev, low, N, out, mu, delta, thr_low, thr_bands, s);
        case 2: return launch_syn<2>(zlev, low, N, out, mu, delta, thr_low, thr_bands, s);
        case 4: return launch_syn<4>(zlev, low, N, out, mu, delta, thr_low, thr_bands, s);
        case 8: return launch_syn<8>(zlev, low, N, out, mu, delta, thr_low, thr_bands, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- batched levels: workgroup b serves image bmap[b], tile b - bfirst[img] ----

int synthesis_level_tiles(int N, int d) {
    const int IW = kBlock - 2 * d;
    return ((N + IW - 1) / IW) * ((N + FR_TY - 1) / FR_TY);
}

int analysis_level_tiles(int N, int d) { return ((N + kBlock - 1) / kBlock) * ((N + AN_TY - 1) / AN_TY); }

// level `lev` of W^T (delta S_mu(z)) for image I, exactly as the single-image
// path sequences it: level L reads the thresholded low-pass z_0, lower levels
// the previous level's output; level 1 writes u (or f for the final image).
template <int D>
__global__ __launch_bounds__(kBlock) void synthesis_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                   const int* __restrict__ bmap,
                                                                   const int* __restrict__ bfirst, int lev,
                                                                   int final_out, int thr) {
    __shared__ float ys[3][FR_TY][kBlock];
    const int xb = xcd_block(blockIdx.x, gridDim.x);  // adjacent tiles of an image in one L2
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const size_t nn = (size_t)I.N * I.N;
    const float* zlev = I.zin + (size_t)(1 + 8 * (lev - 1)) * nn;
    const bool top = lev == I.levels;
    const float* low = top ? I.zin : ((lev + 1) & 1 ? I.tmp1 : I.tmp0);
    float* out = lev == 1 ? (final_out ? I.f : I.u) : ((lev & 1) ? I.tmp1 : I.tmp0);
    LevelMu mu;
    mu.low = I.mu[0];
#pragma unroll
    for (int q = 0; q < 8; ++q) mu.band[q] = I.mu[1 + 8 * (lev - 1) + q];
    const int IW = kBlock - 2 * D;
    const int gx = (I.N + IW - 1) / IW;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    synthesis_tile<D>(zlev, low, I.N, out, mu, thr ? I.delta : 1.0f, (thr && top) ? 1 : 0, thr, local - by * gx,
                      by, ys);
}

template <int D>
__global__ __launch_bounds__(kBlock) void analysis_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                  const int* __restrict__ bmap,
                                                                  const int* __restrict__ bfirst, int lev) {
    const int xb = xcd_block(blockIdx.x, gridDim.x);  // adjacent tiles of an image in one L2
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const size_t nn = (size_t)I.N * I.N;
    const float* in = lev == 1 ? I.w : (((lev - 1) & 1) ? I.tmp1 : I.tmp0);
    const bool last = lev == I.levels;
    float* low = last ? I.z : ((lev & 1) ? I.tmp1 : I.tmp0);
    float* zlev = I.z + (size_t)(1 + 8 * (lev - 1)) * nn;
    const float* zin_lev = I.zin + (size_t)(1 + 8 * (lev - 1)) * nn;
    const int gx = (I.N + kBlock - 1) / kBlock;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    analysis_tile<D>(in, I.N, zin_lev, last ? I.zin : low, zlev, low, 1, last ? 1 : 0, local - by * gx, by);
}

template <int D>
__global__ __launch_bounds__(kBlock) void analysis_adjoint_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                          const int* __restrict__ bmap,
                                                                          const int* __restrict__ bfirst, int lev,
                                                                          int init, double* __restrict__ part) {
    __shared__ double red[9][kBlock / 64];
    const int xb = xcd_block(blockIdx.x, gridDim.x);  // adjacent tiles of an image in one L2
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const size_t nn = (size_t)I.N * I.N;
    const float* in = lev == 1 ? I.w : (((lev - 1) & 1) ? I.tmp1 : I.tmp0);
    const bool last = lev == I.levels;
    const size_t lo = (size_t)(1 + 8 * (lev - 1)) * nn;
    LevelMu mu;
    mu.low = I.mu[0];
#pragma unroll
    for (int q = 0; q < 8; ++q) mu.band[q] = I.mu[1 + 8 * (lev - 1) + q];
    const int gx = (I.N + ADJ_TX - 1) / ADJ_TX;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    float ps[9];
    analysis_adjoint_tile<D>(in, I.N, I.zk + lo, I.zbar + lo, last ? I.zk : nullptr, last ? I.zbar : nullptr,
                             last ? nullptr : ((lev & 1) ? I.tmp1 : I.tmp0), mu, I.delta, init, local - by * gx, by,
                             ps);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        double v = (double)ps[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[q][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[threadIdx.x][w];
        part[(size_t)blockIdx.x * 9 + threadIdx.x] += t;
    }
}

int analysis_adjoint_tiles(int N, int d) {
    constexpr int rows = (kBlock / ADJ_TX) * ADJ_TY;
    return ((N + ADJ_TX - 1) / ADJ_TX) * ((N + rows - 1) / rows);
}

hipError_t launch_analysis_adjoint_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                           int lev, int d, int init, double* part, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (d) {
        case 1: hipLaunchKernelGGL(analysis_adjoint_batched_kernel<1>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, init, part); break;
        case 2: hipLaunchKernelGGL(analysis_adjoint_batched_kernel<2>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, init, part); break;
        case 4: hipLaunchKernelGGL(analysis_adjoint_batched_kernel<4>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, init, part); break;
        case 8: hipLaunchKernelGGL(analysis_adjoint_batched_kernel<8>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, init, part); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_synthesis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                    int lev, int d, int final_out, hipStream_t s, int thr) {
    if (nblocks <= 0) return hipSuccess;
    switch (d) {
        case 1: hipLaunchKernelGGL(synthesis_batched_kernel<1>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, final_out, thr); break;
        case 2: hipLaunchKernelGGL(synthesis_batched_kernel<2>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, final_out, thr); break;
        case 4: hipLaunchKernelGGL(synthesis_batched_kernel<4>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, final_out, thr); break;
        case 8: hipLaunchKernelGGL(synthesis_batched_kernel<8>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev, final_out, thr); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_analysis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                   int lev, int d, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (d) {
        case 1: hipLaunchKernelGGL(analysis_batched_kernel<1>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        case 2: hipLaunchKernelGGL(analysis_batched_kernel<2>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        case 4: hipLaunchKernelGGL(analysis_batched_kernel<4>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        case 8: hipLaunchKernelGGL(analysis_batched_kernel<8>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

constexpr int FILL_CHUNK = kBlock * 1024;

int fill_tiles(const BatchImage& I) {
    const size_t count = (size_t)I.state_planes * I.N * I.N;
    return (int)((count + FILL_CHUNK - 1) / FILL_CHUNK);
}

__global__ __launch_bounds__(kBlock) void fill_batched_kernel(const BatchImage* __restrict__ imgs,
                                                              const int* __restrict__ bmap,
                                                              const int* __restrict__ bfirst) {
    const int xb = xcd_block(blockIdx.x, gridDim.x);  // adjacent tiles of an image in one L2
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const size_t count = (size_t)I.state_planes * I.N * I.N;
    const size_t beg = (size_t)(xb - bfirst[im]) * FILL_CHUNK;
    const size_t end = beg + FILL_CHUNK < count ? beg + FILL_CHUNK : count;
    for (size_t i = beg + threadIdx.x; i < end; i += kBlock) I.z[i] = 0.0f;
}

hipError_t launch_fill_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                               hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_batched_kernel, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void soft_threshold_kernel(const float* __restrict__ z,
                                                                float* __restrict__ x, size_t band_elems,
                                                                BandMu mu, float delta) {
    const int b = blockIdx.y;
    const size_t base = (size_t)b * band_elems;
    const float m = mu.v[b];
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < band_elems; i += (size_t)gridDim.x * kBlock)
        x[base + i] = shrink(z[base + i], m, delta);
}

hipError_t launch_soft_threshold(const float* z, float* x, int bands, size_t band_elems, BandMu mu,
                                 float delta, hipStream_t s) {
    size_t blocks = (band_elems + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) return hipSuccess;
    dim3 grid((unsigned)blocks, bands);
    hipLaunchKernelGGL(soft_threshold_kernel, grid, dim3(kBlock), 0, s, z, x, band_elems, mu, delta);
    return hipGetLastError();
}

}  // namespace mlba
