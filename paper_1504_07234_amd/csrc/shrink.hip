// Implicit state of the framelet iteration (paper section 6.1 framelet,
// eq. (MLBA2) with z = W omega): the low-pass chain and the fused
// band / soft-threshold / synthesis levels.
#include "common.hpp"
#include "framelet.hpp"
#include "kernels.hpp"

namespace mlba {

// ---- implicit state: z = W omega is never stored -------------------------
// Every update of eq. (MLBA2) is W applied to A^T t, so z^k = W omega^k with
// omega^{k+1} = omega^k + A^T t_k (one N x N plane).  u = W^T(delta S_mu(W omega))
// is evaluated level by level from the low-pass chain low_0 = omega,
// low_l = (b0 x b0) low_{l-1}: the synthesis of level l recomputes that level's
// eight bands from low_{l-1} instead of reading them.
//
// Extension: with the half-sample symmetric extension of low_{l-1}, a
// symmetric mask (b0, b2) yields a symmetrically extended band and the
// antisymmetric b1 an antisymmetrically extended one; the soft threshold is
// odd, so it keeps both.  Evaluating the bands at extended positions from the
// extended low-pass therefore gives exactly the signed extension that the
// synthesis transposes need (the sign flips of synthesis_tile come out of the
// arithmetic), and no other boundary logic is required.

// low_out = (b0 x b0) v with dilation D: the (0,0) band of analysis_tile,
// over the AN_TY-row strip by of the kBlock-column block bx
template <int D>
__device__ __forceinline__ void lowpass_tile(const float* __restrict__ v, int N, float* __restrict__ out, int bx,
                                             int by) {
    const int x = bx * kBlock + threadIdx.x;
    const int y0 = by * AN_TY;
    if (x >= N) return;
    const int rows = min(AN_TY, N - y0);
    const int xl = reflect_index(x - D, N), xr = reflect_index(x + D, N);
    float h0[AN_TY + 2 * D];
#pragma unroll
    for (int q = 0; q < AN_TY + 2 * D; ++q) {
        const float* row = v + (size_t)reflect_index(y0 - D + q, N) * N;
        h0[q] = fmaf(0.25f, row[xl] + row[xr], 0.5f * row[x]);
    }
#pragma unroll
    for (int r = 0; r < AN_TY; ++r) {
        if (r >= rows) break;
        out[(size_t)(y0 + r) * N + x] = fmaf(0.25f, h0[r] + h0[r + 2 * D], 0.5f * h0[r + D]);
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void lowpass_level_kernel(const float* __restrict__ v, int N,
                                                               float* __restrict__ out) {
    lowpass_tile<D>(v, N, out, blockIdx.x, blockIdx.y);
}

// low_1 = (b0 x b0) v (dilation 1) and low_2 = (b0 x b0) low_1 (dilation 2)
// in one pass over v.  Thread c holds the extended column xe = x0 - 2 + c;
// low_1 is computed there for the strip rows and a 2-row halo straight from
// v (b0 is symmetric, so at a reflected position it equals low_1 at the
// mirrored one, with the same additions), kept in LDS for the dilation-2
// filter, and written for the strip's own rows and columns.
constexpr int LP2_TY = 8;

__global__ __launch_bounds__(kBlock) void lowpass_two_levels_kernel(const float* __restrict__ v, int N,
                                                                    float* __restrict__ low1,
                                                                    float* __restrict__ low2) {
    constexpr int IW = kBlock - 4;
    constexpr int HR = LP2_TY + 4;  // low_1 rows y0-2 .. y0+TY+1
    __shared__ float l1[HR][kBlock];
    int bx, by;
    xcd_tile(&bx, &by);
    const int x0 = bx * IW;
    const int y0 = by * LP2_TY;
    const int c = threadIdx.x;
    const int xe = x0 - 2 + c;
    const int xm = reflect_index(xe, N), xl = reflect_index(xe - 1, N), xr = reflect_index(xe + 1, N);
    size_t rowo[HR + 2];
#pragma unroll
    for (int q = 0; q < HR + 2; ++q) rowo[q] = (size_t)reflect_index(y0 - 3 + q, N) * N;
    float h[HR + 2];
#pragma unroll
    for (int q = 0; q < HR + 2; ++q) {
        const float* row = v + rowo[q];
        h[q] = fmaf(0.25f, row[xl] + row[xr], 0.5f * row[xm]);
    }
#pragma unroll
    for (int q = 0; q < HR; ++q) l1[q][c] = fmaf(0.25f, h[q] + h[q + 2], 0.5f * h[q + 1]);
    const bool own = c >= 2 && c < kBlock - 2 && xe < N;
    if (own) {
#pragma unroll
        for (int r = 0; r < LP2_TY; ++r) {
            if (y0 + r < N) low1[(size_t)(y0 + r) * N + xe] = l1[r + 2][c];
        }
    }
    __syncthreads();
    if (!own) return;
    float g[HR];
#pragma unroll
    for (int q = 0; q < HR; ++q) g[q] = fmaf(0.25f, l1[q][c - 2] + l1[q][c + 2], 0.5f * l1[q][c]);
#pragma unroll
    for (int r = 0; r < LP2_TY; ++r) {
        if (y0 + r >= N) break;
        low2[(size_t)(y0 + r) * N + xe] = fmaf(0.25f, g[r] + g[r + 4], 0.5f * g[r + 2]);
    }
}

hipError_t launch_lowpass_two_levels(const float* v, int N, float* low1, float* low2, hipStream_t s) {
    dim3 grid((N + kBlock - 5) / (kBlock - 4), (N + LP2_TY - 1) / LP2_TY);
    hipLaunchKernelGGL(lowpass_two_levels_kernel, grid, dim3(kBlock), 0, s, v, N, low1, low2);
    return hipGetLastError();
}

// Level with dilation D of W^T(delta S_mu(.)) fed by low = low_{l-1}: the
// eight bands of the level are computed from low, thresholded and transposed;
// the (0,0) input is the thresholded low-pass (s_in == null: top level) or
// s_in, the output of the level above.  Same workgroup geometry as
// synthesis_tile: one thread per column of an FR_TY-row strip, 256 - 2D
// output columns per workgroup.
template <int D, int TY>
struct SsTile {
    static constexpr int IW = kBlock - 2 * D;  // output columns per workgroup
    static constexpr int HR = TY + 4 * D;      // low-pass rows: y0-2D .. y0+TY+2D-1
    static constexpr int BR = TY + 2 * D;      // band rows: y0-D .. y0+TY+D-1
    static constexpr int LW = kBlock + 2 * D;  // low-pass columns: x0-2D .. x0+kBlock-1
    static constexpr int LOW_FLOATS = HR * LW;
    static constexpr int YS_FLOATS = 2 * TY * kBlock;
    static constexpr int LDS_FLOATS = LOW_FLOATS > YS_FLOATS ? LOW_FLOATS : YS_FLOATS;
};

// The low-pass tile is staged in LDS once (coalesced rows, reflected
// indices); each thread then filters its extended column from LDS.  The LDS
// is reused for the x-synthesis after the last x-filter.  With y_i the
// y-synthesised input of x-filter i at a column, the three x-synthesis
// transposes sum to
//   out(x) = 2 (y_0 + y_2)(x) + (y_0 - y_2 + y_1)(x - d) + (y_0 - y_2 - y_1)(x + d),
// so each thread keeps the first term and passes only the two neighbour
// terms through LDS.
//
// Arithmetic: the masks are applied unnormalised, b0 = [1 2 1] / 4,
// b1 = [-1 0 1] sqrt(2)/4, b2 = [-1 2 -1] / 4, i.e. b_i = c_i m_i with
// c = (1/4, sqrt(2)/4, 1/4); the three x (and y) filters then share a + e and
// 2b.  Band (i, j) computed with the unnormalised masks is the band divided by
// c_i c_j, and S_mu(c v) = c S_{mu/c}(v) for c > 0, so it is thresholded at
// mu / (c_i c_j); its synthesis with the unnormalised transposes is weighted
// by F_ij = delta (c_i c_j)^2 (both scale factors and the step).  Below the top
// level the (0, 0) input is the level above's output itself, weighted by
// c_0^2 only.
// Per band (i, j): the threshold of the unnormalised coefficient and its
// synthesis weight (SsCoef, computed on the host by ss_coef).

template <int D, int TY, bool SIN>
__device__ __forceinline__ void shrink_synthesis_tile(const float* __restrict__ low, const float* __restrict__ s_in,
                                                      int N, float* __restrict__ out, const SsCoef& cf, int bx,
                                                      int by, float* lds) {
    using G = SsTile<D, TY>;
    constexpr int HR = G::HR, BR = G::BR, LW = G::LW;
    const int x0 = bx * G::IW;
    const int y0 = by * TY;
    const int c = threadIdx.x;
    const int xe = x0 - D + c;  // extended column of this thread
    float* L = lds;             // [HR][LW]
    // row offsets first (uniform), so that every load of a column is in flight at once
    size_t rowo[HR];
#pragma unroll
    for (int q = 0; q < HR; ++q) rowo[q] = (size_t)reflect_index(y0 - 2 * D + q, N) * N;
    // tile columns 0 .. kBlock-1: one per thread; the 2D columns beyond them
    // (HR x 2D values) spread over the threads, loaded in the same batch
    constexpr int HALO = HR * 2 * D;
    constexpr int HPT = (HALO + kBlock - 1) / kBlock;
    float v[HR], hv[HPT];
    int hslot[HPT];
    {
        const int col = reflect_index(x0 - 2 * D + c, N);
#pragma unroll
        for (int q = 0; q < HR; ++q) v[q] = low[rowo[q] + col];
#pragma unroll
        for (int h = 0; h < HPT; ++h) {
            const int e = h * kBlock + c;
            hslot[h] = -1;
            if (HALO % kBlock == 0 || e < HALO) {
                const int q = e / (2 * D), k = kBlock + e % (2 * D);
                hslot[h] = q * LW + k;
                hv[h] = low[(size_t)reflect_index(y0 - 2 * D + q, N) * N + reflect_index(x0 - 2 * D + k, N)];
            }
        }
    }
    // the level above's output at this column (read by the first filter pass)
    float sc[BR];
    if constexpr (SIN) {
        const int xm = reflect_index(xe, N);
#pragma unroll
        for (int q = 0; q < BR; ++q) sc[q] = s_in[rowo[q + D] + xm];
    }
#pragma unroll
    for (int q = 0; q < HR; ++q) L[q * LW + c] = v[q];
#pragma unroll
    for (int h = 0; h < HPT; ++h)
        if (hslot[h] >= 0) L[hslot[h]] = hv[h];
    __syncthreads();

    float acc[3][TY];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < TY; ++r) acc[i][r] = 0.0f;

#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // one filter pass at a time: keeps the three passes' loads from piling up in registers
        __builtin_amdgcn_sched_barrier(0);
        // unnormalised x-filter m_i of low at this column
        float hh[HR];
#pragma unroll
        for (int q = 0; q < HR; ++q) {
            const float a = L[q * LW + c], b = L[q * LW + c + D], e = L[q * LW + c + 2 * D];
            if (i == 0) hh[q] = fmaf(2.0f, b, a + e);
            else if (i == 1) hh[q] = e - a;
            else hh[q] = fmaf(2.0f, b, -(a + e));
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const bool from_above = SIN && i == 0 && j == 0;  // folds once the loops unroll
            const float m = cf.thr[i][j];
            float col[BR];
#pragma unroll
            for (int q = 0; q < BR; ++q) {
                if (from_above) {
                    col[q] = sc[q];
                } else {
                    const float a = hh[q], b = hh[q + D], e = hh[q + 2 * D];
                    float v;
                    if (j == 0) v = fmaf(2.0f, b, a + e);
                    else if (j == 1) v = e - a;
                    else v = fmaf(2.0f, b, -(a + e));
                    col[q] = v - __builtin_amdgcn_fmed3f(v, -m, m);
                }
            }
            const float f = cf.wgt[i][j];
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                const float wm = col[r], w0 = col[r + D], wp = col[r + 2 * D];  // y-d, y, y+d
                float t;
                if (j == 0) t = fmaf(2.0f, w0, wp + wm);
                else if (j == 1) t = wm - wp;
                else t = fmaf(2.0f, w0, -(wp + wm));
                acc[i][r] = fmaf(f, t, acc[i][r]);
            }
        }
    }
    __syncthreads();  // the low-pass tile is no longer read
    float* ys = lds;  // [2][TY][kBlock]: the terms read from x + d, from x - d
    float mid[TY];
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        const float dlt = acc[0][r] - acc[2][r];
        ys[r * kBlock + c] = dlt + acc[1][r];
        ys[(TY + r) * kBlock + c] = dlt - acc[1][r];
        mid[r] = acc[0][r] + acc[2][r];
    }
    __syncthreads();

    if (c < D || c >= kBlock - D) return;
    const int x = x0 + c - D;
    if (x >= N) return;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        const int y = y0 + r;
        if (y >= N) break;
        out[(size_t)y * N + x] = fmaf(2.0f, mid[r], ys[r * kBlock + c - D] + ys[(TY + r) * kBlock + c + D]);
    }
}

// rows per strip of the shrink-synthesis of dilation D
template <int D>
constexpr int ss_rows() { return 8; }

template <int D, bool SIN>
__global__ __launch_bounds__(kBlock) void shrink_synthesis_kernel(const float* __restrict__ low,
                                                                  const float* __restrict__ s_in, int N,
                                                                  float* __restrict__ out, SsCoef cf) {
    __shared__ float lds[SsTile<D, ss_rows<D>()>::LDS_FLOATS];
    int bx, by;
    xcd_tile(&bx, &by);  // each XCD takes a band of strips: the row halos stay in its L2
    shrink_synthesis_tile<D, ss_rows<D>(), SIN>(low, s_in, N, out, cf, bx, by, lds);
}

hipError_t launch_lowpass_level(const float* v, int N, int d, float* out, hipStream_t s) {
    dim3 grid((N + kBlock - 1) / kBlock, (N + AN_TY - 1) / AN_TY);
    switch (d) {
        case 1: hipLaunchKernelGGL(lowpass_level_kernel<1>, grid, dim3(kBlock), 0, s, v, N, out); break;
        case 2: hipLaunchKernelGGL(lowpass_level_kernel<2>, grid, dim3(kBlock), 0, s, v, N, out); break;
        case 4: hipLaunchKernelGGL(lowpass_level_kernel<4>, grid, dim3(kBlock), 0, s, v, N, out); break;
        case 8: hipLaunchKernelGGL(lowpass_level_kernel<8>, grid, dim3(kBlock), 0, s, v, N, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

SsCoef ss_coef(const LevelMu& mu, float delta, bool from_above) {
    const double cs[3] = {0.25, 0.35355339059327376, 0.25};  // c_i of b_i = c_i m_i
    SsCoef cf;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double cc = cs[i] * cs[j];
            const double m = (i == 0 && j == 0) ? mu.low : mu.band[pair_slot(i, j)];
            cf.thr[i][j] = (float)(m / cc);
            cf.wgt[i][j] = (float)(delta * cc * cc);
        }
    if (from_above) cf.wgt[0][0] = 0.0625f;  // c_0^2: the level above's output enters unthresholded
    return cf;
}

template <int D>
static hipError_t launch_ss(const float* low, const float* s_in, int N, float* out, LevelMu mu, float delta,
                            hipStream_t s) {
    constexpr int IW = kBlock - 2 * D;
    constexpr int TY = ss_rows<D>();
    const SsCoef cf = ss_coef(mu, delta, s_in != nullptr);
    dim3 grid((N + IW - 1) / IW, (N + TY - 1) / TY);
    if (s_in)
        hipLaunchKernelGGL((shrink_synthesis_kernel<D, true>), grid, dim3(kBlock), 0, s, low, s_in, N, out, cf);
    else
        hipLaunchKernelGGL((shrink_synthesis_kernel<D, false>), grid, dim3(kBlock), 0, s, low, s_in, N, out, cf);
    return hipGetLastError();
}

// ---- batched implicit state --------------------------------------------
// The tiles of many images per launch (workgroup -> image bmap[b], local tile
// b - bfirst[image]), each running the single-image tile body on its image's
// buffers, so that every image gets exactly its own plan's arithmetic.

int lowpass_level_tiles(int N) { return ((N + kBlock - 1) / kBlock) * ((N + AN_TY - 1) / AN_TY); }

int shrink_level_tiles(int N, int d) {
    const int iw = kBlock - 2 * d;
    return ((N + iw - 1) / iw) * ((N + 8 - 1) / 8);
}

// low_lev = (b0 x b0) low_{lev-1}, low_0 = omega (the state z)
template <int D>
__global__ __launch_bounds__(kBlock) void lowpass_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                 const int* __restrict__ bmap,
                                                                 const int* __restrict__ bfirst, int lev) {
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const float* in = lev == 1 ? I.zin : I.lows[lev - 2];
    const int gx = (I.N + kBlock - 1) / kBlock;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    lowpass_tile<D>(in, I.N, I.lows[lev - 1], local - by * gx, by);
}

hipError_t launch_lowpass_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int lev,
                                  int d, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (d) {
        case 1: hipLaunchKernelGGL(lowpass_batched_kernel<1>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        case 2: hipLaunchKernelGGL(lowpass_batched_kernel<2>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        case 4: hipLaunchKernelGGL(lowpass_batched_kernel<4>, dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap, bfirst, lev); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Level lev of W^T(delta S_mu(W omega)) as the single-image sequence runs it:
// the bands of low_{lev-1} (omega at level 1), the level above's output
// (tmp[(lev + 1) & 1]) below the top, the output to tmp[lev & 1], or at level 1
// to u (f for the final image).
template <int D, bool SIN>
__global__ __launch_bounds__(kBlock) void shrink_synthesis_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                          const int* __restrict__ bmap,
                                                                          const int* __restrict__ bfirst, int lev,
                                                                          int final_out) {
    constexpr int TY = ss_rows<D>();
    __shared__ float lds[SsTile<D, TY>::LDS_FLOATS];
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const float* low = lev == 1 ? I.zin : I.lows[lev - 2];
    const float* s_in = SIN ? (((lev + 1) & 1) ? I.tmp1 : I.tmp0) : nullptr;
    float* out = lev == 1 ? (final_out ? I.f : I.u) : ((lev & 1) ? I.tmp1 : I.tmp0);
    const int gx = (I.N + SsTile<D, TY>::IW - 1) / SsTile<D, TY>::IW;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    shrink_synthesis_tile<D, TY, SIN>(low, s_in, I.N, out, I.ss[lev - 1], local - by * gx, by, lds);
}

template <int D>
static hipError_t launch_ssb(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int lev,
                             int top, int final_out, hipStream_t s) {
    if (top)
        hipLaunchKernelGGL((shrink_synthesis_batched_kernel<D, false>), dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap,
                           bfirst, lev, final_out);
    else
        hipLaunchKernelGGL((shrink_synthesis_batched_kernel<D, true>), dim3(nblocks), dim3(kBlock), 0, s, imgs, bmap,
                           bfirst, lev, final_out);
    return hipGetLastError();
}

hipError_t launch_shrink_synthesis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                           int lev, int d, int top, int final_out, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (d) {
        case 1: return launch_ssb<1>(imgs, bmap, bfirst, nblocks, lev, top, final_out, s);
        case 2: return launch_ssb<2>(imgs, bmap, bfirst, nblocks, lev, top, final_out, s);
        case 4: return launch_ssb<4>(imgs, bmap, bfirst, nblocks, lev, top, final_out, s);
        case 8: return launch_ssb<8>(imgs, bmap, bfirst, nblocks, lev, top, final_out, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_shrink_synthesis_level(const float* low, const float* s_in, int N, int d, float* out,
                                         LevelMu mu, float delta, hipStream_t s) {
    switch (d) {
        case 1: return launch_ss<1>(low, s_in, N, out, mu, delta, s);
        case 2: return launch_ss<2>(low, s_in, N, out, mu, delta, s);
        case 4: return launch_ss<4>(low, s_in, N, out, mu, delta, s);
        case 8: return launch_ss<8>(low, s_in, N, out, mu, delta, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mlba
