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
#include "kernels.hpp"

namespace mlba {

constexpr int FR_TY = 8;
constexpr float kB1 = 0.35355339059327376f;  // sqrt(2) / 4

// pair (i, j) != (0, 0) -> position in the level's band block
__host__ __device__ constexpr int pair_slot(int i, int j) { return i * 3 + j - 1; }

// Analysis of one level: one thread per column, AN_TY rows per thread.  The
// x-direction filters read the two neighbouring columns straight from memory
// (cache hits); every old coefficient of the strip is loaded before the first
// store so that 9 * AN_TY independent loads are in flight per thread.
constexpr int AN_TY = 8;

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

// low_out = (b0 x b0) v with dilation D: the (0,0) band of analysis_tile
template <int D>
__global__ __launch_bounds__(kBlock) void lowpass_level_kernel(const float* __restrict__ v, int N,
                                                               float* __restrict__ out) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const int y0 = blockIdx.y * AN_TY;
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
    static constexpr int YS_FLOATS = 3 * TY * kBlock;
    static constexpr int LDS_FLOATS = LOW_FLOATS > YS_FLOATS ? LOW_FLOATS : YS_FLOATS;
};

// The low-pass tile is staged in LDS once (coalesced rows, reflected
// indices); each thread then filters its extended column from LDS.  The LDS
// is reused for the three x-synthesis inputs after the last x-filter.
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
// synthesis weight (computed on the host).
struct SsCoef {
    float thr[3][3];
    float wgt[3][3];
};

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
#pragma unroll
    for (int k0 = 0; k0 < LW; k0 += kBlock) {
        const int k = k0 + c;
        if (k0 + kBlock <= LW || k < LW) {
            const int col = reflect_index(x0 - 2 * D + k, N);
            float v[HR];
#pragma unroll
            for (int q = 0; q < HR; ++q) v[q] = low[rowo[q] + col];
#pragma unroll
            for (int q = 0; q < HR; ++q) L[q * LW + k] = v[q];
        }
    }
    float sc[BR];
    if constexpr (SIN) {
        const int xm = reflect_index(xe, N);
#pragma unroll
        for (int q = 0; q < BR; ++q) sc[q] = s_in[rowo[q + D] + xm];
    }
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
    float* ys = lds;  // [3][TY][kBlock]
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int r = 0; r < TY; ++r) ys[(i * TY + r) * kBlock + c] = acc[i][r];
    __syncthreads();

    if (c < D || c >= kBlock - D) return;
    const int x = x0 + c - D;
    if (x >= N) return;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        const int y = y0 + r;
        if (y >= N) break;
        const float* y0r = ys + (0 * TY + r) * kBlock;
        const float* y1r = ys + (1 * TY + r) * kBlock;
        const float* y2r = ys + (2 * TY + r) * kBlock;
        float sum = fmaf(2.0f, y0r[c], y0r[c + D] + y0r[c - D]);
        sum += y1r[c - D] - y1r[c + D];
        sum += fmaf(2.0f, y2r[c], -(y2r[c + D] + y2r[c - D]));
        out[(size_t)y * N + x] = sum;
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

template <int D>
static hipError_t launch_ss(const float* low, const float* s_in, int N, float* out, LevelMu mu, float delta,
                            hipStream_t s) {
    constexpr int IW = kBlock - 2 * D;
    constexpr int TY = ss_rows<D>();
    const double cs[3] = {0.25, 0.35355339059327376, 0.25};  // c_i of b_i = c_i m_i
    SsCoef cf;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double cc = cs[i] * cs[j];
            const double m = (i == 0 && j == 0) ? mu.low : mu.band[pair_slot(i, j)];
            cf.thr[i][j] = (float)(m / cc);
            cf.wgt[i][j] = (float)(delta * cc * cc);
        }
    dim3 grid((N + IW - 1) / IW, (N + TY - 1) / TY);
    if (s_in) {
        cf.wgt[0][0] = 0.0625f;  // c_0^2: the level above's output enters unthresholded
        hipLaunchKernelGGL((shrink_synthesis_kernel<D, true>), grid, dim3(kBlock), 0, s, low, s_in, N, out, cf);
    } else {
        hipLaunchKernelGGL((shrink_synthesis_kernel<D, false>), grid, dim3(kBlock), 0, s, low, s_in, N, out, cf);
    }
    return hipGetLastError();
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
    const int im = bmap[blockIdx.x];
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
    const int local = blockIdx.x - bfirst[im];
    const int by = local / gx;
    synthesis_tile<D>(zlev, low, I.N, out, mu, thr ? I.delta : 1.0f, (thr && top) ? 1 : 0, thr, local - by * gx,
                      by, ys);
}

template <int D>
__global__ __launch_bounds__(kBlock) void analysis_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                  const int* __restrict__ bmap,
                                                                  const int* __restrict__ bfirst, int lev) {
    const int im = bmap[blockIdx.x];
    const BatchImage& I = imgs[im];
    const size_t nn = (size_t)I.N * I.N;
    const float* in = lev == 1 ? I.w : (((lev - 1) & 1) ? I.tmp1 : I.tmp0);
    const bool last = lev == I.levels;
    float* low = last ? I.z : ((lev & 1) ? I.tmp1 : I.tmp0);
    float* zlev = I.z + (size_t)(1 + 8 * (lev - 1)) * nn;
    const float* zin_lev = I.zin + (size_t)(1 + 8 * (lev - 1)) * nn;
    const int gx = (I.N + kBlock - 1) / kBlock;
    const int local = blockIdx.x - bfirst[im];
    const int by = local / gx;
    analysis_tile<D>(in, I.N, zin_lev, last ? I.zin : low, zlev, low, 1, last ? 1 : 0, local - by * gx, by);
}

template <int D>
__global__ __launch_bounds__(kBlock) void analysis_adjoint_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                          const int* __restrict__ bmap,
                                                                          const int* __restrict__ bfirst, int lev,
                                                                          int init, double* __restrict__ part) {
    __shared__ double red[9][kBlock / 64];
    const int im = bmap[blockIdx.x];
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
    const int local = blockIdx.x - bfirst[im];
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
    const size_t count = (size_t)I.bands * I.N * I.N;
    return (int)((count + FILL_CHUNK - 1) / FILL_CHUNK);
}

__global__ __launch_bounds__(kBlock) void fill_batched_kernel(const BatchImage* __restrict__ imgs,
                                                              const int* __restrict__ bmap,
                                                              const int* __restrict__ bfirst) {
    const int im = bmap[blockIdx.x];
    const BatchImage& I = imgs[im];
    const size_t count = (size_t)I.bands * I.N * I.N;
    const size_t beg = (size_t)(blockIdx.x - bfirst[im]) * FILL_CHUNK;
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
