// Kernels of the reverse sweep through K unrolled iterations of eq. (MLBA2)
// (rectangular blur of section 2.1, BCCB preconditioner of Algorithm 1) that
// have no forward counterpart:
//
//  * the PSF correlations: A u = sum_{a,q} H[a][q] u[. + p-1-a][. + p-1-q]
//    is linear in H, so d<y, A u>/dH[a][q] is the correlation of y with u at
//    lag (a, q).  Each step contributes corr(W^T zbar, t_k) - corr(u_k, rbar);
//  * the observation gradient (sum of the rbar) and the alpha gradient
//    (-<rbar, t_k>, from dP/dalpha = -P^2);
//  * the spectral term through P: with E = sum_k Re(conj(F rbar) F t_k) / n^2
//    (accumulated inside the preconditioner's column pass) and Lambda the
//    DFT of the zero-padded PSF, the derivative of |Lambda|^2 gives
//    -2 Re sum E conj(Lambda) e^{-2 pi i (ua + vq)/n}, which equals
//    -2 sum_{a',q'} H[a'][q'] e[(a'-a) mod n][(q'-q) mod n] with e the
//    (real, even) inverse transform of E;
//  * the final fixed-order reduction of every running partial.
//
// Running partials: every launch of a phase uses the same workgroup -> tile
// map, so workgroup b adds its tile's contribution to slot b at each step; the
// sums are therefore deterministic.
#include "common.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int PC_TY = 32;  // output rows per tile
constexpr int PC_TX = 64;  // output columns per tile
constexpr int PC_RB = 8;   // lags q per thread item
constexpr int PC_XC = 8;   // columns per register segment

struct CorrShape {
    int p, nch, padl, wr, wc, lsw, items, yg;
};

__host__ __device__ inline CorrShape corr_shape(int p) {
    CorrShape c;
    c.p = p;
    c.nch = (p + PC_RB - 1) / PC_RB;
    c.padl = c.nch * PC_RB - p;
    c.wr = PC_TY + p - 1;
    c.wc = PC_TX + p - 1 + c.padl;
    c.lsw = c.wc | 1;
    c.items = p * c.nch;
    c.yg = c.items >= kBlock ? 1 : kBlock / c.items;
    return c;
}

static size_t corr_lds_floats(int p) {
    const CorrShape c = corr_shape(p);
    const size_t win = 2 * (size_t)c.wr * c.lsw + 2 * PC_TY * PC_TX;
    const size_t red = (size_t)c.yg * p * p;
    return win > red ? win : red;
}

int psf_corr_tiles(const BatchImage& I) {
    return ((I.n + PC_TX - 1) / PC_TX) * ((I.n + PC_TY - 1) / PC_TY);
}

__global__ __launch_bounds__(kBlock) void psf_corr_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                  const int* __restrict__ bmap,
                                                                  const int* __restrict__ bfirst, int first,
                                                                  double* __restrict__ part,
                                                                  double* __restrict__ apart) {
    extern __shared__ float smem[];
    __shared__ double red[kBlock / 64];
    const int xb = xcd_block(blockIdx.x, gridDim.x);  // adjacent tiles of an image in one L2
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const int n = I.n, N = I.N, p = I.p;
    const CorrShape cs = corr_shape(p);
    const int gx = (n + PC_TX - 1) / PC_TX;
    const int local = xb - bfirst[im];
    const int by = local / gx;
    const int oy0 = by * PC_TY, ox0 = (local - by * gx) * PC_TX;

    float* Wl = smem;                    // W^T zbar window
    float* Ul = Wl + cs.wr * cs.lsw;     // u_k window
    float* Tl = Ul + cs.wr * cs.lsw;     // t_k tile
    float* Rl = Tl + PC_TY * PC_TX;      // rbar tile
    const float* wbar = I.u;
    const float* uk = I.uk;
    for (int idx = threadIdx.x; idx < cs.wr * cs.wc; idx += kBlock) {
        const int ly = idx / cs.wc, lx = idx - ly * cs.wc;
        const int y = oy0 + ly, x = ox0 + lx - cs.padl;
        const bool in = y < N && x >= 0 && x < N;
        const size_t o = (size_t)y * N + x;
        Wl[ly * cs.lsw + lx] = in ? wbar[o] : 0.0f;
        Ul[ly * cs.lsw + lx] = in ? uk[o] : 0.0f;
    }
    double dot = 0.0;
    for (int idx = threadIdx.x; idx < PC_TY * PC_TX; idx += kBlock) {
        const int ly = idx / PC_TX, lx = idx - ly * PC_TX;
        const int y = oy0 + ly, x = ox0 + lx;
        float tv = 0.0f, rv = 0.0f;
        if (y < n && x < n) {
            const size_t o = (size_t)y * n + x;
            tv = I.tk[o];
            rv = I.t[o];
            if (I.dg) I.dg[o] = first ? rv : I.dg[o] + rv;
            dot += (double)rv * (double)tv;
        }
        Tl[idx] = tv;
        Rl[idx] = rv;
    }
    __syncthreads();

    // thread item (a, chunk) accumulates lags q = chunk*8 + i over rows yg, yg+YG, ...
    float acc[PC_RB];
    int a_it = -1, c_it = 0, yg_it = 0;
    const int total = cs.items * cs.yg;
    // more than one item per thread only when items >= kBlock (then yg == 1)
    for (int it = threadIdx.x; it < total; it += kBlock) {
        const int item = it % cs.items;
        const int yg = it / cs.items;
        const int a = item / cs.nch, ch = item - (item / cs.nch) * cs.nch;
#pragma unroll
        for (int i = 0; i < PC_RB; ++i) acc[i] = 0.0f;
        for (int yl = yg; yl < PC_TY; yl += cs.yg) {
            const float* wrow = Wl + (yl + p - 1 - a) * cs.lsw;
            const float* urow = Ul + (yl + p - 1 - a) * cs.lsw;
            const float* trow = Tl + yl * PC_TX;
            const float* rrow = Rl + yl * PC_TX;
            const int sbase = p - 1 - ch * PC_RB - (PC_RB - 1) + cs.padl;
            for (int x0 = 0; x0 < PC_TX; x0 += PC_XC) {
                float tv[PC_XC], rv[PC_XC], ws[PC_XC + PC_RB - 1], us[PC_XC + PC_RB - 1];
#pragma unroll
                for (int k = 0; k < PC_XC; ++k) {
                    tv[k] = trow[x0 + k];
                    rv[k] = rrow[x0 + k];
                }
#pragma unroll
                for (int k = 0; k < PC_XC + PC_RB - 1; ++k) {
                    ws[k] = wrow[sbase + x0 + k];
                    us[k] = urow[sbase + x0 + k];
                }
#pragma unroll
                for (int xi = 0; xi < PC_XC; ++xi)
#pragma unroll
                    for (int i = 0; i < PC_RB; ++i) {
                        acc[i] = fmaf(tv[xi], ws[xi + PC_RB - 1 - i], acc[i]);
                        acc[i] = fmaf(-rv[xi], us[xi + PC_RB - 1 - i], acc[i]);
                    }
            }
        }
        if (cs.items >= kBlock) {
            // one row group: write straight to the running partial
            for (int i = 0; i < PC_RB; ++i) {
                const int q = ch * PC_RB + i;
                if (q < p) part[(size_t)blockIdx.x * p * p + a * p + q] += (double)acc[i];
            }
        } else {
            a_it = a;
            c_it = ch;
            yg_it = yg;
        }
    }
    if (cs.items < kBlock) {
        __syncthreads();  // the windows are no longer read: reuse LDS for the row-group sums
        float* rs = smem;  // [yg][p*p]
        if (a_it >= 0)
            for (int i = 0; i < PC_RB; ++i) {
                const int q = c_it * PC_RB + i;
                if (q < p) rs[yg_it * p * p + a_it * p + q] = acc[i];
            }
        __syncthreads();
        for (int l = threadIdx.x; l < p * p; l += kBlock) {
            float s = 0.0f;
            for (int g = 0; g < cs.yg; ++g) s += rs[g * p * p + l];
            part[(size_t)blockIdx.x * p * p + l] += (double)s;
        }
    }
    const double d = block_sum(dot, red);
    if (threadIdx.x == 0) apart[blockIdx.x] -= d;
}

hipError_t launch_psf_corr_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int p,
                                   int first, double* part, double* apart, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    const size_t lds = corr_lds_floats(p) * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(psf_corr_batched_kernel, dim3(nblocks), dim3(kBlock), lds, s, imgs, bmap, bfirst, first,
                       part, apart);
    return hipGetLastError();
}

// One workgroup per image; e = I.t holds the inverse transform of E / n^2.
__global__ __launch_bounds__(kBlock) void psf_spectral_kernel(const BatchImage* __restrict__ imgs, int p,
                                                              double* __restrict__ spec) {
    const BatchImage& I = imgs[blockIdx.x];
    const int n = I.n;
    const float* e = I.t;
    const float* H = I.psf;
    const double scale = -2.0 * (double)n * (double)n;
    for (int l = threadIdx.x; l < p * p; l += kBlock) {
        const int a = l / p, q = l - (l / p) * p;
        double s = 0.0;
        for (int a2 = 0; a2 < p; ++a2) {
            const float* erow = e + (size_t)mod_pos(a2 - a, n) * n;
            for (int q2 = 0; q2 < p; ++q2) s += (double)H[a2 * p + q2] * (double)erow[mod_pos(q2 - q, n)];
        }
        spec[(size_t)blockIdx.x * p * p + l] = scale * s;
    }
}

hipError_t launch_psf_spectral_batched(const BatchImage* imgs, int count, int p, double* spec, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(psf_spectral_kernel, dim3(count), dim3(kBlock), 0, s, imgs, p, spec);
    return hipGetLastError();
}

// Workgroup o reduces output o: o < bands -> dmu[o]; o == bands -> dalpha;
// o > bands -> dpsf[o - bands - 1].  Sums in a fixed order.
__global__ __launch_bounds__(kBlock) void unrolled_reduce_kernel(UnrolledSums S, double* __restrict__ dmu,
                                                                 double* __restrict__ dalpha,
                                                                 double* __restrict__ dpsf) {
    __shared__ double red[kBlock / 64];
    const int o = blockIdx.x;
    double s = 0.0;
    if (o < S.bands) {
        const int lev = o == 0 ? S.levels : (o - 1) / 8 + 1;
        const int slot = o == 0 ? 8 : (o - 1) % 8;
        const double* pl = S.mu_part[lev - 1];
        for (int b = threadIdx.x; b < S.mu_blocks[lev - 1]; b += kBlock) s += pl[(size_t)b * 9 + slot];
    } else if (o == S.bands) {
        for (int b = threadIdx.x; b < S.corr_blocks; b += kBlock) s += S.alpha_part[b];
    } else {
        const int l = o - S.bands - 1;
        const int pp = S.p * S.p;
        for (int b = threadIdx.x; b < S.corr_blocks; b += kBlock) s += S.corr_part[(size_t)b * pp + l];
        for (int i = threadIdx.x; i < S.count; i += kBlock) s += S.spec[(size_t)i * pp + l];
    }
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (o < S.bands) dmu[o] = t;
        else if (o == S.bands) *dalpha = t;
        else dpsf[o - S.bands - 1] = t;
    }
}

hipError_t launch_unrolled_reduce(const UnrolledSums& S, double* dmu, double* dalpha, double* dpsf, hipStream_t s) {
    const int outs = S.bands + 1 + S.p * S.p;
    hipLaunchKernelGGL(unrolled_reduce_kernel, dim3(outs), dim3(kBlock), 0, s, S, dmu, dalpha, dpsf);
    return hipGetLastError();
}

}  // namespace mlba
