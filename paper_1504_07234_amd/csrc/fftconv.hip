// The blur of the rectangular model by FFTs (section 2.1: A and A^T computed
// with FFTs of a grid that holds the whole unknown), an alternative to the
// direct convolution for large PSFs.
//
// On an M x M grid (M >= N = n + p - 1, M = 2^a 3^b) the circular convolution
// with H (placed at the origin) has no wrap-around on the outputs that matter:
//   A u   = crop_{[p-1, N)^2} F^{-1}[ F(pad u) * F(pad H) ] / M^2
//   A^T t = crop_{[0, N)^2}   F^{-1}[ F(t placed at (p-1, p-1)) * conj(F(pad H)) ] / M^2
// (the second is the circular correlation, the transpose of the first).
//
// Three passes like the preconditioner: rows (two real rows packed into one
// complex FFT, written transposed as a half spectrum), columns (forward FFT,
// product with the PSF spectrum, inverse FFT), rows (inverse, with the crop
// and the epilogue: residual g - . with its squared-norm partials, plain
// write, or accumulation).  Rows that are zero in the padded input are skipped
// by the row pass and read as zero by the column pass.  Transforms of up to
// 3072 points use 12 values per thread.
#include "artrans.hpp"
#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"

namespace mlba {

// Makhoul's DCT through an n-point FFT (as the DCT plan's row passes):
// sample l goes to position dct_perm(l) (evens ascending, odds descending).
__device__ __forceinline__ int fc_dct_perm(int l, int n) { return (l & 1) ? n - 1 - (l >> 1) : (l >> 1); }
__device__ __forceinline__ float fc_re_mul(float2 w, float2 v) { return w.x * v.x - w.y * v.y; }

constexpr int FC_EPT = 12;
constexpr int FC_MAX = FC_EPT * kBlock;

int fftconv_max_size() { return FC_MAX; }

// Sequences per workgroup: more than one only while the grid still gives at
// least 512 workgroups (two per CU), so that small grids hide the latency of
// their LDS phases with several resident workgroups.
static int fc_pairs_per_block(int M) {
    int G = 1;
    while ((G * 2) * M <= FC_MAX && ((M / 2) % (G * 2)) == 0 && G * 2 <= 4 && M / 2 / (G * 2) >= 512) G *= 2;
    return G;
}

static int fc_cols_per_block(int M) {
    int cc = 1;
    while ((cc * 2) * M <= FC_MAX && (M / 2 + 1) / (cc * 2) >= 512) cc *= 2;
    return cc;
}

static int fc_seq_shift(int batch) {
    int sh = 8;
    while (batch > 1) {
        batch >>= 1;
        --sh;
    }
    return sh;
}

// Rows pass: row pairs pair0 + blk*G + g of the M grid; entry (Y, X) is
// src[Y - off][X - off] inside the S x S box at (off, off), else 0.  With an
// extension `ext` other than EXT_ZERO, the box is widened by off on every
// side and holds the source's extension there (Table 1 and section 2.2: the
// reflective, periodic or antireflective pad): the grid then carries
// E src E^T.  NT > 0: M == NT and G == 1.
// DIR (Algorithm 2's PCG): the source is the direction d, first updated in
// place to d = z + b d with b = rho_new / rho (nothing once the CG has
// stopped), as the separate direction kernel does; rho_new null: d = z.
// GT > 1 (compiled length only): GT row pairs per workgroup of GT x kBlock
// threads, each pair transformed by its own kBlock threads in its own LDS
// slice; the transposed half spectrum is then written with the GT pairs of
// one frequency next to each other (16 GT contiguous bytes per frequency
// instead of 16).
template <int NT, bool DIR = false, int GT = 1>
__global__ __launch_bounds__(kBlock * GT) void fc_rows_fwd_kernel(const float* __restrict__ src, int S, int off, int M_,
                                                                  float2* __restrict__ T, int ts, FftDesc fd,
                                                                  const float2* __restrict__ tw, int G_, int seq_shift,
                                                                  int pair0, int pair_end, int ext, PcgDir dir) {
    static_assert(GT == 1 || NT > 0, "several pairs of kBlock threads: compiled lengths only");
    extern __shared__ float2 lds[];
    const int M = NT > 0 ? NT : M_;
    const int G = NT > 0 ? GT : G_;
    // this thread's pair slice (GT > 1) or the whole workgroup's (GT == 1)
    const int gs = GT > 1 ? (int)threadIdx.x / kBlock : 0;
    const int tid = GT > 1 ? (int)threadIdx.x % kBlock : (int)threadIdx.x;
    constexpr int SL = NT > 0 ? lds_data_slots(NT > 0 ? NT : 1) : 0;
    float2* buf = lds + gs * SL;
    const int pb = pair0 + xcd_block(blockIdx.x, gridDim.x) * G;
    bool dir_on = false, dir_copy = false;
    float dir_b = 0.0f;
    if constexpr (DIR) {
        dir_copy = dir.rho_new == nullptr;  // the first direction: d = z
        dir_on = dir_copy || *dir.act != 0.0;
        if (dir_on && !dir_copy) dir_b = (float)(*dir.rho_new / *dir.rho);
    }
    auto rd = [&](size_t i) {
        if constexpr (DIR) {
            if (!dir_on) return src[i];
            const float v = dir_copy ? dir.z[i] : fmaf(dir_b, dir.d[i], dir.z[i]);
            dir.d[i] = v;
            return v;
        } else {
            return src[i];
        }
    };
    // value X of pair q (zero outside the image and past pair_end)
    auto fetch = [&](int q, int X) {
        const int Y = 2 * q;
        const int x = X - off;
        float a = 0.0f, b = 0.0f;
        const int y0 = Y - off, y1 = Y + 1 - off;
        if (ext != EXT_ZERO) {
            if (q < pair_end && x >= -off && x < S + off) {
                if (y0 >= -off && y0 < S + off) a = fetch_ext(src, S, y0, x, ext);
                if (y1 >= -off && y1 < S + off) b = fetch_ext(src, S, y1, x, ext);
            }
        } else if (q < pair_end && x >= 0 && x < S) {
            if (y0 >= 0 && y0 < S) a = rd((size_t)y0 * S + x);
            if (y1 >= 0 && y1 < S) b = rd((size_t)y1 * S + x);
        }
        return make_float2(a, b);
    };
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) {
        fixed_tw_load<NT>(tw, twp.w, tid);
        strided_copy<NT, float2>(
            NT, [&](int X) { return fetch(pb + gs, X); }, [&](int X, float2 v) { buf[lds_slot(X)] = v; }, tid);
        __syncthreads();
        lds_fft_fixed<-1, NT>(buf, tw, twp.w, tid);
    } else {
        strided_copy<NT, float2>(
            G * M,
            [&](int idx) {
                const int g = idx / M;
                return fetch(pb + g, idx - g * M);
            },
            [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
        __syncthreads();
        lds_fft_any<-1, NT, FC_EPT>(buf, fd, G, seq_shift, tw, nullptr);
    }
    const int half = M / 2 + 1;
    for (int idx = threadIdx.x; idx < G * half; idx += kBlock * GT) {
        const int k = idx / G;
        const int g = idx - k * G;
        if (pb + g >= pair_end) continue;
        // compiled length: pair g's slice; run-time plan: the G sequences back to back
        auto at = [&](int e) { return NT > 0 ? lds[g * SL + lds_slot(e)] : lds[lds_slot(g * M + e)]; };
        const float2 Z = at(k);
        const float2 Zc = cconj(at(k == 0 ? 0 : M - k));
        const float2 Xa = cscale(cadd(Z, Zc), 0.5f);
        const float2 D = csub(Z, Zc);
        const float2 Xb = make_float2(0.5f * D.y, -0.5f * D.x);
        *reinterpret_cast<float4*>(T + (size_t)k * ts + 2 * (pb + g)) = make_float4(Xa.x, Xa.y, Xb.x, Xb.y);
    }
}

// The transpose E^T of a square model's extension along one axis: the grid
// positions (0 <= Y < n + 2c) whose extended value is pixel k of the n-point
// axis: k + c itself, and under the reflective or periodic model its copies
// in the pads of width c (p <= n keeps them distinct).
__device__ __forceinline__ int ext_preimages(int k, int n, int c, int ext, int* pre) {
    int cnt = 0;
    pre[cnt++] = k + c;
    if (ext == EXT_REFLECT) {
        if (k < c) pre[cnt++] = c - 1 - k;
        if (k >= n - c) pre[cnt++] = 2 * n - 1 - k + c;
    } else if (ext == EXT_PERIODIC) {
        if (k < c) pre[cnt++] = k + n + c;
        if (k >= n - c) pre[cnt++] = k - n + c;
    }
    return cnt;
}

// Sum of v(Y) over the preimages Y of pixel k (fold < 0: v(k) itself).
template <class F>
__device__ __forceinline__ float2 fold_sum(int k, int n, int c, int fold, F v) {
    if (fold < 0) return v(k);
    int pre[3];
    const int cnt = ext_preimages(k, n, c, fold, pre);
    float2 a = v(pre[0]);
    for (int i = 1; i < cnt; ++i) a = cadd(a, v(pre[i]));
    return a;
}

// The factor of the column pass's product: H (conj_h 0), conj(H) (1) or
// |H|^2 (2: A A^T of the rectangular model in one transform pair).
__device__ __forceinline__ float2 spectrum_factor(float2 h, int conj_h) {
    if (conj_h == 2) return make_float2(h.x * h.x + h.y * h.y, 0.0f);
    return conj_h ? cconj(h) : h;
}

// Columns pass over CC half-spectrum rows per workgroup; rows outside
// [y_lo, y_hi) of the input are zero.  mode 0: forward FFT, times Hs (or
// conj(Hs)) * inv, inverse FFT, written back for the rows [o_lo, o_hi) that the
// inverse row pass reads; mode 1: forward FFT into cspec.  With fold >= 0
// (a square model's extension, n-point image, pad c) mode 0 stores instead
// the rows of E^T applied along the columns: row y < n holds the sum over the
// preimages of y, rows [0, n + (n & 1)) are written (an odd n's last one 0).
template <int NT>
__global__ __launch_bounds__(kBlock) void fc_cols_kernel(float2* __restrict__ T, int M_, int ts,
                                                         const float2* __restrict__ Hs, int conj_h, float inv,
                                                         int y_lo, int y_hi, int mode, float2* __restrict__ cspec,
                                                         FftDesc fd, const float2* __restrict__ tw, int CC_,
                                                         int seq_shift, int o_lo, int o_hi, int fold, int fn,
                                                         int fcn) {
    extern __shared__ float2 buf[];
    const int M = NT > 0 ? NT : M_;
    const int CC = NT > 0 ? 1 : CC_;
    const int half = M / 2 + 1;
    const int k0 = blockIdx.x * CC;
    const int cc = min(CC, half - k0);
    const size_t base = (size_t)k0 * M;
    if constexpr (NT > 0 && fixed_conv_ok<(NT > 0 ? NT : 1)>()) {
        if (mode == 0 && fold < 0) {  // the product with the PSF spectrum in registers
            constexpr int SL = fixed_conv_slots<NT>();
            FixedTw<NT> twf;
            FixedTw<NT, true> twi;
            fixed_tw_load<NT>(tw, twf.w);
            fixed_tw_load<NT, 0, true>(tw, twi.w);
            float2 h[SL];
#pragma unroll
            for (int r = 0; r < SL; ++r) {
                const float2 hv = Hs[base + threadIdx.x + r * kBlock];
                h[r] = spectrum_factor(hv, conj_h);
            }
            float2* col = T + (size_t)k0 * ts;
            fixed_conv<NT>(
                buf, tw, twf.w, twi.w,
                [&](int y) { return (y >= y_lo && y < y_hi) ? col[y] : make_float2(0.0f, 0.0f); },
                [&](int r, int, float2 v) { return cscale(cmul(v, h[r]), inv); },
                [&](int y, float2 v) {
                    if (y >= o_lo && y < o_hi) col[y] = v;
                },
                false);
            return;
        }
    }
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        cc * M,
        [&](int idx) {
            const int q = idx / M;
            const int y = idx - q * M;
            return (y >= y_lo && y < y_hi) ? T[(size_t)(k0 + q) * ts + y] : make_float2(0.0f, 0.0f);
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
    // compiled length: the PSF spectrum of the column is loaded with the
    // column, before the transform, and held in registers
    constexpr int HPER = NT > 0 ? (NT + kBlock - 1) / kBlock : 1;
    float2 hreg[HPER];
    if constexpr (NT > 0) {
        if (mode == 0) {
#pragma unroll
            for (int k = 0; k < HPER; ++k) {
                const int e = k * kBlock + (int)threadIdx.x;
                if (NT % kBlock == 0 || e < NT) hreg[k] = Hs[base + e];
            }
        }
    }
    __syncthreads();
    lds_fft_any<-1, NT, FC_EPT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    if (mode == 1) {
        for (int idx = threadIdx.x; idx < cc * M; idx += kBlock) cspec[base + idx] = buf[lds_slot(idx)];
        return;
    }
    if constexpr (NT > 0) {
#pragma unroll
        for (int k = 0; k < HPER; ++k) {
            const int e = k * kBlock + (int)threadIdx.x;
            if (NT % kBlock == 0 || e < NT) {
                const float2 h = spectrum_factor(hreg[k], conj_h);
                buf[lds_slot(e)] = cscale(cmul(buf[lds_slot(e)], h), inv);
            }
        }
    } else {
        for (int idx = threadIdx.x; idx < cc * M; idx += kBlock) {
            float2 h = Hs[base + idx];
            h = spectrum_factor(h, conj_h);
            buf[lds_slot(idx)] = cscale(cmul(buf[lds_slot(idx)], h), inv);
        }
    }
    __syncthreads();
    lds_fft_any<1, NT, FC_EPT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    if (fold >= 0) {
        const int rows = fn + (fn & 1);
        for (int idx = threadIdx.x; idx < cc * rows; idx += kBlock) {
            const int q = idx / rows;
            const int y = idx - q * rows;
            T[(size_t)(k0 + q) * ts + y] =
                y < fn ? fold_sum(y, fn, fcn, fold, [&](int Y) { return buf[lds_slot(q * M + Y)]; })
                       : make_float2(0.0f, 0.0f);
        }
        return;
    }
    for (int idx = threadIdx.x; idx < cc * M; idx += kBlock) {
        const int q = idx / M;
        const int y = idx - q * M;
        if (y >= o_lo && y < o_hi) T[(size_t)(k0 + q) * ts + y] = buf[lds_slot(idx)];
    }
}

// Inverse rows pass over row pairs pair0 + blk*G + g; output (Y, X) of the M
// grid inside [oy, oy + D) x [ox, ox + D) goes to dst[Y - oy][X - ox]:
// g ? g - v (squared-norm partial per workgroup) : (accum ? dst + v : v).
// With fold >= 0 (ox = 0) the value at x is instead the sum over the
// preimages of x under the square model's extension (E^T along the rows, pad
// fcn).  axd (instead of g): dst = v + axa axd with the partials of
// sum axd dst (the PCG product (A A^T + alpha I) d and d . q of Algorithm 2).
template <int NT>
__global__ __launch_bounds__(kBlock) void fc_rows_inv_kernel(const float2* __restrict__ T, int M_, int ts,
                                                             FftDesc fd, const float2* __restrict__ tw, int G_,
                                                             int seq_shift, int pair0, int pair_end, int oy, int ox,
                                                             int D, float* __restrict__ dst,
                                                             const float* __restrict__ g, int accum,
                                                             double* __restrict__ partials, int fold, int fcn,
                                                             const float* __restrict__ axd, float axa) {
    extern __shared__ float2 buf[];
    __shared__ double red[kBlock / 64];
    const int M = NT > 0 ? NT : M_;
    const int G = NT > 0 ? 1 : G_;
    const int pb = pair0 + xcd_block(blockIdx.x, gridDim.x) * G;
    constexpr int HALF_T = NT > 0 ? NT / 2 + 1 : 0;
    const int half = M / 2 + 1;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<HALF_T, float4>(
        G * half,
        [&](int idx) {
            const int k = idx / G;
            const int gg = idx - k * G;
            float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (pb + gg < pair_end) q = *reinterpret_cast<const float4*>(T + (size_t)k * ts + 2 * (pb + gg));
            return q;
        },
        [&](int idx, float4 q) {
            const int k = idx / G;
            const int gg = idx - k * G;
            float2 Xa = make_float2(q.x, q.y), Xb = make_float2(q.z, q.w);
            const bool edge = (k == 0) || (2 * k == M);
            if (edge) {
                Xa.y = 0.0f;
                Xb.y = 0.0f;
            }
            buf[lds_slot(gg * M + k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            if (!edge) buf[lds_slot(gg * M + M - k)] = make_float2(Xa.x + Xb.y, -Xa.y + Xb.x);
        });
    // compiled length: the epilogue's operand (g or the accumulated dst) is
    // loaded before the transform, with the spectrum
    constexpr int XPER = NT > 0 ? (NT + kBlock - 1) / kBlock : 1;
    float2 pre[XPER];
    if constexpr (NT > 0) {
        const float* opnd = g ? g : (axd ? axd : (accum ? dst : nullptr));
#pragma unroll
        for (int k = 0; k < XPER; ++k) {
            pre[k] = make_float2(0.0f, 0.0f);
            const int X = k * kBlock + (int)threadIdx.x;
            const int x = X - ox;
            if (opnd && (NT % kBlock == 0 || X < NT) && pb < pair_end && x >= 0 && x < D) {
                const int ya = 2 * pb - oy;
                if (ya >= 0 && ya < D) pre[k].x = opnd[(size_t)ya * D + x];
                if (ya + 1 >= 0 && ya + 1 < D) pre[k].y = opnd[(size_t)(ya + 1) * D + x];
            }
        }
    }
    __syncthreads();
    lds_fft_any<1, NT, FC_EPT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    double ss = 0.0;
    if constexpr (NT > 0) {
#pragma unroll
        for (int k = 0; k < XPER; ++k) {
            const int X = k * kBlock + (int)threadIdx.x;
            const int x = X - ox;
            if ((NT % kBlock != 0 && X >= NT) || pb >= pair_end || x < 0 || x >= D) continue;
            const float2 v = fold_sum(X, D, fcn, fold, [&](int Xs) { return buf[lds_slot(Xs)]; });
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int y = 2 * pb + h - oy;
                if (y < 0 || y >= D) continue;
                const size_t o = (size_t)y * D + x;
                const float p = h == 0 ? pre[k].x : pre[k].y;
                float val = h == 0 ? v.x : v.y;
                if (g) {
                    val = p - val;
                    ss += (double)val * (double)val;
                } else if (axd) {
                    val = fmaf(axa, p, val);
                    ss += (double)p * (double)val;
                } else if (accum) {
                    val = p + val;
                }
                dst[o] = val;
            }
        }
    } else {
        for (int idx = threadIdx.x; idx < G * M; idx += kBlock) {
            const int gg = idx / M;
            const int X = idx - gg * M;
            if (pb + gg >= pair_end) continue;
            const int x = X - ox;
            if (x < 0 || x >= D) continue;
            const float2 v = fold_sum(X, D, fcn, fold, [&](int Xs) { return buf[lds_slot(gg * M + Xs)]; });
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int y = 2 * (pb + gg) + h - oy;
                if (y < 0 || y >= D) continue;
                const size_t o = (size_t)y * D + x;
                float val = h == 0 ? v.x : v.y;
                if (g) {
                    val = g[o] - val;
                    ss += (double)val * (double)val;
                } else if (axd) {
                    const float dv = axd[o];
                    val = fmaf(axa, dv, val);
                    ss += (double)dv * (double)val;
                } else if (accum) {
                    val = dst[o] + val;
                }
                dst[o] = val;
            }
        }
    }
    if (partials) {
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// ---- row passes fused with the preconditioner's ---------------------------
// The residual's inverse row pass (FFT-blur grid) and the preconditioner's
// forward row pass both run over the same two observed rows, so one
// workgroup does both: inverse transform of the grid pair, crop and residual
// (with its squared-norm partial), then the forward transform of the two
// residual rows, split and written transposed into the preconditioner's half
// spectrum.  The arithmetic of every value is that of the separate passes.
template <int NTM, int NTN, bool DCT = false>
__global__ __launch_bounds__(kBlock) void fc_residual_precond_kernel(
    const float2* __restrict__ Tc, int M_, int tsc, FftDesc fdm, const float2* __restrict__ twm, int pair0, int n_,
    int off, const float* __restrict__ g, float* __restrict__ r_out, double* __restrict__ partials,
    float2* __restrict__ Tp, int tsp, FftDesc fdn, const float2* __restrict__ twn,
    const float2* __restrict__ dtw) {
    extern __shared__ float2 buf[];
    __shared__ double red[kBlock / 64];
    const int M = NTM > 0 ? NTM : M_;
    const int n = NTN > 0 ? NTN : n_;
    const int q = xcd_block(blockIdx.x, gridDim.x);  // observed rows 2q, 2q + 1
    const int pb = pair0 + q;                        // the same rows of the grid
    const int half = M / 2 + 1;
    FixedTw<(NTM > 0 ? NTM : 1)> twpm;
    if constexpr (NTM > 0) fixed_tw_load<NTM>(twm, twpm.w);
    strided_copy<(NTM > 0 ? NTM / 2 + 1 : 0), float4>(
        half, [&](int k) { return *reinterpret_cast<const float4*>(Tc + (size_t)k * tsc + 2 * pb); },
        [&](int k, float4 v) {
            float2 Xa = make_float2(v.x, v.y), Xb = make_float2(v.z, v.w);
            const bool edge = (k == 0) || (2 * k == M);
            if (edge) {
                Xa.y = 0.0f;
                Xb.y = 0.0f;
            }
            buf[lds_slot(k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            if (!edge) buf[lds_slot(M - k)] = make_float2(Xa.x + Xb.y, -Xa.y + Xb.x);
        });
    const size_t ra = (size_t)(2 * q) * n;
    // the observed rows, loaded with the spectrum before the transform
    float2 gp[FC_EPT];
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        gp[j] = make_float2(0.0f, 0.0f);
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) {
            gp[j].x = g[ra + x];
            if (true) gp[j].y = g[ra + n + x];
        }
    }
    __syncthreads();
    lds_fft_any<1, NTM, FC_EPT>(buf, fdm, 1, 8, twm, NTM > 0 ? twpm.w : nullptr);
    FixedTw<(NTN > 0 ? NTN : 1)> twpn;
    if constexpr (NTN > 0) fixed_tw_load<NTN>(twn, twpn.w);
    float2 rr[FC_EPT];
    double ss = 0.0;
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        rr[j] = make_float2(0.0f, 0.0f);
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) {
            const float2 v = buf[lds_slot(X)];
            const float a = gp[j].x - v.x;
            ss += (double)a * (double)a;
            const float b = gp[j].y - v.y;
            ss += (double)b * (double)b;
            rr[j] = make_float2(a, b);
            if (r_out) {
                r_out[ra + x] = a;
                r_out[ra + n + x] = b;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) buf[lds_slot(DCT ? fc_dct_perm(x, n) : x)] = rr[j];
    }
    __syncthreads();
    lds_fft_any<-1, NTN, FFT_EPT>(buf, fdn, 1, 8, twn, NTN > 0 ? twpn.w : nullptr);
    if constexpr (DCT) {  // DCT-II of the two rows, written transposed as the DCT row pass does
        float* Tr = reinterpret_cast<float*>(Tp);
        for (int k = threadIdx.x; k < n; k += kBlock) {
            const float2 Z = buf[lds_slot(k)];
            const float2 Zc = cconj(buf[lds_slot(k == 0 ? 0 : n - k)]);
            const float2 Va = cscale(cadd(Z, Zc), 0.5f);
            const float2 D = csub(Z, Zc);
            const float2 Vb = make_float2(0.5f * D.y, -0.5f * D.x);
            const float2 w = dtw[k];
            *reinterpret_cast<float2*>(Tr + (size_t)k * tsp + 2 * q) = make_float2(fc_re_mul(w, Va), fc_re_mul(w, Vb));
        }
    } else {
        const int hn = n / 2 + 1;
        for (int k = threadIdx.x; k < hn; k += kBlock) {
            const float2 Z = buf[lds_slot(k)];
            const float2 Zc = cconj(buf[lds_slot(k == 0 ? 0 : n - k)]);
            const float2 Xa = cscale(cadd(Z, Zc), 0.5f);
            const float2 D = csub(Z, Zc);
            const float2 Xb = make_float2(0.5f * D.y, -0.5f * D.x);  // D / (2i)
            *reinterpret_cast<float4*>(Tp + (size_t)k * tsp + 2 * q) = make_float4(Xa.x, Xa.y, Xb.x, Xb.y);
        }
    }
    if (partials) {
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// The residual's inverse row pass on the FFT-blur grid (observed rows 2q and
// 2q + 1; the second is absent for the last pair of an odd n) and the forward
// row pass of the antireflective transform of those residual rows, in one
// workgroup: inverse M-point row FFT, crop, g - . with the squared-norm
// partial, then the odd extension of the detrended rows and its L-point FFT
// (L = 2(n-1)), written transposed into Tr like ar_rows_fwd_body.
template <int NTM, int NTL>
__global__ __launch_bounds__(kBlock) void fc_residual_ar_kernel(
    const float2* __restrict__ Tc, int M_, int tsc, FftDesc fdm, const float2* __restrict__ twm, int pair0, int n,
    int off, const float* __restrict__ g, double* __restrict__ partials, float* __restrict__ Tr, int tsr,
    FftDesc fdl, const float2* __restrict__ twl) {
    extern __shared__ float2 buf[];
    __shared__ double red[kBlock / 64];
    __shared__ float2 ends[2];  // (r_a, r_b) at x = 0 and x = n - 1
    const int M = NTM > 0 ? NTM : M_;
    const int N = n - 1, L = NTL > 0 ? NTL : 2 * N;
    const float invN = 1.0f / (float)N;
    const int q = xcd_block(blockIdx.x, gridDim.x);
    const int pb = pair0 + q;
    const bool has_b = 2 * q + 1 < n;
    const int half = M / 2 + 1;
    FixedTw<(NTM > 0 ? NTM : 1)> twpm;
    if constexpr (NTM > 0) fixed_tw_load<NTM>(twm, twpm.w);
    strided_copy<(NTM > 0 ? NTM / 2 + 1 : 0), float4>(
        half, [&](int k) { return *reinterpret_cast<const float4*>(Tc + (size_t)k * tsc + 2 * pb); },
        [&](int k, float4 v) {
            float2 Xa = make_float2(v.x, v.y), Xb = make_float2(v.z, v.w);
            const bool edge = (k == 0) || (2 * k == M);
            if (edge) {
                Xa.y = 0.0f;
                Xb.y = 0.0f;
            }
            buf[lds_slot(k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            if (!edge) buf[lds_slot(M - k)] = make_float2(Xa.x + Xb.y, -Xa.y + Xb.x);
        });
    const size_t ra = (size_t)(2 * q) * n;
    // the observed rows, loaded with the spectrum before the transform
    float2 gp[FC_EPT];
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        gp[j] = make_float2(0.0f, 0.0f);
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) {
            gp[j].x = g[ra + x];
            if (has_b) gp[j].y = g[ra + n + x];
        }
    }
    __syncthreads();
    lds_fft_any<1, NTM, FC_EPT>(buf, fdm, 1, 8, twm, NTM > 0 ? twpm.w : nullptr);
    FixedTw<(NTL > 0 ? NTL : 1)> twpl;
    if constexpr (NTL > 0) fixed_tw_load<NTL>(twl, twpl.w);
    float2 rr[FC_EPT];
    double ss = 0.0;
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        rr[j] = make_float2(0.0f, 0.0f);
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) {
            const float2 v = buf[lds_slot(X)];
            const float a = gp[j].x - v.x;
            ss += (double)a * (double)a;
            float b = 0.0f;
            if (has_b) {
                b = gp[j].y - v.y;
                ss += (double)b * (double)b;
            }
            rr[j] = make_float2(a, b);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        if (X < M && x >= 0 && x < n) {
            buf[lds_slot(x)] = rr[j];
            if (x == 0) ends[0] = rr[j];
            if (x == N) ends[1] = rr[j];
        }
    }
    __syncthreads();
    // odd extension of the detrended residual rows (positions 0 and N zero)
    constexpr int KE = FFT_MAX_ELEMS / kBlock;
    float2 ext[KE];
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        ext[j] = make_float2(0.0f, 0.0f);
        if (k < L) {
            ext[j].x = ar_odd_detrended([&](int i) { return buf[lds_slot(i)].x; }, k, N, invN);
            ext[j].y = ar_odd_detrended([&](int i) { return buf[lds_slot(i)].y; }, k, N, invN);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        if (k < L) buf[lds_slot(k)] = ext[j];
    }
    __syncthreads();
    lds_fft_any<-1, NTL, FFT_EPT>(buf, fdl, 1, 8, twl, NTL > 0 ? twpl.w : nullptr);
    for (int jj = threadIdx.x; jj < n; jj += kBlock) {
        float2 c;
        if (jj == 0 || jj == N) {
            c = ends[jj == 0 ? 0 : 1];
        } else {
            const float2 X = buf[lds_slot(jj)];
            c = make_float2(-X.y * invN, X.x * invN);  // (2/N) DST-I
        }
        *reinterpret_cast<float2*>(Tr + (size_t)jj * tsr + 2 * q) = c;
    }
    if (partials) {
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// The preconditioner's inverse row pass (t = P r, two observed rows) and the
// forward row pass of A^T on the FFT-blur grid, where those rows sit at
// (y + off, x + off), in one workgroup.
template <int NTN, int NTM, bool DCT = false>
__global__ __launch_bounds__(kBlock) void precond_fc_blurT_kernel(
    const float2* __restrict__ Tp, int n_, int tsp, FftDesc fdn, const float2* __restrict__ twn,
    float* __restrict__ t_out, int off, float2* __restrict__ Tc, int M_, int tsc, FftDesc fdm,
    const float2* __restrict__ twm, int pair0, const float2* __restrict__ dtw) {
    extern __shared__ float2 buf[];
    const int M = NTM > 0 ? NTM : M_;
    const int n = NTN > 0 ? NTN : n_;
    const int q = xcd_block(blockIdx.x, gridDim.x);
    const int hn = n / 2 + 1;
    FixedTw<(NTN > 0 ? NTN : 1)> twpn;
    if constexpr (NTN > 0) fixed_tw_load<NTN>(twn, twpn.w);
    if constexpr (DCT) {  // DCT-III of the two rows as the DCT plan's inverse row pass
        const float* Tr = reinterpret_cast<const float*>(Tp);
        strided_copy<(NTN > 0 ? NTN : 0), float2>(
            n, [&](int k) { return *reinterpret_cast<const float2*>(Tr + (size_t)k * tsp + 2 * q); },
            [&](int k, float2 v) { buf[lds_slot(k)] = v; });
        __syncthreads();
        float2 keep[FFT_EPT];
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int k = threadIdx.x + i * kBlock;
            if (k < n) {
                const float2 Y = buf[lds_slot(k)];
                const float2 Yr = (k == 0) ? make_float2(0.0f, 0.0f) : buf[lds_slot(n - k)];
                const float2 wc = cconj(dtw[k]);
                const float2 Va = cmul(wc, make_float2(Y.x, -Yr.x));
                const float2 Vb = cmul(wc, make_float2(Y.y, -Yr.y));
                keep[i] = make_float2(Va.x - Vb.y, Va.y + Vb.x);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int k = threadIdx.x + i * kBlock;
            if (k < n) buf[lds_slot(k)] = keep[i];
        }
    } else {
        strided_copy<(NTN > 0 ? NTN / 2 + 1 : 0), float4>(
            hn, [&](int k) { return *reinterpret_cast<const float4*>(Tp + (size_t)k * tsp + 2 * q); },
            [&](int k, float4 v) {
                float2 Xa = make_float2(v.x, v.y), Xb = make_float2(v.z, v.w);
                const bool edge = (k == 0) || (2 * k == n);
                if (edge) {  // spectra of real rows are real at DC and Nyquist
                    Xa.y = 0.0f;
                    Xb.y = 0.0f;
                }
                buf[lds_slot(k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
                if (!edge) buf[lds_slot(n - k)] = make_float2(Xa.x + Xb.y, -Xa.y + Xb.x);
            });
    }
    __syncthreads();
    lds_fft_any<1, NTN, FFT_EPT>(buf, fdn, 1, 8, twn, NTN > 0 ? twpn.w : nullptr);
    // t at column x of the two rows
    auto tv = [&](int x) { return buf[lds_slot(DCT ? fc_dct_perm(x, n) : x)]; };
    if (t_out) {
        const size_t ra = (size_t)(2 * q) * n;
        for (int x = threadIdx.x; x < n; x += kBlock) {
            const float2 v = tv(x);
            t_out[ra + x] = v.x;
            t_out[ra + n + x] = v.y;
        }
    }
    FixedTw<(NTM > 0 ? NTM : 1)> twpm;
    if constexpr (NTM > 0) fixed_tw_load<NTM>(twm, twpm.w);
    float2 e[FC_EPT];
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        const int X = (int)threadIdx.x + j * kBlock;
        const int x = X - off;
        e[j] = (X < M && x >= 0 && x < n) ? tv(x) : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FC_EPT; ++j) {
        const int X = (int)threadIdx.x + j * kBlock;
        if (X < M) buf[lds_slot(X)] = e[j];
    }
    __syncthreads();
    lds_fft_any<-1, NTM, FC_EPT>(buf, fdm, 1, 8, twm, NTM > 0 ? twpm.w : nullptr);
    const int half = M / 2 + 1;
    const int pb = pair0 + q;
    for (int k = threadIdx.x; k < half; k += kBlock) {
        const float2 Z = buf[lds_slot(k)];
        const float2 Zc = cconj(buf[lds_slot(k == 0 ? 0 : M - k)]);
        const float2 Xa = cscale(cadd(Z, Zc), 0.5f);
        const float2 D = csub(Z, Zc);
        const float2 Xb = make_float2(0.5f * D.y, -0.5f * D.x);
        *reinterpret_cast<float4*>(Tc + (size_t)k * tsc + 2 * pb) = make_float4(Xa.x, Xa.y, Xb.x, Xb.y);
    }
}

// ---- launchers ------------------------------------------------------------

template <bool DIR>
static hipError_t launch_fc_rows_fwd_t(const FftConv& c, const float* src, int S, int off, int y_lo, int y_hi,
                                       hipStream_t s, int ext, const PcgDir& dir) {
    const int G = fc_pairs_per_block(c.M);
    const int p0 = y_lo / 2, p1 = (y_hi + 1) / 2;
    const int blocks = (p1 - p0 + G - 1) / G;
    if (blocks <= 0) return hipSuccess;
    if (c.M == kFixedM && G == 1)  // two row pairs per workgroup: 32-byte transposed writes
        hipLaunchKernelGGL((fc_rows_fwd_kernel<kFixedM, DIR, 2>), dim3((p1 - p0 + 1) / 2), dim3(2 * kBlock),
                           2 * lds_bytes(c.M, c.M), s, src, S, off, c.M, c.T, c.ts, c.fd, c.tw, 2, fc_seq_shift(1), p0,
                           p1, ext, dir);
    else if (c.M == kFixedM2 && G == 1)
        hipLaunchKernelGGL((fc_rows_fwd_kernel<kFixedM2, DIR>), dim3(blocks), dim3(kBlock), lds_bytes(c.M, c.M), s,
                           src, S, off, c.M, c.T, c.ts, c.fd, c.tw, 1, fc_seq_shift(1), p0, p1, ext, dir);
    else
        hipLaunchKernelGGL((fc_rows_fwd_kernel<0, DIR>), dim3(blocks), dim3(kBlock), lds_bytes(G * c.M, c.M), s, src,
                           S, off, c.M, c.T, c.ts, c.fd, c.tw, G, fc_seq_shift(G), p0, p1, ext, dir);
    return hipGetLastError();
}

hipError_t launch_fc_rows_fwd(const FftConv& c, const float* src, int S, int off, int y_lo, int y_hi,
                              hipStream_t s, int ext, const PcgDir* dir) {
    if (dir) {
        if (ext != EXT_ZERO || dir->d != src) return hipErrorInvalidValue;
        return launch_fc_rows_fwd_t<true>(c, src, S, off, y_lo, y_hi, s, ext, *dir);
    }
    return launch_fc_rows_fwd_t<false>(c, src, S, off, y_lo, y_hi, s, ext, PcgDir{});
}

// ---- the column pass without column transforms ----------------------------
// After the row pass, column k of the grid holds U(y, k) = sum_x u(y, x) W^(x k)
// (W = exp(-2 pi i / M)).  In those coordinates the 2-D convolution with the
// PSF is, column by column, a P-tap convolution along y whose taps are the
// PSF's rows transformed the same way, G(a, k) = sum_b h(a, b) W^(b k):
//   A:   V(o, k) = sum_a G(a, k) U(o - a, k)
//   A^T: V(o, k) = sum_a conj(G(a, k)) U(o + a, k)     (the correlation)
// These are the values the column transform pair with F(pad H) (or its
// conjugate) gives, as long as no input index that wraps around the grid
// lands on a nonzero row (the launcher checks); `scale` is the 1/M of the
// inverse row pass (no column transforms, so no second 1/M).  R consecutive
// outputs per thread (4, 5, 8 or 9, the fewest that cover the column): a
// column's inputs are staged in LDS once (rows outside [y_lo, y_hi) as zero),
// each thread reads its R + P - 1 of them, the P taps are uniform over the
// workgroup (scalar registers), and the outputs leave through LDS as one
// coalesced store.  Each workgroup walks the columns k = blockIdx.x,
// + gridDim.x, ...: the next column's global loads are issued before the
// current one's multiply-adds, so that the loads of one column and the
// arithmetic of another overlap.
// fold >= 0 (A^T of a square model): the outputs are the grid rows [0, m)
// and the column's rows [0, fn) receive E^T of them, the sum over each
// pixel's preimages under the pad of width fcn, as the transform pair's
// write-back does.
template <int P, int R, bool CORR>
__global__ __launch_bounds__(kBlock) void fc_cols_direct_kernel(float2* __restrict__ T, int ts,
                                                                const float2* __restrict__ G, float scale, int y_lo,
                                                                int y_hi, int o_lo, int o_hi, int half, int fold,
                                                                int fn, int fcn) {
    constexpr int W = R + P - 1;           // inputs per thread
    constexpr int S = kBlock * R + P - 1;  // inputs per column
    constexpr int J = (S + kBlock - 1) / kBlock;
    // lanes read at stride R: an odd stride meets no bank twice already, an
    // even one gets a spare slot every R entries (stride R + 1)
    constexpr bool PAD = R % 2 == 0;
    auto slot = [](int l) { return PAD ? l + l / R : l; };
    __shared__ float2 in[PAD ? S + S / R + 1 : S];
    __shared__ float2 out[PAD ? kBlock * R + kBlock : kBlock * R];
    const int base = CORR ? o_lo : o_lo - (P - 1);  // grid row of LDS entry 0
    const int count = o_hi - o_lo;
    const int t0 = (int)threadIdx.x * R;
    float2 pre[J];
    auto fetch = [&](int k) {
        const float2* col = T + (size_t)k * ts;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int l = j * kBlock + (int)threadIdx.x;
            const int i = base + l;
            pre[j] = ((S % kBlock == 0 || l < S) && i >= y_lo && i < y_hi) ? col[i] : make_float2(0.0f, 0.0f);
        }
    };
    int k = blockIdx.x;
    fetch(k);
    for (; k < half; k += gridDim.x) {
        const float2* __restrict__ g = G + (size_t)k * P;
        float2 tap[P];
#pragma unroll
        for (int a = 0; a < P; ++a) tap[a] = g[a];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int l = j * kBlock + (int)threadIdx.x;
            if (S % kBlock == 0 || l < S) in[slot(l)] = pre[j];
        }
        __syncthreads();  // the column is staged (and the previous one's outputs are stored)
        if (k + (int)gridDim.x < half) fetch(k + gridDim.x);
        // window entry c (input t0 + c) meets output r through tap a = c - r
        // (A^T) or r + P - 1 - c (A); each entry is read once from LDS
        float ax[R], ay[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ax[r] = ay[r] = 0.0f;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const float2 v = in[slot(t0 + c)];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int a = CORR ? c - r : r + P - 1 - c;
                if (a < 0 || a >= P) continue;
                const float2 h = tap[a];
                if constexpr (CORR) {  // conj(h) v
                    ax[r] = fmaf(h.x, v.x, ax[r]);
                    ax[r] = fmaf(h.y, v.y, ax[r]);
                    ay[r] = fmaf(h.x, v.y, ay[r]);
                    ay[r] = fmaf(-h.y, v.x, ay[r]);
                } else {
                    ax[r] = fmaf(h.x, v.x, ax[r]);
                    ax[r] = fmaf(-h.y, v.y, ax[r]);
                    ay[r] = fmaf(h.x, v.y, ay[r]);
                    ay[r] = fmaf(h.y, v.x, ay[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) out[slot(t0 + r)] = make_float2(ax[r] * scale, ay[r] * scale);
        __syncthreads();  // the outputs are complete and every window has been read
        float2* col = T + (size_t)k * ts;
        if (fold >= 0) {
            const int rows = fn + (fn & 1);
            for (int l = threadIdx.x; l < rows; l += kBlock)
                col[l] = l < fn ? fold_sum(l, fn, fcn, fold, [&](int Y) { return out[slot(Y - o_lo)]; })
                                : make_float2(0.0f, 0.0f);
        } else {
            for (int l = threadIdx.x; l < count; l += kBlock) col[o_lo + l] = out[slot(l)];
        }
    }
}

// Workgroups of the direct column pass: three per CU of the 256-CU device,
// each walking about 1.5 columns of the 2304-point grid (measured against one
// column per workgroup: 17.5 against 18.5 us per launch).
constexpr int kDirectGrid = 768;

// The taps G of the direct column pass: the first p rows of every column
// after the row pass of the PSF placed at the origin.
__global__ __launch_bounds__(kBlock) void fc_taps_kernel(const float2* __restrict__ T, int ts, int half, int p,
                                                         float2* __restrict__ G) {
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= half * p) return;
    const int k = idx / p;
    G[idx] = T[(size_t)k * ts + (idx - k * p)];
}

// The direct column pass, when the plan has the taps for this PSF size and
// the outputs' inputs stay inside the grid; false: not taken.
template <int P>
static bool fc_cols_direct_t(const FftConv& c, bool corr, int y_lo, int y_hi, int o_lo, int o_hi, int fold, int fn,
                             int fcn, hipStream_t s) {
    const int count = o_hi - o_lo;
    if (count <= 0 || count > 9 * kBlock || o_lo < 0 || o_hi > c.M || y_lo < 0 || y_hi > c.M) return false;
    // the transform pair's convolution is circular: an input index past the
    // grid wraps around, and the direct pass (which reads zero there) agrees
    // only while no wrapped index lands on a nonzero row
    if (corr ? (o_hi + P - 2 >= c.M && o_hi + P - 2 - c.M >= y_lo)
             : (o_lo - (P - 1) < 0 && o_lo - (P - 1) + c.M < y_hi))
        return false;
    const int half = c.M / 2 + 1;
    const float scale = (float)(1.0 / (double)c.M);
    // outputs per thread: the fewest of 4, 5, 8, 9 that cover the column
    const int R = count <= 4 * kBlock ? 4 : count <= 5 * kBlock ? 5 : count <= 8 * kBlock ? 8 : 9;
    const int grid = half < kDirectGrid ? half : kDirectGrid;
#define FC_DIRECT(R, CO)                                                                                     \
    hipLaunchKernelGGL((fc_cols_direct_kernel<P, R, CO>), dim3(grid), dim3(kBlock), 0, s, c.T, c.ts,        \
                       (const float2*)c.G, scale, y_lo, y_hi, o_lo, o_hi, half, fold, fn, fcn)
    switch (R) {
        case 4:
            if (corr) FC_DIRECT(4, true);
            else FC_DIRECT(4, false);
            break;
        case 5:
            if (corr) FC_DIRECT(5, true);
            else FC_DIRECT(5, false);
            break;
        case 8:
            if (corr) FC_DIRECT(8, true);
            else FC_DIRECT(8, false);
            break;
        default:
            if (corr) FC_DIRECT(9, true);
            else FC_DIRECT(9, false);
            break;
    }
#undef FC_DIRECT
    return true;
}

static bool fc_cols_direct(const FftConv& c, int conj_h, int y_lo, int y_hi, int mode, int o_lo, int o_hi,
                           int fold, int fn, int fcn, hipStream_t s) {
    if (!c.G || mode != 0 || (conj_h != 0 && conj_h != 1)) return false;
    if (fold >= 0) {  // E^T folds the grid rows [0, fn + 2 fcn) of the correlation
        if (conj_h != 1) return false;
        o_lo = 0;
        o_hi = fn + 2 * fcn;
    }
    switch (c.p) {
        case 5: return fc_cols_direct_t<5>(c, conj_h == 1, y_lo, y_hi, o_lo, o_hi, fold, fn, fcn, s);
        case 9: return fc_cols_direct_t<9>(c, conj_h == 1, y_lo, y_hi, o_lo, o_hi, fold, fn, fcn, s);
        case 17: return fc_cols_direct_t<17>(c, conj_h == 1, y_lo, y_hi, o_lo, o_hi, fold, fn, fcn, s);
        case 31: return fc_cols_direct_t<31>(c, conj_h == 1, y_lo, y_hi, o_lo, o_hi, fold, fn, fcn, s);
        default: return false;
    }
}

bool fftconv_direct_taps(int p) { return p == 5 || p == 9 || p == 17 || p == 31; }

hipError_t launch_fc_cols(const FftConv& c, int conj_h, int y_lo, int y_hi, int mode, float2* cspec, hipStream_t s,
                          int o_lo, int o_hi, int fold, int fn, int fcn) {
    if (fc_cols_direct(c, conj_h, y_lo, y_hi, mode, o_lo, o_hi, fold, fn, fcn, s)) return hipGetLastError();
    const int CC = fc_cols_per_block(c.M);
    const int half = c.M / 2 + 1;
    const float inv = (float)(1.0 / ((double)c.M * (double)c.M));
    if (c.M == kFixedM && CC == 1)
        hipLaunchKernelGGL(fc_cols_kernel<kFixedM>, dim3(half), dim3(kBlock), lds_bytes(c.M, c.M), s, c.T, c.M, c.ts,
                           (const float2*)c.H, conj_h, inv, y_lo, y_hi, mode, cspec, c.fd, c.tw, 1, fc_seq_shift(1), o_lo,
                           o_hi, fold, fn, fcn);
    else if (c.M == kFixedM2 && CC == 1)
        hipLaunchKernelGGL(fc_cols_kernel<kFixedM2>, dim3(half), dim3(kBlock), lds_bytes(c.M, c.M), s, c.T, c.M, c.ts,
                           (const float2*)c.H, conj_h, inv, y_lo, y_hi, mode, cspec, c.fd, c.tw, 1, fc_seq_shift(1), o_lo,
                           o_hi, fold, fn, fcn);
    else
        hipLaunchKernelGGL(fc_cols_kernel<0>, dim3((half + CC - 1) / CC), dim3(kBlock), lds_bytes(CC * c.M, c.M), s,
                           c.T, c.M, c.ts, (const float2*)c.H, conj_h, inv, y_lo, y_hi, mode, cspec, c.fd, c.tw, CC,
                           fc_seq_shift(CC), o_lo, o_hi, fold, fn, fcn);
    return hipGetLastError();
}

hipError_t launch_fc_rows_inv(const FftConv& c, int oy, int ox, int D, float* dst, const float* g, int accum,
                              double* partials, int* n_partials, hipStream_t s, int fold, int fcn, const float* axd,
                              float axa) {
    if (fold >= 0 && ox != 0) return hipErrorInvalidValue;
    const int G = fc_pairs_per_block(c.M);
    const int p0 = oy / 2, p1 = (oy + D + 1) / 2;
    const int blocks = (p1 - p0 + G - 1) / G;
    if (n_partials) *n_partials = blocks;
    if (c.M == kFixedM && G == 1)
        hipLaunchKernelGGL(fc_rows_inv_kernel<kFixedM>, dim3(blocks), dim3(kBlock), lds_bytes(c.M, c.M), s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, 1, fc_seq_shift(1), p0, p1, oy, ox, D, dst, g,
                           accum, partials, fold, fcn, axd, axa);
    else if (c.M == kFixedM2 && G == 1)
        hipLaunchKernelGGL(fc_rows_inv_kernel<kFixedM2>, dim3(blocks), dim3(kBlock), lds_bytes(c.M, c.M), s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, 1, fc_seq_shift(1), p0, p1, oy, ox, D, dst, g,
                           accum, partials, fold, fcn, axd, axa);
    else
        hipLaunchKernelGGL(fc_rows_inv_kernel<0>, dim3(blocks), dim3(kBlock), lds_bytes(G * c.M, c.M), s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, G, fc_seq_shift(G), p0, p1, oy, ox, D, dst, g,
                           accum, partials, fold, fcn, axd, axa);
    return hipGetLastError();
}

int fftconv_partials_count(int M, int n) {
    const int G = fc_pairs_per_block(M);
    return (n / 2 + 1 + G) / G + 1;
}

hipError_t launch_fftconv_spectrum(const FftConv& c, const float* psf, int p, hipStream_t s) {
    hipError_t e = launch_fc_rows_fwd(c, psf, p, 0, 0, p, s);
    if (e != hipSuccess) return e;
    if (c.G) {
        if (c.p != p) return hipErrorInvalidValue;
        const int n = (c.M / 2 + 1) * p;
        hipLaunchKernelGGL(fc_taps_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, (const float2*)c.T,
                           c.ts, c.M / 2 + 1, p, c.G);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return launch_fc_cols(c, 0, 0, p, 1, c.H, s, 0, c.M, -1, 0, 0);
}

template <bool DCT>
static hipError_t launch_frp(const FftConv& c, int n, int p, const float* g, float* r_out, double* partials,
                             const PrecondRows& pr, hipStream_t s) {
    const int blocks = n / 2;
    const size_t lds = lds_bytes(c.M > n ? c.M : n, 0);
    if (c.M == kFixedM && n == kFixedN)
        hipLaunchKernelGGL((fc_residual_precond_kernel<kFixedM, kFixedN, DCT>), dim3(blocks), dim3(kBlock), lds, s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, (p - 1) / 2, n, p - 1, g, r_out, partials, pr.T,
                           pr.ts, pr.fd, pr.tw, pr.dtw);
    else
        hipLaunchKernelGGL((fc_residual_precond_kernel<0, 0, DCT>), dim3(blocks), dim3(kBlock), lds, s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, (p - 1) / 2, n, p - 1, g, r_out, partials, pr.T,
                           pr.ts, pr.fd, pr.tw, pr.dtw);
    return hipGetLastError();
}

hipError_t launch_fc_residual_precond_rows(const FftConv& c, int n, int p, const float* g, float* r_out,
                                           double* partials, int* n_partials, const PrecondRows& pr, hipStream_t s) {
    if (!fftconv_fusable(c, n, pr)) return hipErrorInvalidValue;
    if (n_partials) *n_partials = n / 2;
    return pr.dtw ? launch_frp<true>(c, n, p, g, r_out, partials, pr, s)
                  : launch_frp<false>(c, n, p, g, r_out, partials, pr, s);
}

bool fftconv_ar_fusable(const FftConv& c, int n, const FftDesc& fdl) {
    return c.M <= FC_MAX && fdl.m == 0 && fdl.n == 2 * (n - 1) && fdl.n <= FFT_MAX_ELEMS;
}

hipError_t launch_fc_residual_ar_rows(const FftConv& c, int n, int p, const float* g, double* partials,
                                     int* n_partials, float* Tr, int tsr, const FftDesc& fdl, const float2* twl,
                                     hipStream_t s) {
    if (!fftconv_ar_fusable(c, n, fdl)) return hipErrorInvalidValue;
    const int blocks = (n + 1) / 2;
    if (n_partials) *n_partials = blocks;
    const size_t lds = lds_bytes(c.M > fdl.n ? c.M : fdl.n, 0);
    if (c.M == kFixedM2 && fdl.n == kFixedN)
        hipLaunchKernelGGL((fc_residual_ar_kernel<kFixedM2, kFixedN>), dim3(blocks), dim3(kBlock), lds, s,
                           (const float2*)c.T, c.M, c.ts, c.fd, c.tw, (p - 1) / 2, n, p - 1, g, partials, Tr, tsr, fdl,
                           twl);
    else
        hipLaunchKernelGGL((fc_residual_ar_kernel<0, 0>), dim3(blocks), dim3(kBlock), lds, s, (const float2*)c.T,
                           c.M, c.ts, c.fd, c.tw, (p - 1) / 2, n, p - 1, g, partials, Tr, tsr, fdl, twl);
    return hipGetLastError();
}

template <bool DCT>
static hipError_t launch_pfb(const FftConv& c, int n, int p, const PrecondRows& pr, float* t_out, hipStream_t s) {
    const size_t lds = lds_bytes(c.M > n ? c.M : n, 0);
    if (c.M == kFixedM && n == kFixedN)
        hipLaunchKernelGGL((precond_fc_blurT_kernel<kFixedN, kFixedM, DCT>), dim3(n / 2), dim3(kBlock), lds, s,
                           (const float2*)pr.T, n, pr.ts, pr.fd, pr.tw, t_out, p - 1, c.T, c.M, c.ts, c.fd, c.tw,
                           (p - 1) / 2, pr.dtw);
    else
        hipLaunchKernelGGL((precond_fc_blurT_kernel<0, 0, DCT>), dim3(n / 2), dim3(kBlock), lds, s,
                           (const float2*)pr.T, n, pr.ts, pr.fd, pr.tw, t_out, p - 1, c.T, c.M, c.ts, c.fd, c.tw,
                           (p - 1) / 2, pr.dtw);
    return hipGetLastError();
}

hipError_t launch_precond_rows_fc_fwd(const FftConv& c, int n, int p, const PrecondRows& pr, float* t_out,
                                      hipStream_t s) {
    if (!fftconv_fusable(c, n, pr)) return hipErrorInvalidValue;
    return pr.dtw ? launch_pfb<true>(c, n, p, pr, t_out, s) : launch_pfb<false>(c, n, p, pr, t_out, s);
}

bool fftconv_fusable(const FftConv& c, int n, const PrecondRows& pr) {
    return c.T && n % 2 == 0 && n <= FFT_MAX_ELEMS && pr.T && pr.fd.n == n && pr.fd.m == 0;
}

}  // namespace mlba
