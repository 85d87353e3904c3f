// Spectral Tikhonov preconditioners (paper section 4):
//   Algorithm 1: P r = F^-1[ F r / (|Lambda|^2 + alpha) ]   (2-D DFT, BCCB C)
//   Algorithm 3: P r = C2^T[ C2 r / (lambda^2 + alpha) ]     (2-D DCT-II, Q of the
//                symmetrised PSF)
//
// Both are three passes over an n x n image:
//   1. rows: two real rows are packed into one complex sequence, transformed
//      in LDS and split; the result is written transposed (frequency-major), so
//   2. columns become contiguous: forward transform, multiply by the
//      spectral filter, inverse transform, all in LDS in one kernel;
//   3. rows: gather transposed, inverse transform, write rows.
//
// The complex FFT is a mixed-radix (8, 4, 2, 3, 5) Stockham autosort transform
// held in LDS; every thread carries up to 8 complex values per stage in
// registers between the read and the write barrier.  Twiddles come from a
// table of exp(-2 pi i q / n) computed in double precision on the host.
// The DCT-II of length n is computed from a length-n complex FFT of the even
// samples followed by the reversed odd samples, with a quarter-sample
// post-twiddle (Makhoul's reordering); DCT-III inverts those steps.
// All transforms here are unnormalised; the filter carries the 1/n^2.
#include "artrans.hpp"
#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"

namespace mlba {

// ---------------------------------------------------------------------------
// BCCB (Algorithm 1)
// ---------------------------------------------------------------------------

// G row pairs per workgroup -> T[k][row], k = 0..n/2 (row stride ts complex).
// NT > 0: n == NT and one row pair per workgroup (fixed-size transform).
// src(i): the value at flat index i of the n x n input (read once per element).
template <int NT, class Src>
__device__ __forceinline__ void fft_rows_r2c_body_f(Src src, int n_, float2* __restrict__ T, int ts,
                                                    const FftDesc& fd, const float2* __restrict__ tw, int G_,
                                                    int seq_shift, int blk, float2* buf) {
    const int n = NT > 0 ? NT : n_;
    const int G = NT > 0 ? 1 : G_;
    const int row0 = blk * 2 * G;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        G * n,
        [&](int idx) {
            const int g = idx / n;
            const int x = idx - g * n;
            const size_t ra = (size_t)(row0 + 2 * g) * n;
            return make_float2(src(ra + x), src(ra + n + x));
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    const int half = n / 2 + 1;
    for (int idx = threadIdx.x; idx < G * half; idx += kBlock) {
        const int k = idx / G;
        const int g = idx - k * G;
        const float2 Z = buf[lds_slot(g * n + k)];
        const float2 Zc = cconj(buf[lds_slot(g * n + (k == 0 ? 0 : n - k))]);
        const float2 Xa = cscale(cadd(Z, Zc), 0.5f);
        const float2 D = csub(Z, Zc);
        const float2 Xb = make_float2(0.5f * D.y, -0.5f * D.x);  // D / (2i)
        *reinterpret_cast<float4*>(T + (size_t)k * ts + row0 + 2 * g) = make_float4(Xa.x, Xa.y, Xb.x, Xb.y);
    }
}

template <int NT = 0>
__device__ __forceinline__ void fft_rows_r2c_body(const float* __restrict__ src, int n_, float2* __restrict__ T,
                                                  int ts, const FftDesc& fd, const float2* __restrict__ tw, int G_,
                                                  int seq_shift, int blk, float2* buf) {
    fft_rows_r2c_body_f<NT>([&](size_t i) { return src[i]; }, n_, T, ts, fd, tw, G_, seq_shift, blk, buf);
}

// CC rows of T per workgroup, along the column index:
//   mode 0: forward FFT, filter inv / (spec + alpha) (times conj(lamc) when
//           lamc is given: C^T (C C^T + alpha I)^{-1} of Algorithm 4), inverse FFT;
//   mode 1: forward FFT, |.|^2 into `power`;
//   mode 2: forward FFT, the complex values into `cspec`;
//   mode 3: forward FFT only, written back to T;
//   mode 4: filter of mode 0 on the spectrum already in T, inverse FFT.
// alpha_dev (optional) replaces alpha by a value computed on the device.
template <int NT = 0>
__device__ __forceinline__ void fft_cols_body(float2* __restrict__ T, int n_, int ts,
                                                          const float* __restrict__ spec, float alpha,
                                                          float inv, const FftDesc& fd,
                                                          const float2* __restrict__ tw, int CC_, int mode,
                                                          float* __restrict__ power, int seq_shift, int blk, float2* buf,
                                                          float2* __restrict__ sstore = nullptr,
                                                          const float2* __restrict__ sfwd = nullptr,
                                                          float* __restrict__ eacc = nullptr,
                                                          const float2* __restrict__ lamc = nullptr,
                                                          const double* __restrict__ alpha_dev = nullptr,
                                                          float2* __restrict__ cspec = nullptr) {
    const int n = NT > 0 ? NT : n_;
    const int CC = NT > 0 ? 1 : CC_;
    const int half = n / 2 + 1;
    const int k0 = blk * CC;
    const int cc = min(CC, half - k0);
    const size_t base = (size_t)k0 * n;  // dense [n/2+1][n] spectrum
    if constexpr (NT > 0 && fixed_conv_ok<(NT > 0 ? NT : 1)>()) {
        if (mode == 0) {  // the filter between the transforms, in registers
            constexpr int SL = fixed_conv_slots<NT>();
            FixedTw<NT> twf;
            FixedTw<NT, true> twi;
            fixed_tw_load<NT>(tw, twf.w);
            fixed_tw_load<NT, 0, true>(tw, twi.w);
            float sr[SL];
#pragma unroll
            for (int r = 0; r < SL; ++r) sr[r] = spec[base + threadIdx.x + r * kBlock];
            if (alpha_dev) alpha = (float)*alpha_dev;
            float2* col = T + (size_t)k0 * ts;
            fixed_conv<NT>(
                buf, tw, twf.w, twi.w, [&](int y) { return col[y]; },
                [&](int r, int y, float2 v) {
                    v = cscale(v, inv / (sr[r] + alpha));
                    if (lamc) v = cmul(v, cconj(lamc[base + y]));
                    if (sstore) sstore[base + y] = v;  // reverse sweep of unrolled iterations
                    if (eacc) {
                        const float2 f = sfwd[base + y];
                        eacc[base + y] += fmaf(v.x, f.x, v.y * f.y);
                    }
                    return v;
                },
                [&](int y, float2 v) { col[y] = v; }, false);
            return;
        }
    }
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        cc * n,
        [&](int idx) {
            const int q = idx / n;
            return T[(size_t)(k0 + q) * ts + (idx - q * n)];
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
    // compiled length, filter modes: the filter's denominators are loaded
    // with the column, before the transform
    constexpr int SPER = NT > 0 ? (NT + kBlock - 1) / kBlock : 1;
    float sreg[SPER];
    if constexpr (NT > 0) {
        if (mode == 0 || mode == 4) {
#pragma unroll
            for (int k = 0; k < SPER; ++k) {
                const int e = k * kBlock + (int)threadIdx.x;
                if (NT % kBlock == 0 || e < NT) sreg[k] = spec[base + e];
            }
        }
    }
    __syncthreads();
    if (mode != 4) lds_fft_any<-1, NT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    if (mode == 1) {
        for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
            const float2 v = buf[lds_slot(idx)];
            power[base + idx] = v.x * v.x + v.y * v.y;
        }
        return;
    }
    if (mode == 2) {
        for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) cspec[base + idx] = buf[lds_slot(idx)];
        return;
    }
    if (mode == 3) {
        for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
            const int q = idx / n;
            T[(size_t)(k0 + q) * ts + (idx - q * n)] = buf[lds_slot(idx)];
        }
        return;
    }
    if (alpha_dev) alpha = (float)*alpha_dev;
    if constexpr (NT > 0) {
#pragma unroll
        for (int k = 0; k < SPER; ++k) {
            const int idx = k * kBlock + (int)threadIdx.x;
            if (NT % kBlock == 0 || idx < NT) {
                float2 v = cscale(buf[lds_slot(idx)], inv / (sreg[k] + alpha));
                if (lamc) v = cmul(v, cconj(lamc[base + idx]));
                buf[lds_slot(idx)] = v;
            }
        }
    } else {
        for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
            float2 v = cscale(buf[lds_slot(idx)], inv / (spec[base + idx] + alpha));
            if (lamc) v = cmul(v, cconj(lamc[base + idx]));
            buf[lds_slot(idx)] = v;
        }
    }
    if (sstore || eacc) {  // reverse sweep of unrolled iterations (same thread owns each slot)
        for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
            const float2 v = buf[lds_slot(idx)];
            if (sstore) sstore[base + idx] = v;
            if (eacc) {
                const float2 f = sfwd[base + idx];
                eacc[base + idx] += fmaf(v.x, f.x, v.y * f.y);
            }
        }
    }
    __syncthreads();
    lds_fft_any<1, NT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
        const int q = idx / n;
        T[(size_t)(k0 + q) * ts + (idx - q * n)] = buf[lds_slot(idx)];
    }
}

// CC rows of T per workgroup: inverse FFT along the column index of the real
// dense spectrum e ([n/2+1][n]), written to T.
template <int NT = 0>
__device__ __forceinline__ void fft_cols_inverse_real_body(const float* __restrict__ e, float2* __restrict__ T,
                                                           int n, int ts, const FftDesc& fd,
                                                           const float2* __restrict__ tw, int CC, int seq_shift,
                                                           int blk, float2* buf) {
    const int half = n / 2 + 1;
    const int k0 = blk * CC;
    const int cc = min(CC, half - k0);
    const size_t base = (size_t)k0 * n;
    for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) buf[lds_slot(idx)] = make_float2(e[base + idx], 0.0f);
    __syncthreads();
    lds_fft_any<1, NT>(buf, fd, cc, seq_shift, tw);
    for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
        const int q = idx / n;
        T[(size_t)(k0 + q) * ts + (idx - q * n)] = buf[lds_slot(idx)];
    }
}

// put(i, v): the value v of flat index i of the n x n output.
template <int NT, class Put>
__device__ __forceinline__ void fft_rows_c2r_body_f(const float2* __restrict__ T, int n_, int ts, Put put,
                                                    const FftDesc& fd, const float2* __restrict__ tw, int G_,
                                                    int seq_shift, int blk, float2* buf) {
    const int n = NT > 0 ? NT : n_;
    const int G = NT > 0 ? 1 : G_;
    const int row0 = blk * 2 * G;
    const int half = n / 2 + 1;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<(NT > 0 ? NT / 2 + 1 : 0), float4>(
        G * half,
        [&](int idx) {
            const int k = idx / G;
            const int g = idx - k * G;
            return *reinterpret_cast<const float4*>(T + (size_t)k * ts + row0 + 2 * g);
        },
        [&](int idx, float4 q) {
            const int k = idx / G;
            const int g = idx - k * G;
            float2 Xa = make_float2(q.x, q.y), Xb = make_float2(q.z, q.w);
            const bool edge = (k == 0) || (2 * k == n);
            if (edge) {  // spectra of real rows are real at DC and Nyquist
                Xa.y = 0.0f;
                Xb.y = 0.0f;
            }
            buf[lds_slot(g * n + k)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);  // Xa + i Xb
            if (!edge) buf[lds_slot(g * n + n - k)] = make_float2(Xa.x + Xb.y, -Xa.y + Xb.x);  // conj(Xa) + i conj(Xb)
        });
    __syncthreads();
    lds_fft_any<1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < G * n; idx += kBlock) {
        const int g = idx / n;
        const int x = idx - g * n;
        const size_t ra = (size_t)(row0 + 2 * g) * n;
        const float2 v = buf[lds_slot(idx)];
        put(ra + x, v.x);
        put(ra + n + x, v.y);
    }
}

template <int NT = 0>
__device__ __forceinline__ void fft_rows_c2r_body(const float2* __restrict__ T, int n_, int ts,
                                                  float* __restrict__ dst, const FftDesc& fd,
                                                  const float2* __restrict__ tw, int G_, int seq_shift, int blk,
                                                  float2* buf, int accum = 0) {
    if (accum)
        fft_rows_c2r_body_f<NT>(T, n_, ts, [&](size_t i, float v) { dst[i] += v; }, fd, tw, G_, seq_shift, blk, buf);
    else
        fft_rows_c2r_body_f<NT>(T, n_, ts, [&](size_t i, float v) { dst[i] = v; }, fd, tw, G_, seq_shift, blk, buf);
}

// ---------------------------------------------------------------------------
// DCT (Algorithm 3)
// ---------------------------------------------------------------------------

// position of sample l in the reordered sequence (evens ascending, odds descending)
__device__ __forceinline__ int dct_perm(int l, int n) { return (l & 1) ? n - 1 - (l >> 1) : (l >> 1); }

__device__ __forceinline__ float re_mul(float2 w, float2 v) { return w.x * v.x - w.y * v.y; }

// G row pairs -> Tr[k][row] (real, row stride ts), k = 0..n-1
// NT > 0 (here and in the two DCT bodies below): n == NT with one sequence per
// workgroup, the compiled fixed-size transform.
template <int NT = 0>
__device__ __forceinline__ void dct_rows_fwd_body(const float* __restrict__ src, int n_,
                                                              float* __restrict__ Tr, int ts, const FftDesc& fd,
                                                              const float2* __restrict__ tw,
                                                              const float2* __restrict__ dtw, int G_, int seq_shift, int blk, float2* buf) {
    const int n = NT > 0 ? NT : n_;
    const int G = NT > 0 ? 1 : G_;
    const int row0 = blk * 2 * G;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        G * n,
        [&](int idx) {
            const int g = idx / n;
            const int x = idx - g * n;
            const size_t ra = (size_t)(row0 + 2 * g) * n;
            return make_float2(src[ra + x], src[ra + n + x]);
        },
        [&](int idx, float2 v) {
            const int g = idx / n;
            buf[lds_slot(g * n + dct_perm(idx - g * n, n))] = v;
        });
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < G * n; idx += kBlock) {
        const int k = idx / G;
        const int g = idx - k * G;
        const float2 Z = buf[lds_slot(g * n + k)];
        const float2 Zc = cconj(buf[lds_slot(g * n + (k == 0 ? 0 : n - k))]);
        const float2 Va = cscale(cadd(Z, Zc), 0.5f);
        const float2 D = csub(Z, Zc);
        const float2 Vb = make_float2(0.5f * D.y, -0.5f * D.x);
        const float2 w = dtw[k];
        *reinterpret_cast<float2*>(Tr + (size_t)k * ts + row0 + 2 * g) = make_float2(re_mul(w, Va), re_mul(w, Vb));
    }
}

// CP pairs of Tr rows per workgroup.  mode 0: DCT-II along the row, multiply
// by inv / (spec + alpha) (times lamr: C^T (C C^T + alpha I)^{-1} of
// Algorithm 4), DCT-III back; mode 1: DCT-II only, the coefficients written
// back (Algorithm 4-NS solves for alpha from them); mode 2: from those
// coefficients, multiply by inv lamr / (spec + alpha_dev[0]), DCT-III back.
template <int NT = 0>
__device__ __forceinline__ void dct_cols_filter_body(float* __restrict__ Tr, int n_, int ts,
                                                                 const float* __restrict__ spec, float alpha,
                                                                 float inv, const FftDesc& fd,
                                                                 const float2* __restrict__ tw,
                                                                 const float2* __restrict__ dtw, int CP_, int seq_shift, int blk, float2* buf,
                                                                 const float* __restrict__ lamr = nullptr,
                                                                 int mode = 0,
                                                                 const double* __restrict__ alpha_dev = nullptr) {
    const int n = NT > 0 ? NT : n_;
    const int CP = NT > 0 ? 1 : CP_;
    const int pairs = n / 2;
    const int p0 = blk * CP;
    const int cp = min(CP, pairs - p0);
    const int total = cp * n;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    float2 keep[FFT_EPT];
    if (mode == 2) {
        const float a = (float)alpha_dev[0];
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int idx = threadIdx.x + i * kBlock;
            if (idx < total) {
                const int q = idx / n;
                const int l = idx - q * n;
                const size_t r1 = (size_t)(2 * (p0 + q)) * ts;
                const size_t s1 = (size_t)(2 * (p0 + q)) * n;
                const float f1 = inv / (spec[s1 + l] + a) * lamr[s1 + l];
                const float f2 = inv / (spec[s1 + n + l] + a) * lamr[s1 + n + l];
                keep[i] = make_float2(Tr[r1 + l] * f1, Tr[r1 + ts + l] * f2);
            }
        }
    } else {
        strided_copy<NT, float2>(
            total,
            [&](int idx) {
                const int q = idx / n;
                const int l = idx - q * n;
                const size_t r1 = (size_t)(2 * (p0 + q)) * ts;
                return make_float2(Tr[r1 + l], Tr[r1 + ts + l]);
            },
            [&](int idx, float2 v) {
                const int q = idx / n;
                buf[lds_slot(q * n + dct_perm(idx - q * n, n))] = v;
            });
        __syncthreads();
        lds_fft_any<-1, NT>(buf, fd, cp, seq_shift, tw, NT > 0 ? twp.w : nullptr);
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int idx = threadIdx.x + i * kBlock;
            if (idx < total) {
                const int q = idx / n;
                const int l = idx - q * n;
                const float2 Z = buf[lds_slot(q * n + l)];
                const float2 Zc = cconj(buf[lds_slot(q * n + (l == 0 ? 0 : n - l))]);
                const float2 V1 = cscale(cadd(Z, Zc), 0.5f);
                const float2 D = csub(Z, Zc);
                const float2 V2 = make_float2(0.5f * D.y, -0.5f * D.x);
                const float2 w = dtw[l];
                if (mode == 1) {
                    keep[i] = make_float2(re_mul(w, V1), re_mul(w, V2));
                } else {
                    const size_t s1 = (size_t)(2 * (p0 + q)) * n;  // dense [n][n] spectrum
                    float f1 = inv / (spec[s1 + l] + alpha);
                    float f2 = inv / (spec[s1 + n + l] + alpha);
                    if (lamr) {
                        f1 *= lamr[s1 + l];
                        f2 *= lamr[s1 + n + l];
                    }
                    keep[i] = make_float2(re_mul(w, V1) * f1, re_mul(w, V2) * f2);
                }
            }
        }
        if (mode == 1) {  // the coefficients over the rows this workgroup read
#pragma unroll
            for (int i = 0; i < FFT_EPT; ++i) {
                const int idx = threadIdx.x + i * kBlock;
                if (idx < total) {
                    const int q = idx / n;
                    const int l = idx - q * n;
                    const size_t r1 = (size_t)(2 * (p0 + q)) * ts;
                    Tr[r1 + l] = keep[i].x;
                    Tr[r1 + ts + l] = keep[i].y;
                }
            }
            return;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < total) buf[lds_slot(idx)] = keep[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < total) {
            const int q = idx / n;
            const int l = idx - q * n;
            const float2 Y = buf[lds_slot(q * n + l)];
            const float2 Yr = (l == 0) ? make_float2(0.0f, 0.0f) : buf[lds_slot(q * n + n - l)];
            const float2 wc = cconj(dtw[l]);
            const float2 V1 = cmul(wc, make_float2(Y.x, -Yr.x));
            const float2 V2 = cmul(wc, make_float2(Y.y, -Yr.y));
            keep[i] = make_float2(V1.x - V2.y, V1.y + V2.x);  // V1 + i V2
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < total) buf[lds_slot(idx)] = keep[i];
    }
    __syncthreads();
    lds_fft_any<1, NT>(buf, fd, cp, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < total; idx += kBlock) {
        const int q = idx / n;
        const int l = idx - q * n;
        const size_t r1 = (size_t)(2 * (p0 + q)) * ts;
        const float2 v = buf[lds_slot(q * n + dct_perm(l, n))];
        Tr[r1 + l] = v.x;
        Tr[r1 + ts + l] = v.y;
    }
}

template <int NT = 0>
__device__ __forceinline__ void dct_rows_inv_body(const float* __restrict__ Tr, int n_, int ts,
                                                              float* __restrict__ dst, const FftDesc& fd,
                                                              const float2* __restrict__ tw,
                                                              const float2* __restrict__ dtw, int G_, int seq_shift, int blk, float2* buf,
                                                              int accum = 0) {
    const int n = NT > 0 ? NT : n_;
    const int G = NT > 0 ? 1 : G_;
    const int row0 = blk * 2 * G;
    const int total = G * n;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        total,
        [&](int idx) {
            const int k = idx / G;
            const int g = idx - k * G;
            return *reinterpret_cast<const float2*>(Tr + (size_t)k * ts + row0 + 2 * g);
        },
        [&](int idx, float2 v) {
            const int k = idx / G;
            buf[lds_slot((idx - k * G) * n + k)] = v;
        });
    __syncthreads();
    float2 keep[FFT_EPT];
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < total) {
            const int g = idx / n;
            const int k = idx - g * n;
            const float2 Y = buf[lds_slot(g * n + k)];
            const float2 Yr = (k == 0) ? make_float2(0.0f, 0.0f) : buf[lds_slot(g * n + n - k)];
            const float2 wc = cconj(dtw[k]);
            const float2 Va = cmul(wc, make_float2(Y.x, -Yr.x));
            const float2 Vb = cmul(wc, make_float2(Y.y, -Yr.y));
            keep[i] = make_float2(Va.x - Vb.y, Va.y + Vb.x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int idx = threadIdx.x + i * kBlock;
        if (idx < total) buf[lds_slot(idx)] = keep[i];
    }
    __syncthreads();
    lds_fft_any<1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < total; idx += kBlock) {
        const int g = idx / n;
        const int x = idx - g * n;
        const size_t ra = (size_t)(row0 + 2 * g) * n;
        const float2 v = buf[lds_slot(g * n + dct_perm(x, n))];
        if (accum) {
            dst[ra + x] += v.x;
            dst[ra + n + x] += v.y;
        } else {
            dst[ra + x] = v.x;
            dst[ra + n + x] = v.y;
        }
    }
}

// ---- Algorithm 4 with the periodic model: the blur inside the transform ----
// For periodic boundary conditions A is the BCCB matrix C of the PSF centred
// at the origin (eigenvalues Lambda_c), so the residual is formed in the
// spectrum: R = F g - Lambda_c F u, and ||r||^2 = sum |R|^2 / n^2 (Parseval;
// the half spectrum counts the columns 0 < k < n/2 twice).  Over CC columns of
// T holding the row transforms of u: forward FFT, R, the partial of ||r||^2
// per workgroup into part[blockIdx.x]; then (store_r == 0) the direction of
// eq. (Alg4), conj(Lambda_c) R inv / (|Lambda|^2 + alpha), inverse FFT, or
// (store_r) R itself, for the 4-NS alpha and the filter that follows.
template <int NT>
__global__ __launch_bounds__(kBlock) void fft_cols_residual_kernel(float2* __restrict__ T, int n_, int ts,
                                                                   const float2* __restrict__ ghat,
                                                                   const float2* __restrict__ lamc,
                                                                   const float* __restrict__ spec, float alpha,
                                                                   float inv, FftDesc fd,
                                                                   const float2* __restrict__ tw, int CC_,
                                                                   int seq_shift, int store_r,
                                                                   double* __restrict__ part) {
    extern __shared__ float2 buf[];
    __shared__ double red[kBlock / 64];
    const int n = NT > 0 ? NT : n_;
    const int CC = NT > 0 ? 1 : CC_;
    const int half = n / 2 + 1;
    const int k0 = blockIdx.x * CC;
    const int cc = min(CC, half - k0);
    const size_t base = (size_t)k0 * n;  // dense [n/2+1][n] spectra
    const double to_r = 1.0 / ((double)n * (double)n);
    if constexpr (NT > 0 && fixed_conv_ok<(NT > 0 ? NT : 1)>()) {  // R and the filter in registers
        FixedTw<NT> twf;
        FixedTw<NT, true> twi;
        fixed_tw_load<NT>(tw, twf.w);
        if (!store_r) fixed_tw_load<NT, 0, true>(tw, twi.w);
        const double wgt = (k0 == 0 || 2 * k0 == n) ? to_r : 2.0 * to_r;
        double ss = 0.0;
        float2* col = T + (size_t)k0 * ts;
        fixed_conv<NT>(
            buf, tw, twf.w, twi.w, [&](int y) { return col[y]; },
            [&](int, int y, float2 v) {
                const float2 L = lamc[base + y];
                const float2 R = csub(ghat[base + y], cmul(L, v));
                ss += wgt * ((double)R.x * (double)R.x + (double)R.y * (double)R.y);
                return store_r ? R : cmul(cscale(R, inv / (spec[base + y] + alpha)), cconj(L));
            },
            [&](int y, float2 v) { col[y] = v; }, store_r != 0);
        const double t = block_sum(ss, red);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
        return;
    }
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        cc * n,
        [&](int idx) {
            const int q = idx / n;
            return T[(size_t)(k0 + q) * ts + (idx - q * n)];
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    double ss = 0.0;
    for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
        const int kx = k0 + idx / n;
        const float2 L = lamc[base + idx];
        const float2 R = csub(ghat[base + idx], cmul(L, buf[lds_slot(idx)]));
        const double wgt = (kx == 0 || 2 * kx == n) ? to_r : 2.0 * to_r;
        ss += wgt * ((double)R.x * (double)R.x + (double)R.y * (double)R.y);
        buf[lds_slot(idx)] = store_r ? R : cmul(cscale(R, inv / (spec[base + idx] + alpha)), cconj(L));
    }
    const double t = block_sum(ss, red);  // its barriers also order the writes above before the transform
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    if (!store_r) lds_fft_any<1, NT>(buf, fd, cc, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    for (int idx = threadIdx.x; idx < cc * n; idx += kBlock) {
        const int q = idx / n;
        T[(size_t)(k0 + q) * ts + (idx - q * n)] = buf[lds_slot(idx)];
    }
}

// ---- Algorithm 2: the PCG step's vector updates in P's row passes --------
// (BCCB plan.)  The forward row pass applies the step's update t += a d,
// res -= a q (a = rho / pq, device doubles; nothing once the CG has stopped)
// to the rows it reads and transforms the new res; the inverse row pass
// writes z = P res with the partial sums of res . z per workgroup.  The
// arithmetic of every value is that of the separate update and dot kernels.
template <int NT>
__global__ __launch_bounds__(kBlock) void pcg_rows_r2c_kernel(int n, float2* __restrict__ T, int ts, FftDesc fd,
                                                              const float2* __restrict__ tw, int G, int seq_shift,
                                                              PcgVec v) {
    extern __shared__ float2 buf[];
    const bool on = *v.act != 0.0;
    const float a = on ? (float)(*v.rho / *v.pq) : 0.0f;
    fft_rows_r2c_body_f<NT>(
        [&](size_t i) {
            if (!on) return v.res[i];
            v.t[i] = fmaf(a, v.d[i], v.t[i]);
            const float r = fmaf(-a, v.q[i], v.res[i]);
            v.res[i] = r;
            return r;
        },
        n, T, ts, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void pcg_rows_c2r_kernel(const float2* __restrict__ T, int n, int ts,
                                                              float* __restrict__ z, const float* __restrict__ res,
                                                              FftDesc fd, const float2* __restrict__ tw, int G,
                                                              int seq_shift, double* __restrict__ part) {
    extern __shared__ float2 buf[];
    __shared__ double red[kBlock / 64];
    double acc = 0.0;
    fft_rows_c2r_body_f<NT>(
        T, n, ts,
        [&](size_t i, float val) {
            z[i] = val;
            acc += (double)res[i] * (double)val;
        },
        fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ---- single-image kernels ------------------------------------------------

template <int NT>
__global__ __launch_bounds__(kBlock) void fft_rows_r2c_kernel(const float* __restrict__ src, int n,
                                                              float2* __restrict__ T, int ts, FftDesc fd,
                                                              const float2* __restrict__ tw, int G, int seq_shift) {
    extern __shared__ float2 buf[];
    fft_rows_r2c_body<NT>(src, n, T, ts, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
}

// red_out (optional): workgroup 0 first sums red_count partials of the
// previous launch into *red_out, in the order of the separate reduction.
template <int NT>
__global__ __launch_bounds__(kBlock) void fft_cols_kernel(float2* __restrict__ T, int n, int ts,
                                                          const float* __restrict__ spec, float alpha,
                                                          float inv, FftDesc fd,
                                                          const float2* __restrict__ tw, int CC, int mode,
                                                          float* __restrict__ power, int seq_shift,
                                                          const float2* __restrict__ lamc,
                                                          const double* __restrict__ alpha_dev,
                                                          float2* __restrict__ cspec,
                                                          const double* __restrict__ red_in, int red_count,
                                                          double* __restrict__ red_out) {
    extern __shared__ float2 buf[];
    if (red_out && blockIdx.x == 0) {
        __shared__ double red[kBlock / 64];
        const double acc = strided_sum(red_in, red_count);
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) *red_out = t;
    }
    fft_cols_body<NT>(T, n, ts, spec, alpha, inv, fd, tw, CC, mode, power, seq_shift, blockIdx.x, buf, nullptr,
                      nullptr, nullptr, lamc, alpha_dev, cspec);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void fft_rows_c2r_kernel(const float2* __restrict__ T, int n, int ts,
                                                              float* __restrict__ dst, FftDesc fd,
                                                              const float2* __restrict__ tw, int G, int seq_shift,
                                                              int accum) {
    extern __shared__ float2 buf[];
    fft_rows_c2r_body<NT>(T, n, ts, dst, fd, tw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf, accum);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void dct_rows_fwd_kernel(const float* __restrict__ src, int n,
                                                              float* __restrict__ Tr, int ts, FftDesc fd,
                                                              const float2* __restrict__ tw,
                                                              const float2* __restrict__ dtw, int G, int seq_shift) {
    extern __shared__ float2 buf[];
    dct_rows_fwd_body<NT>(src, n, Tr, ts, fd, tw, dtw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void dct_cols_filter_kernel(float* __restrict__ Tr, int n, int ts,
                                                                 const float* __restrict__ spec, float alpha,
                                                                 float inv, FftDesc fd,
                                                                 const float2* __restrict__ tw,
                                                                 const float2* __restrict__ dtw, int CP, int seq_shift,
                                                                 const float* __restrict__ lamr, int mode,
                                                                 const double* __restrict__ alpha_dev) {
    extern __shared__ float2 buf[];
    dct_cols_filter_body<NT>(Tr, n, ts, spec, alpha, inv, fd, tw, dtw, CP, seq_shift, blockIdx.x, buf, lamr, mode,
                             alpha_dev);
}

template <int NT>
__global__ __launch_bounds__(kBlock) void dct_rows_inv_kernel(const float* __restrict__ Tr, int n, int ts,
                                                              float* __restrict__ dst, FftDesc fd,
                                                              const float2* __restrict__ tw,
                                                              const float2* __restrict__ dtw, int G, int seq_shift,
                                                              int accum) {
    extern __shared__ float2 buf[];
    dct_rows_inv_body<NT>(Tr, n, ts, dst, fd, tw, dtw, G, seq_shift, xcd_block(blockIdx.x, gridDim.x), buf, accum);
}

// Cosine spectra of the symmetrised PSF H~ (reflective blur, Algorithm 3;
// antireflective blur, with the two linear functions at frequency zero):
//   lambda[ky][kx] = sum_a cos(w_ky (a-c)) rows[a][kx],
//   rows[a][kx]    = sum_b H~[a][b] cos(w_kx (b-c)),
// w_k = pi k / K (costab[q] = cos(pi q / K), q < 2K); with lin_last the last
// frequency index K takes w = 0.  Two passes, O(n^2 p) instead of O(n^2 p^2).
__device__ __forceinline__ int cos_freq(int k, int K, int lin_last) { return (lin_last && k == K) ? 0 : k; }

__global__ __launch_bounds__(kBlock) void cos_spectrum_rows_kernel(const float* __restrict__ psf, int p, int n,
                                                                   int K, int lin_last,
                                                                   const float* __restrict__ costab,
                                                                   float* __restrict__ rows) {
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= p * n) return;
    const int a = idx / n;
    const int fx = cos_freq(idx - a * n, K, lin_last);
    const int c = (p - 1) / 2;
    float row = 0.0f;
    for (int b = 0; b < p; ++b) {
        const float hs = 0.25f * (psf[a * p + b] + psf[(p - 1 - a) * p + b] + psf[a * p + (p - 1 - b)] +
                                  psf[(p - 1 - a) * p + (p - 1 - b)]);
        row += hs * costab[mod_pos(fx * (b - c), 2 * K)];
    }
    rows[idx] = row;
}

// written squared into spec[kx][ky] and, when given, as is into lam
__global__ __launch_bounds__(kBlock) void cos_spectrum_cols_kernel(const float* __restrict__ rows, int p, int n,
                                                                   int K, int lin_last,
                                                                   const float* __restrict__ costab,
                                                                   float* __restrict__ spec,
                                                                   float* __restrict__ lam) {
    const int ky = blockIdx.x * kBlock + threadIdx.x;
    const int kx = blockIdx.y;
    if (ky >= n) return;
    const int fy = cos_freq(ky, K, lin_last);
    const int c = (p - 1) / 2;
    float acc = 0.0f;
    for (int a = 0; a < p; ++a) acc += costab[mod_pos(fy * (a - c), 2 * K)] * rows[a * n + kx];
    spec[(size_t)kx * n + ky] = acc * acc;
    if (lam) lam[(size_t)kx * n + ky] = acc;
}

hipError_t launch_cos_spectrum(const float* psf, int p, int n, int K, int lin_last, const float* costab, float* tmp,
                               float* spec, float* lam, hipStream_t s) {
    hipLaunchKernelGGL(cos_spectrum_rows_kernel, dim3((p * n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, psf, p, n,
                       K, lin_last, costab, tmp);
    hipLaunchKernelGGL(cos_spectrum_cols_kernel, dim3((n + kBlock - 1) / kBlock, n), dim3(kBlock), 0, s, tmp, p, n, K,
                       lin_last, costab, spec, lam);
    return hipGetLastError();
}

// the PSF centred at the origin of a zeroed n x n image: H[a][b] at
// ((a - c) mod n, (b - c) mod n) -- the kernel of the periodic-boundary blur
__global__ __launch_bounds__(kBlock) void pad_psf_centred_kernel(const float* __restrict__ psf, int p,
                                                                 float* __restrict__ dst, int n) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (size_t)n * n) return;
    const int y = (int)(i / n), x = (int)(i % n);
    const int c = (p - 1) / 2;
    const int a = (y + c) % n, b = (x + c) % n;  // inverse of the shift
    dst[i] = (a < p && b < p) ? psf[a * p + b] : 0.0f;
}

__global__ __launch_bounds__(kBlock) void pad_psf_kernel(const float* __restrict__ psf, int p,
                                                         float* __restrict__ dst, int n) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (size_t)n * n) return;
    const int y = (int)(i / n), x = (int)(i % n);
    dst[i] = (y < p && x < p) ? psf[y * p + x] : 0.0f;
}

// ---------------------------------------------------------------------------
// Algorithm 4-NS: alpha_n with alpha_n ||(C C^T + alpha_n I)^{-1} r|| = q_n ||r||
// (eq. Alg4_rev_7), solved on the device from the half spectrum of r (T after
// a forward column pass) and s = |Lambda|^2.  By Parseval the equation reads
// h(alpha) = alpha^2 S0(alpha) = q_n^2 R with S0 = sum w / (s + alpha)^2,
// R = sum w, w = |F r|^2 (each x-frequency other than 0 and n/2 stands for
// itself and its conjugate twin, weight 2).  h increases with alpha; Newton on
// log h against log alpha (slope d log h / d log alpha = 2 S1 / S0,
// S1 = sum w s / (s + alpha)^3) with a bracket [lo, hi] that every step
// narrows, falling back to bisection of log alpha when a step leaves it.
// state (device doubles): [0] alpha, [1] log lo, [2] log hi, [3] q_n.
// ---------------------------------------------------------------------------
constexpr int NS_BLOCKS = 512;
constexpr int NS_UNROLL = 8;

// Layout of the 4-NS state buffer (24 doubles): [0, 4) the result
// {alpha, log lo, log hi, q_n}; [4] sum |psf| (written with the PSF); the
// steps' states alternately at [8, 13) and [16, 21) (the four values, then a
// converged flag).
constexpr int NS_L1 = 4;
__host__ __device__ constexpr int ns_buf(int k) { return 8 + 8 * (k & 1); }

// The state after one Newton step from the sums S0, S1, R at st[0] = alpha;
// true once converged: the step stays (r = 0, or h matches to rounding), or
// moves log alpha by less than kNsLogStep.  The sums take alpha in FP32, so a
// step that small is below what they resolve (4 units in the last place of
// an FP32 alpha), and no later step is taken.
constexpr double kNsLogStep = 0x1p-22;
__device__ __forceinline__ bool ns_newton(double* st, double S0, double S1, double R) {
    const double a = st[0], la = log(a);
    double lo = st[1], hi = st[2];
    const double qn = st[3];
    const double h = a * a * S0, target = qn * qn * R;
    const double g = log(h) - log(target);
    if (R <= 0.0 || fabs(g) < 1e-13) return true;
    if (g > 0.0) hi = la; else lo = la;
    const double slope = 2.0 * S1 / S0;
    double t = (slope > 0.0 && isfinite(g)) ? la - g / slope : 0.5 * (lo + hi);
    // a Newton point on the bracket's closed interval is kept (it sits on the
    // end just moved when g is near rounding); outside it, bisect
    if (!(t >= lo && t <= hi)) t = 0.5 * (lo + hi);
    st[0] = exp(t);
    st[1] = lo;
    st[2] = hi;
    return fabs(t - la) < kNsLogStep;
}

// q_n from ||r^n||^2 (rn_sq) and the noise level; bracket [hi 1e-14, hi] with
// hi = q_n smax / (1 - q_n), smax = (sum |H|)^2 >= max |Lambda|^2 (there
// alpha / (s + alpha) >= q_n for every s); start from the previous alpha (a)
// when it lies inside, else from hi / 2.
__device__ __forceinline__ void ns_init(double* st, double a, double rn_sq, double l1, double noise, double q,
                                        double rho) {
    const double smax = l1 * l1;
    const double tau_n = sqrt(rn_sq) / noise;
    const double qn = fmax(q, 2.0 * rho + (1.0 + rho) / tau_n);
    const double hi = qn * smax / (1.0 - qn) * 1.0001 + 1e-30;
    const double lo = hi * 1e-14;
    if (!(a > lo && a < hi)) a = 0.5 * hi;
    st[0] = a;
    st[1] = log(lo);
    st[2] = log(hi);
    st[3] = qn;
}

// sum |psf| in index order (one thread), for the bracket of every iteration
__global__ void ns_psf_l1_kernel(const float* __restrict__ psf, int p, double* __restrict__ state) {
    double l1 = 0.0;
    for (int i = 0; i < p * p; ++i) l1 += fabs((double)psf[i]);
    state[NS_L1] = l1;
}

// The sums S0, S1, R of one step's NS_BLOCKS x 3 partials, in one fixed
// order (the same in every workgroup that forms them); all threads call.
__device__ __forceinline__ void ns_sums(const double* __restrict__ part, double (*red)[kBlock / 64], double* S) {
    double u[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < NS_BLOCKS; b += kBlock)
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] += part[(size_t)b * 3 + q];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x = u[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[q][wid] = x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        S[q] = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) S[q] += red[q][w];
    }
    __syncthreads();
}

struct NsStep {
    const double* rn_sq;
    double noise, q, rho, alpha_first;
    int first;  // start from alpha_first rather than the previous alpha
    int k;      // the step
};

// Newton step k of the 4-NS alpha.  Every workgroup first brings the state
// up to date itself: step 0 starts it (ns_init); a later step takes the
// Newton update of step k-1's state with step k-1's partials (each
// workgroup forms the same sums), unless step k-1 had converged.  Workgroup 0
// stores the state for the next step; unless converged, every workgroup then
// sums S0 = sum w / (s + a)^2, S1 = sum w s / (s + a)^3 and R = sum w over
// its share of the spectrum into this step's partials.
//
// Weights w: the BCCB half spectrum T[kx][ky] (kx <= n/2) counts the columns
// 0 < kx < n/2 twice (Parseval for real r).  REAL: the 2-D DCT-II
// coefficients Tr[kx][ky] (real, n rows) of the DCT plan instead; with the
// unnormalised X_k = sum_j x_j cos(pi k (2j+1) / 2n) the orthonormal
// coefficient is sqrt((2 - [k == 0]) / n) X_k along each axis, so Parseval
// weighs X^2 by (kx ? 2 : 1)(ky ? 2 : 1) (the common 1/n^2 cancels in the
// equation).
template <bool REAL>
__global__ __launch_bounds__(kBlock) void ns_step_kernel(const void* __restrict__ Tv, int n, int ts,
                                                         const float* __restrict__ spec, double* __restrict__ st,
                                                         double* __restrict__ part, NsStep a_) {
    __shared__ double red[3][kBlock / 64];
    __shared__ double stl[5];
    const int k = a_.k;
    if (k == 0) {
        if (threadIdx.x == 0) {
            double v[4];
            ns_init(v, a_.first ? a_.alpha_first : st[0], *a_.rn_sq, st[NS_L1], a_.noise, a_.q, a_.rho);
            for (int i = 0; i < 4; ++i) stl[i] = v[i];
            stl[4] = 0.0;
        }
    } else {
        const double* prev = st + ns_buf(k - 1);
        if (prev[4] != 0.0) {
            if (threadIdx.x < 5) stl[threadIdx.x] = prev[threadIdx.x];
        } else {
            double S[3];
            ns_sums(part + (size_t)3 * NS_BLOCKS * ((k - 1) & 1), red, S);
            if (threadIdx.x == 0) {
                double v[4] = {prev[0], prev[1], prev[2], prev[3]};
                const bool stay = ns_newton(v, S[0], S[1], S[2]);
                for (int i = 0; i < 4; ++i) stl[i] = v[i];
                stl[4] = stay ? 1.0 : 0.0;
            }
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < 5) st[ns_buf(k) + threadIdx.x] = stl[threadIdx.x];
    if (stl[4] != 0.0) return;
    double* __restrict__ out = part + (size_t)3 * NS_BLOCKS * (k & 1);
    const float a = (float)stl[0];
    const int rows = REAL ? n : n / 2 + 1;
    const int total = rows * n;
    // a contiguous share of the row-major spectrum per workgroup (a multiple
    // of kBlock elements), NS_UNROLL loads per thread in flight at a time
    const int per = (total + NS_BLOCKS * kBlock - 1) / (NS_BLOCKS * kBlock) * kBlock;
    const int i0 = blockIdx.x * per;
    const int i1 = min(total, i0 + per);
    const float rn = 1.0f / (float)n;
    double s0 = 0.0, s1 = 0.0, rr = 0.0;
    for (int b = i0 + (int)threadIdx.x; b < i1; b += NS_UNROLL * kBlock) {
        using V = typename std::conditional<REAL, float, float2>::type;
        V tv[NS_UNROLL];
        float wf[NS_UNROLL], sk[NS_UNROLL];
#pragma unroll
        for (int u = 0; u < NS_UNROLL; ++u) {
            // past the share's end: reread its last element with weight 0
            const int i = b + u * kBlock;
            const bool ok = i < i1;
            const int ic = ok ? i : i1 - 1;
            // row kx = ic / n: a float estimate (ic < 2^24, off by at most
            // one), then exact
            int kx = (int)((float)ic * rn);
            kx -= kx * n > ic ? 1 : 0;
            kx += (kx + 1) * n <= ic ? 1 : 0;
            const int ky = ic - kx * n;
            if constexpr (REAL) wf[u] = ok ? (kx == 0 ? 1.0f : 2.0f) * (ky == 0 ? 1.0f : 2.0f) : 0.0f;
            else wf[u] = ok ? ((kx == 0 || 2 * kx == n) ? 1.0f : 2.0f) : 0.0f;
            tv[u] = static_cast<const V*>(Tv)[(size_t)kx * ts + ky];
            sk[u] = spec[ic];
        }
        // every load of the batch is issued before the first use
        asm volatile("" ::: "memory");
        float w[NS_UNROLL];
#pragma unroll
        for (int u = 0; u < NS_UNROLL; ++u) {
            if constexpr (REAL) w[u] = wf[u] * (tv[u] * tv[u]);
            else w[u] = wf[u] * (tv[u].x * tv[u].x + tv[u].y * tv[u].y);
        }
#pragma unroll
        for (int u = 0; u < NS_UNROLL; ++u) {  // w = 0 adds exact zeros
            const float id = 1.0f / (sk[u] + a);
            const float t0 = w[u] * id * id;
            s0 += (double)t0;
            s1 += (double)(t0 * sk[u] * id);
            rr += (double)w[u];
        }
    }
    double v[3] = {s0, s1, rr};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[threadIdx.x][w];
        out[(size_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

// The update after the last step: the result to st[0, 4) and hist.
__global__ __launch_bounds__(kBlock) void ns_final_kernel(double* __restrict__ st, const double* __restrict__ part,
                                                          int k_last, double* __restrict__ hist) {
    __shared__ double red[3][kBlock / 64];
    const double* prev = st + ns_buf(k_last);
    double v[4] = {prev[0], prev[1], prev[2], prev[3]};
    if (prev[4] == 0.0) {
        double S[3];
        ns_sums(part + (size_t)3 * NS_BLOCKS * (k_last & 1), red, S);
        ns_newton(v, S[0], S[1], S[2]);
    }
    if (threadIdx.x != 0) return;
    for (int i = 0; i < 4; ++i) st[i] = v[i];
    if (hist) *hist = v[0];
}

// `steps` Newton steps (steps + 1 launches); state: the 24-double buffer
// above (sum |psf| set by launch_ns_psf_l1), part: 2 x 3 NS_BLOCKS doubles.
hipError_t launch_ns_alpha(const void* T, int real, int n, int ts, const float* spec, double* state, double* part,
                           const double* rn_sq, double noise, double q, double rho, double alpha_first, int first,
                           int steps, double* hist, hipStream_t s) {
    if (steps < 1 || (long)(real ? n : n / 2 + 1) * n >= (1L << 24)) return hipErrorInvalidValue;
    for (int k = 0; k < steps; ++k) {
        const NsStep a{rn_sq, noise, q, rho, alpha_first, first, k};
        if (real)
            hipLaunchKernelGGL(ns_step_kernel<true>, dim3(NS_BLOCKS), dim3(kBlock), 0, s, T, n, ts, spec, state, part,
                               a);
        else
            hipLaunchKernelGGL(ns_step_kernel<false>, dim3(NS_BLOCKS), dim3(kBlock), 0, s, T, n, ts, spec, state,
                               part, a);
    }
    hipLaunchKernelGGL(ns_final_kernel, dim3(1), dim3(kBlock), 0, s, state, (const double*)part, steps - 1, hist);
    return hipGetLastError();
}

hipError_t launch_ns_psf_l1(const float* psf, int p, double* state, hipStream_t s) {
    hipLaunchKernelGGL(ns_psf_l1_kernel, dim3(1), dim3(1), 0, s, psf, p, state);
    return hipGetLastError();
}

int ns_partials_needed() { return 2 * 3 * NS_BLOCKS; }
int ns_state_doubles() { return 24; }
int ns_alpha_launches(int steps) { return steps + 1; }

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

// threads per sequence = kBlock / batch (batch a power of two)
static int seq_shift_for(int batch) {
    int sh = 8;  // log2(kBlock)
    while (batch > 1) {
        batch >>= 1;
        --sh;
    }
    return sh;
}

static int pick_pairs_per_block(int n) {
    // two rows per pair; stay within the LDS budget; keep >= ~512 workgroups
    int target = n >= 2048 ? 2 : 1;
    int G = 1;
    if (!smooth235(n)) return 1;  // Bluestein: one sequence per workgroup
    while (G * 2 <= target && (G * 2) * n <= FFT_MAX_ELEMS && ((n / 2) % (G * 2)) == 0) G *= 2;
    return G;
}

static int pick_cols_per_block(int n) {
    if (!smooth235(n)) return 1;
    int cc = 1;  // largest power of two with cc * n <= min(4096, FFT_MAX_ELEMS)
    while ((cc * 2) * n <= FFT_MAX_ELEMS && (cc * 2) * n <= 4096) cc *= 2;
    return cc;
}

int fft_rows_batch(int n) { return pick_pairs_per_block(n); }

bool fft_length_supported(int n) {
    return n >= 1 && (smooth235(n) ? n <= FFT_MAX_ELEMS : bluestein_len(n) <= FFT_MAX_ELEMS);
}

int fft_rows_batch_at_most(int n, int want) {
    int G = 1;
    if (!smooth235(n)) return 1;
    while (G * 2 <= want && (G * 2) * n <= FFT_MAX_ELEMS && ((n / 2) % (G * 2)) == 0) G *= 2;
    return G;
}

int fft_cols_batch_at_most(int n, int want) {
    int cc = 1;
    if (!smooth235(n)) return 1;
    while (cc * 2 <= want && (cc * 2) * n <= FFT_MAX_ELEMS) cc *= 2;
    return cc;
}
int fft_cols_batch(int n) { return pick_cols_per_block(n); }
int fft_seq_shift(int batch) { return seq_shift_for(batch); }

// ---- batched preconditioner passes ---------------------------------------
// Workgroup b serves image bmap[b], block b - bfirst[img] of the given pass.

int precond_pass_tiles(const BatchImage& I, int pass) {
    if (I.precond == 2) return 0;  // P = I: the descriptor aliases t to r
    if (I.precond == 3) return pass == 3 ? 0 : (I.n + 1) / 2;  // antireflective: one row pair per workgroup
    if (pass == 3) pass = 1;
    if (pass != 1) return I.n / (2 * I.fft_rows_g);
    if (I.precond == 0) return (I.n / 2 + 1 + I.fft_cols_c - 1) / I.fft_cols_c;
    return (I.n / 2 + I.fft_cols_c - 1) / I.fft_cols_c;
}

template <int PASS, int PRECOND, int NB>
__global__ __launch_bounds__(kBlock) void precond_batched_kernel(const BatchImage* __restrict__ imgs,
                                                                 const int* __restrict__ bmap,
                                                                 const int* __restrict__ bfirst) {
    extern __shared__ float2 buf[];
    // row passes: consecutive row pairs of an image in one L2 (their transposed
    // stores share cache lines); the column passes keep the launch order
    const int xb = (PASS == 0 || PASS == 2) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int im = bmap[xb];
    const BatchImage& I = imgs[im];
    const int blk = xb - bfirst[im];
    const int n = I.n;
    const float inv = (float)(1.0 / ((double)n * (double)n));
    if constexpr (PRECOND == 3) {  // antireflective transform, one row pair per workgroup
        __shared__ float2 lin[2 * kArMaxBatch];
        float* Tr = (float*)I.swork;
        if (PASS == 0) ar_rows_fwd_body<NB>(I.r, n, Tr, I.ts, I.fd, I.tw, 1, I.fft_rows_shift, blk, buf);
        if (PASS == 1)
            ar_cols_filter_body<NB>(Tr, n, I.ts, I.spec, I.alpha, nullptr, I.fd, I.tw, 1, I.fft_cols_shift, blk, buf,
                                   lin);
        if (PASS == 2) ar_rows_inv_body<NB>(Tr, n, I.ts, I.t, I.fd, I.tw, 1, I.fft_rows_shift, blk, buf, 0);
        return;
    }
    if (PRECOND == 0) {
        float2* T = (float2*)I.swork;
        if (PASS == 0) fft_rows_r2c_body<NB>(I.r, n, T, I.ts, I.fd, I.tw, I.fft_rows_g, I.fft_rows_shift, blk, buf);
        if (PASS == 1)
            fft_cols_body<NB>(T, n, I.ts, I.spec, I.alpha, inv, I.fd, I.tw, I.fft_cols_c, 0, nullptr, I.fft_cols_shift,
                          blk, buf, I.sstore, I.sfwd, I.eacc);
        if (PASS == 2) fft_rows_c2r_body<NB>(T, n, I.ts, I.t, I.fd, I.tw, I.fft_rows_g, I.fft_rows_shift, blk, buf);
        if (PASS == 3)
            fft_cols_inverse_real_body<NB>(I.eacc, T, n, I.ts, I.fd, I.tw, I.fft_cols_c, I.fft_cols_shift, blk, buf);
    } else {
        float* Tr = (float*)I.swork;
        if (PASS == 0)
            dct_rows_fwd_body<NB>(I.r, n, Tr, I.ts, I.fd, I.tw, I.dtw, I.fft_rows_g, I.fft_rows_shift, blk, buf);
        if (PASS == 1)
            dct_cols_filter_body<NB>(Tr, n, I.ts, I.spec, I.alpha, inv, I.fd, I.tw, I.dtw, I.fft_cols_c,
                                 I.fft_cols_shift, blk, buf);
        if (PASS == 2)
            dct_rows_inv_body<NB>(Tr, n, I.ts, I.t, I.fd, I.tw, I.dtw, I.fft_rows_g, I.fft_rows_shift, blk, buf);
    }
}

hipError_t launch_precond_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int pass,
                                  int precond, int nmax, hipStream_t s, int any_len) {
    if (nblocks <= 0) return hipSuccess;
    const size_t lds = lds_bytes(FFT_MAX_ELEMS, nmax);
#define MLBA_PB(PA, PC)                                                                                            \
    do {                                                                                                           \
        if (any_len)                                                                                               \
            hipLaunchKernelGGL((precond_batched_kernel<PA, PC, kAnyLen>), dim3(nblocks), dim3(kBlock), lds, s, imgs, \
                               bmap, bfirst);                                                                      \
        else                                                                                                       \
            hipLaunchKernelGGL((precond_batched_kernel<PA, PC, 0>), dim3(nblocks), dim3(kBlock), lds, s, imgs, bmap, \
                               bfirst);                                                                            \
    } while (0)
    if (precond == 0) {
        if (pass == 0) MLBA_PB(0, 0);
        else if (pass == 1) MLBA_PB(1, 0);
        else if (pass == 2) MLBA_PB(2, 0);
        else MLBA_PB(3, 0);
    } else if (precond == 1) {
        if (pass == 3) return hipErrorInvalidValue;
        if (pass == 0) MLBA_PB(0, 1);
        else if (pass == 1) MLBA_PB(1, 1);
        else MLBA_PB(2, 1);
    } else {
        if (pass == 3) return hipErrorInvalidValue;
        if (pass == 0) MLBA_PB(0, 3);
        else if (pass == 1) MLBA_PB(1, 3);
        else MLBA_PB(2, 3);
    }
#undef MLBA_PB
    return hipGetLastError();
}

hipError_t launch_fft_rows_r2c(const float* src, int n, float2* T, int ts, const FftDesc& fd, const float2* tw,
                               hipStream_t s) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(fft_rows_r2c_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, src, n, T, ts, fd, tw, 1,
                           seq_shift_for(1));
    else if (fd.m > 0)
        hipLaunchKernelGGL(fft_rows_r2c_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, src, n, T, ts, fd, tw, G,
                           seq_shift_for(G));
    else
        hipLaunchKernelGGL(fft_rows_r2c_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, src, n, T, ts, fd, tw, G,
                           seq_shift_for(G));
    return hipGetLastError();
}

static hipError_t launch_cols(float2* T, int n, int ts, const float* spec, float alpha, float inv, const FftDesc& fd,
                              const float2* tw, int mode, float* power, const float2* lamc, const double* alpha_dev,
                              float2* cspec, hipStream_t s, const double* red_in = nullptr, int red_count = 0,
                              double* red_out = nullptr) {
    const int CC = pick_cols_per_block(n);
    const int half = n / 2 + 1;
    const size_t lds = lds_bytes(fft_lds_elems(CC * n, n), n);
    if (n == kFixedN && CC == 1)
        hipLaunchKernelGGL(fft_cols_kernel<kFixedN>, dim3(half), dim3(kBlock), lds, s, T, n, ts, spec, alpha, inv, fd,
                           tw, 1, mode, power, seq_shift_for(1), lamc, alpha_dev, cspec, red_in, red_count, red_out);
    else if (fd.m > 0)
        hipLaunchKernelGGL(fft_cols_kernel<kAnyLen>, dim3((half + CC - 1) / CC), dim3(kBlock), lds, s, T, n, ts, spec,
                           alpha, inv, fd, tw, CC, mode, power, seq_shift_for(CC), lamc, alpha_dev, cspec, red_in,
                           red_count, red_out);
    else
        hipLaunchKernelGGL(fft_cols_kernel<0>, dim3((half + CC - 1) / CC), dim3(kBlock), lds, s, T, n, ts, spec,
                           alpha, inv, fd, tw, CC, mode, power, seq_shift_for(CC), lamc, alpha_dev, cspec, red_in,
                           red_count, red_out);
    return hipGetLastError();
}

hipError_t launch_fft_cols_residual(float2* T, int n, int ts, const float2* ghat, const float2* lamc,
                                    const float* spec, float alpha, float inv, const FftDesc& fd, const float2* tw,
                                    int store_r, double* part, int* n_part, hipStream_t s) {
    const int CC = pick_cols_per_block(n);
    const int half = n / 2 + 1;
    const size_t lds = lds_bytes(fft_lds_elems(CC * n, n), n);
    if (n == kFixedN && CC == 1) {
        *n_part = half;
        hipLaunchKernelGGL(fft_cols_residual_kernel<kFixedN>, dim3(half), dim3(kBlock), lds, s, T, n, ts, ghat, lamc,
                           spec, alpha, inv, fd, tw, 1, seq_shift_for(1), store_r, part);
    } else {
        *n_part = (half + CC - 1) / CC;
        if (fd.m > 0)
            hipLaunchKernelGGL(fft_cols_residual_kernel<kAnyLen>, dim3(*n_part), dim3(kBlock), lds, s, T, n, ts, ghat,
                               lamc, spec, alpha, inv, fd, tw, CC, seq_shift_for(CC), store_r, part);
        else
            hipLaunchKernelGGL(fft_cols_residual_kernel<0>, dim3(*n_part), dim3(kBlock), lds, s, T, n, ts, ghat, lamc,
                               spec, alpha, inv, fd, tw, CC, seq_shift_for(CC), store_r, part);
    }
    return hipGetLastError();
}

hipError_t launch_fft_cols_filter(float2* T, int n, int ts, const float* spec, float alpha, float inv,
                                  const FftDesc& fd, const float2* tw, hipStream_t s, const float2* lamc,
                                  const double* red_in, int red_count, double* red_out) {
    return launch_cols(T, n, ts, spec, alpha, inv, fd, tw, 0, nullptr, lamc, nullptr, nullptr, s, red_in, red_count,
                       red_out);
}

hipError_t launch_fft_cols_forward(float2* T, int n, int ts, const FftDesc& fd, const float2* tw, hipStream_t s) {
    return launch_cols(T, n, ts, nullptr, 0.0f, 1.0f, fd, tw, 3, nullptr, nullptr, nullptr, nullptr, s);
}

hipError_t launch_fft_cols_filter_inverse(float2* T, int n, int ts, const float* spec, const double* alpha_dev,
                                          float inv, const float2* lamc, const FftDesc& fd, const float2* tw,
                                          hipStream_t s) {
    return launch_cols(T, n, ts, spec, 0.0f, inv, fd, tw, 4, nullptr, lamc, alpha_dev, nullptr, s);
}

hipError_t launch_fft_cols_complex(const float2* T, int n, int ts, float2* cspec, const FftDesc& fd,
                                   const float2* tw, hipStream_t s) {
    return launch_cols(const_cast<float2*>(T), n, ts, nullptr, 0.0f, 1.0f, fd, tw, 2, nullptr, nullptr, nullptr, cspec,
                       s);
}

hipError_t launch_fft_cols_power(const float2* T, int n, int ts, float* spec, const FftDesc& fd,
                                 const float2* tw, hipStream_t s) {
    return launch_cols(const_cast<float2*>(T), n, ts, nullptr, 0.0f, 1.0f, fd, tw, 1, spec, nullptr, nullptr, nullptr,
                       s);
}

hipError_t launch_fft_rows_c2r(const float2* T, int n, int ts, float* dst, const FftDesc& fd, const float2* tw,
                               hipStream_t s, int accum) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(fft_rows_c2r_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, T, n, ts, dst, fd, tw, 1,
                           seq_shift_for(1), accum);
    else if (fd.m > 0)
        hipLaunchKernelGGL(fft_rows_c2r_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, T, n, ts, dst, fd, tw, G,
                           seq_shift_for(G), accum);
    else
        hipLaunchKernelGGL(fft_rows_c2r_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, T, n, ts, dst, fd, tw, G,
                           seq_shift_for(G), accum);
    return hipGetLastError();
}

hipError_t launch_pcg_rows_r2c(int n, float2* T, int ts, const FftDesc& fd, const float2* tw, const PcgVec& v,
                               hipStream_t s) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(pcg_rows_r2c_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, n, T, ts, fd, tw, 1,
                           seq_shift_for(1), v);
    else if (fd.m > 0)
        hipLaunchKernelGGL(pcg_rows_r2c_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, n, T, ts, fd, tw, G,
                           seq_shift_for(G), v);
    else
        hipLaunchKernelGGL(pcg_rows_r2c_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, n, T, ts, fd, tw, G,
                           seq_shift_for(G), v);
    return hipGetLastError();
}

int pcg_rows_c2r_partials(int n) { return n / (2 * pick_pairs_per_block(n)); }

hipError_t launch_pcg_rows_c2r(const float2* T, int n, int ts, float* z, const float* res, const FftDesc& fd,
                               const float2* tw, double* part, int* n_part, hipStream_t s) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    *n_part = n / (2 * G);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(pcg_rows_c2r_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, T, n, ts, z, res, fd, tw, 1,
                           seq_shift_for(1), part);
    else if (fd.m > 0)
        hipLaunchKernelGGL(pcg_rows_c2r_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, T, n, ts, z, res, fd,
                           tw, G, seq_shift_for(G), part);
    else
        hipLaunchKernelGGL(pcg_rows_c2r_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, T, n, ts, z, res, fd, tw, G,
                           seq_shift_for(G), part);
    return hipGetLastError();
}

hipError_t launch_dct_rows_fwd(const float* src, int n, float* Tr, int ts, const FftDesc& fd, const float2* tw,
                               const float2* dtw, hipStream_t s) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(dct_rows_fwd_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw,
                           dtw, 1, seq_shift_for(1));
    else if (fd.m > 0)
        hipLaunchKernelGGL(dct_rows_fwd_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw,
                           dtw, G, seq_shift_for(G));
    else
        hipLaunchKernelGGL(dct_rows_fwd_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, src, n, Tr, ts, fd, tw,
                           dtw, G, seq_shift_for(G));
    return hipGetLastError();
}

static hipError_t launch_dct_cols(float* Tr, int n, int ts, const float* spec, float alpha, float inv,
                                  const FftDesc& fd, const float2* tw, const float2* dtw, hipStream_t s,
                                  const float* lamr, int mode, const double* alpha_dev) {
    int CP = pick_cols_per_block(n);
    const int pairs = n / 2;
    const size_t lds = lds_bytes(fft_lds_elems(CP * n, n), n);
    if (n == kFixedN && CP == 1)
        hipLaunchKernelGGL(dct_cols_filter_kernel<kFixedN>, dim3(pairs), dim3(kBlock), lds, s, Tr, n, ts, spec, alpha,
                           inv, fd, tw, dtw, 1, seq_shift_for(1), lamr, mode, alpha_dev);
    else if (fd.m > 0)
        hipLaunchKernelGGL(dct_cols_filter_kernel<kAnyLen>, dim3((pairs + CP - 1) / CP), dim3(kBlock), lds, s, Tr, n, ts,
                           spec, alpha, inv, fd, tw, dtw, CP, seq_shift_for(CP), lamr, mode, alpha_dev);
    else
        hipLaunchKernelGGL(dct_cols_filter_kernel<0>, dim3((pairs + CP - 1) / CP), dim3(kBlock), lds, s, Tr, n, ts,
                           spec, alpha, inv, fd, tw, dtw, CP, seq_shift_for(CP), lamr, mode, alpha_dev);
    return hipGetLastError();
}

hipError_t launch_dct_cols_filter(float* Tr, int n, int ts, const float* spec, float alpha, float inv,
                                  const FftDesc& fd, const float2* tw, const float2* dtw, hipStream_t s,
                                  const float* lamr) {
    return launch_dct_cols(Tr, n, ts, spec, alpha, inv, fd, tw, dtw, s, lamr, 0, nullptr);
}

hipError_t launch_dct_cols_forward(float* Tr, int n, int ts, const FftDesc& fd, const float2* tw, const float2* dtw,
                                   hipStream_t s) {
    return launch_dct_cols(Tr, n, ts, nullptr, 0.0f, 1.0f, fd, tw, dtw, s, nullptr, 1, nullptr);
}

hipError_t launch_dct_cols_filter_inverse(float* Tr, int n, int ts, const float* spec, const double* alpha_dev,
                                          float inv, const float* lamr, const FftDesc& fd, const float2* tw,
                                          const float2* dtw, hipStream_t s) {
    return launch_dct_cols(Tr, n, ts, spec, 0.0f, inv, fd, tw, dtw, s, lamr, 2, alpha_dev);
}

hipError_t launch_dct_rows_inv(const float* Tr, int n, int ts, float* dst, const FftDesc& fd, const float2* tw,
                               const float2* dtw, hipStream_t s, int accum) {
    const int G = pick_pairs_per_block(n);
    const size_t lds = lds_bytes(fft_lds_elems(G * n, n), n);
    if (n == kFixedN && G == 1)
        hipLaunchKernelGGL(dct_rows_inv_kernel<kFixedN>, dim3(n / 2), dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw,
                           dtw, 1, seq_shift_for(1), accum);
    else if (fd.m > 0)
        hipLaunchKernelGGL(dct_rows_inv_kernel<kAnyLen>, dim3(n / (2 * G)), dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw,
                           dtw, G, seq_shift_for(G), accum);
    else
        hipLaunchKernelGGL(dct_rows_inv_kernel<0>, dim3(n / (2 * G)), dim3(kBlock), lds, s, Tr, n, ts, dst, fd, tw,
                           dtw, G, seq_shift_for(G), accum);
    return hipGetLastError();
}

hipError_t launch_pad_psf_centred(const float* psf, int p, float* dst, int n, hipStream_t s) {
    const size_t tot = (size_t)n * n;
    hipLaunchKernelGGL(pad_psf_centred_kernel, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, psf,
                       p, dst, n);
    return hipGetLastError();
}

hipError_t launch_pad_psf(const float* psf, int p, float* dst, int n, hipStream_t s) {
    const size_t tot = (size_t)n * n;
    hipLaunchKernelGGL(pad_psf_kernel, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, psf, p,
                       dst, n);
    return hipGetLastError();
}

}  // namespace mlba
