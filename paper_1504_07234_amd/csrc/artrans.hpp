// Device bodies of the antireflective-transform passes (paper sections 2.2
// and 4.3), shared by the single-image kernels (artrans.hip) and the batched
// preconditioner kernel (fft.hip).  The transform and its FFT formulation
// are described in artrans.hip.
#pragma once

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
// NT > 0 (here and in the two bodies below): L == NT with one sequence pair
// per workgroup (G == CP == 1), the compiled fixed-size transform.
template <int NT>
__device__ __forceinline__ void ar_rows_fwd_body(const float* __restrict__ src, int n, float* __restrict__ Tr,
                                                 int ts, const FftDesc& fd, const float2* __restrict__ tw, int G,
                                                 int seq_shift, int blk, float2* buf) {
    const int N = n - 1, L = 2 * N;
    const float invN = 1.0f / (float)N;
    const int row0 = blk * 2 * G;
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        G * L,
        [&](int idx) {
            const int g = idx / L;
            const int k = idx - g * L;
            const int ya = row0 + 2 * g;
            float2 v = make_float2(0.0f, 0.0f);
            if (ya < n) {
                const float* ra = src + (size_t)ya * n;
                v.x = ar_odd_detrended([&](int q) { return ra[q]; }, k, N, invN);
                if (ya + 1 < n) v.y = ar_odd_detrended([&](int q) { return ra[n + q]; }, k, N, invN);
            }
            return v;
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
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
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        cp * L,
        [&](int idx) {
            const int q = idx / L;
            const int k = idx - q * L;
            const int ja = 2 * (p0 + q);
            const float* ra = Tr + (size_t)ja * ts;
            float2 v;
            v.x = ar_odd_detrended([&](int i) { return ra[i]; }, k, N, invN);
            v.y = ja + 1 < n ? ar_odd_detrended([&](int i) { return ra[ts + i]; }, k, N, invN) : 0.0f;
            return v;
        },
        [&](int idx, float2 v) { buf[lds_slot(idx)] = v; });
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
    lds_fft_any<-1, NT>(buf, fd, cp, seq_shift, tw, NT > 0 ? twp.w : nullptr);

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
    lds_fft_any<-1, NT>(buf, fd, cp, seq_shift, tw, NT > 0 ? twp.w : nullptr);
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
    FixedTw<(NT > 0 ? NT : 1)> twp;
    if constexpr (NT > 0) fixed_tw_load<NT>(tw, twp.w);
    strided_copy<NT, float2>(
        G * L,
        [&](int idx) {
            const int k = idx / G;
            const int g = idx - k * G;
            const int ya = row0 + 2 * g;
            float2 v = make_float2(0.0f, 0.0f);
            if (ya < n && k != 0 && k != N) {
                const int kk = k < N ? k : L - k;
                v = *reinterpret_cast<const float2*>(Tr + (size_t)kk * ts + ya);
                if (k > N) v = make_float2(-v.x, -v.y);
            }
            return v;
        },
        [&](int idx, float2 v) {
            const int k = idx / G;
            buf[lds_slot((idx - k * G) * L + k)] = v;
        });
    __syncthreads();
    lds_fft_any<-1, NT>(buf, fd, G, seq_shift, tw, NT > 0 ? twp.w : nullptr);
    auto emit = [&](int g, int x, float2 c0, float2 cN, float2 prev) {
        const int ya = row0 + 2 * g;
        const float2 X = buf[lds_slot(g * L + x)];
        const float t = (float)x * invN;
        const float va = c0.x + (cN.x - c0.x) * t - 0.5f * X.y;
        const float vb = c0.y + (cN.y - c0.y) * t + 0.5f * X.x;
        const size_t oa = (size_t)ya * n + x;
        if (accum) {
            dst[oa] = prev.x + va;
            if (ya + 1 < n) dst[oa + n] = prev.y + vb;
        } else {
            dst[oa] = va;
            if (ya + 1 < n) dst[oa + n] = vb;
        }
    };
    if constexpr (NT > 0) {
        // one row pair: its linear coefficients and the accumulated values
        // loaded as one batch
        const int ya = row0;
        if (ya >= n) return;
        const float2 c0 = *reinterpret_cast<const float2*>(Tr + ya);
        const float2 cN = *reinterpret_cast<const float2*>(Tr + (size_t)N * ts + ya);
        strided_copy<NT / 2 + 1, float2>(
            n,
            [&](int x) {
                float2 prev = make_float2(0.0f, 0.0f);
                if (accum) {
                    const size_t oa = (size_t)ya * n + x;
                    prev.x = dst[oa];
                    if (ya + 1 < n) prev.y = dst[oa + n];
                }
                return prev;
            },
            [&](int x, float2 prev) { emit(0, x, c0, cN, prev); });
    } else {
        for (int idx = threadIdx.x; idx < G * n; idx += kBlock) {
            const int g = idx / n;
            const int x = idx - g * n;
            const int ya = row0 + 2 * g;
            if (ya >= n) continue;
            const float2 c0 = *reinterpret_cast<const float2*>(Tr + ya);
            const float2 cN = *reinterpret_cast<const float2*>(Tr + (size_t)N * ts + ya);
            float2 prev = make_float2(0.0f, 0.0f);
            if (accum) {
                const size_t oa = (size_t)ya * n + x;
                prev.x = dst[oa];
                if (ya + 1 < n) prev.y = dst[oa + n];
            }
            emit(g, x, c0, cN, prev);
        }
    }
}

}  // namespace mlba
