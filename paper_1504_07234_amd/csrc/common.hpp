// Shared device helpers for the MLBA library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlba {

constexpr int kBlock = 256;  // threads per workgroup for every kernel here

// Boundary extension applied when a kernel reads outside [0, S):
//   EXT_ZERO     value 0
//   EXT_REFLECT  half-sample mirror, position x -> s or 2S-1-s, s = x mod 2S
//   EXT_PERIODIC position x -> x mod S
//   EXT_ANTIREFLECT along each axis position -i -> 2 v[0] - v[i] and
//                S-1+i -> 2 v[S-1] - v[S-1-i] (section 2.2); a corner is
//                antireflected along one axis and then the other.  Positions
//                further out than S-1 are clamped (they feed no output).
enum Ext : int { EXT_ZERO = 0, EXT_REFLECT = 1, EXT_PERIODIC = 2, EXT_ANTIREFLECT = 3 };

__device__ __forceinline__ int mod_pos(int x, int m) {
    int r = x % m;
    return r < 0 ? r + m : r;
}

// Reflected index; *flipped is set when the position lands on a mirrored copy.
// Positions within one length of the image (the usual halos) need no modulo.
__device__ __forceinline__ int reflect_index(int x, int S, bool* flipped) {
    if (x >= -S && x < 2 * S) {
        *flipped = x < 0 || x >= S;
        return x < 0 ? -1 - x : (x >= S ? 2 * S - 1 - x : x);
    }
    int s = mod_pos(x, 2 * S);
    *flipped = s >= S;
    return *flipped ? 2 * S - 1 - s : s;
}

__device__ __forceinline__ int reflect_index(int x, int S) {
    if (x >= -S && x < 2 * S) return x < 0 ? -1 - x : (x >= S ? 2 * S - 1 - x : x);
    int s = mod_pos(x, 2 * S);
    return s >= S ? 2 * S - 1 - s : s;
}

// One axis of the antireflective pad: the value at position x is
// wa * v[ia] + wb * v[ib].
__device__ __forceinline__ void antireflect_axis(int x, int S, int* ia, int* ib, float* wa, float* wb) {
    if (x >= 0 && x < S) {
        *ia = *ib = x;
        *wa = 1.0f;
        *wb = 0.0f;
        return;
    }
    const int e = x < 0 ? 0 : S - 1;
    *ia = e;
    *ib = min(max(2 * e - x, 0), S - 1);
    *wa = 2.0f;
    *wb = -1.0f;
}

__device__ __forceinline__ float fetch_antireflect(const float* __restrict__ src, int S, int y, int x) {
    int ya, yb, xa, xb;
    float wya, wyb, wxa, wxb;
    antireflect_axis(y, S, &ya, &yb, &wya, &wyb);
    antireflect_axis(x, S, &xa, &xb, &wxa, &wxb);
    const float* ra = src + (size_t)ya * S;
    const float* rb = src + (size_t)yb * S;
    return wya * (wxa * ra[xa] + wxb * ra[xb]) + wyb * (wxa * rb[xa] + wxb * rb[xb]);
}

// Read src[y][x] of an S x S image under extension `ext`.
__device__ __forceinline__ float fetch_ext(const float* __restrict__ src, int S, int y, int x, int ext) {
    if (y >= 0 && y < S && x >= 0 && x < S) return src[(size_t)y * S + x];
    if (ext == EXT_ZERO) return 0.0f;
    if (ext == EXT_PERIODIC) return src[(size_t)mod_pos(y, S) * S + mod_pos(x, S)];
    if (ext == EXT_ANTIREFLECT) return fetch_antireflect(src, S, y, x);
    return src[(size_t)reflect_index(y, S) * S + reflect_index(x, S)];
}

// Soft threshold of eq. (soft), scaled: delta * sgn(v) * max(|v| - mu, 0),
// written as delta * (v - median(-mu, v, mu)): the same value in every case
// (v - mu and v + mu are the differences the sign form rounds), and a tie
// |v| == mu gives 0.
__device__ __forceinline__ float shrink(float v, float mu, float delta) {
    return (v - __builtin_amdgcn_fmed3f(v, -mu, mu)) * delta;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2.  Renumbering so that every XCD processes one
// contiguous range of logical blocks keeps neighbouring blocks (which share
// cache lines or halos) in the same L2.  A bijection of [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = b % kXcds, s = b / kXcds;
    return x * per + min(x, rem) + s;
}

// The (x, y) tile of a 2-D grid after the XCD renumbering of the linear block
// index (row-major tiles: each XCD takes a band of consecutive tile rows).
__device__ __forceinline__ void xcd_tile(int* bx, int* by) {
    const int gx = (int)gridDim.x;
    const int l = xcd_block((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    *by = l / gx;
    *bx = l - *by * gx;
}

// Wave-level then workgroup-level sum of a double (blockDim.x == kBlock).
__device__ __forceinline__ double block_sum(double v, double* smem /* >= kBlock/64 */) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += smem[i];
    }
    __syncthreads();
    return t;  // valid in thread 0
}

}  // namespace mlba
