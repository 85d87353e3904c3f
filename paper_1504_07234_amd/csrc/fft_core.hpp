// In-LDS mixed-radix (8, 4, 2, 3, 5) Stockham autosort FFT shared by the
// spectral preconditioners and the FFT blur.  Every thread carries up to EPT
// complex values per stage in registers between the read and the write
// barrier; twiddles come from a table of exp(-2 pi i q / n) computed in
// double precision on the host.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace mlba {

constexpr int FFT_EPT = 8;  // complex values per thread per stage (max)

// Lengths with a compiled fixed-size transform (one sequence per workgroup):
// the preconditioner of the 2048 observation, and the FFT-blur grid of that
// observation (the smallest admissible grid for PSFs of 17..227 taps).
constexpr int kFixedN = 2048;
constexpr int kFixedM = 2304;
constexpr int kFixedM2 = 1152;  // the FFT-blur grid of ~1K images (unknowns of 1025..1152)
constexpr int FFT_MAX_ELEMS = FFT_EPT * kBlock;  // complex values per workgroup (16 KB of LDS)

// n = 2^a 3^b 5^c: a Stockham plan of n itself; otherwise the Bluestein form
// over bluestein_len(n), the smallest such length >= 2n - 1.
__host__ __device__ constexpr bool smooth235(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

__host__ __device__ constexpr int bluestein_len(int n) {
    int m = 2 * n - 1;
    while (!smooth235(m)) ++m;
    return m;
}

// LDS elements a pass needs for `elems` values of length-n sequences (a
// Bluestein length transforms in place over m slots, one sequence per
// workgroup).
__host__ __device__ constexpr int fft_lds_elems(int elems, int n) {
    return smooth235(n) ? elems : (elems > bluestein_len(n) ? elems : bluestein_len(n));
}

// LDS slot of element i: one padding slot after every kLdsPad elements (0:
// none), so that the power-of-two strides of the Stockham writes do not pile
// onto one bank.
#ifndef MLBA_LDS_PAD
#define MLBA_LDS_PAD 16
#endif
constexpr int kLdsPad = MLBA_LDS_PAD;
static_assert(kLdsPad == 0 || (kLdsPad & (kLdsPad - 1)) == 0, "LDS padding period: a power of two");
// padding slots before element c (c >= 0)
__host__ __device__ constexpr int lds_pad_of(int c) { return kLdsPad ? (int)((unsigned)c / kLdsPad) : 0; }
// slot(i + c) == slot(i) + c + lds_pad_of(c) for every i when this holds
__host__ __device__ constexpr bool lds_pad_aligned(int c) { return kLdsPad == 0 || c % kLdsPad == 0; }
__host__ __device__ __forceinline__ int lds_slot(int i) { return i + lds_pad_of(i); }
__host__ __device__ constexpr int lds_data_slots(int elems) { return elems + lds_pad_of(elems) + 1; }
__host__ __device__ constexpr size_t lds_bytes(int elems, int n) { return (size_t)lds_data_slots(elems) * 8 + 0 * n; }

// One strided pass of kBlock threads over `count` elements, element
// e = k * kBlock + tid (tid: the thread's index among them, by default
// threadIdx.x): fetch(e) for every element of the thread
// first, then put(e, value).  With a compile-time COUNT > 0 the pass is
// unrolled, so a thread's global loads are all in flight together (one
// memory round trip instead of one per element); COUNT == 0 takes `count`
// at run time and fetches four elements per round trip.
template <int COUNT, typename V, typename Fetch, typename Put>
__device__ __forceinline__ void strided_copy(int count, Fetch fetch, Put put, int tid = threadIdx.x) {
    if constexpr (COUNT > 0) {
        constexpr int PER = (COUNT + kBlock - 1) / kBlock;
        V v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = k * kBlock + tid;
            if (COUNT % kBlock == 0 || e < COUNT) v[k] = fetch(e);
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = k * kBlock + tid;
            if (COUNT % kBlock == 0 || e < COUNT) put(e, v[k]);
        }
    } else {
        for (int e0 = tid; e0 < count; e0 += 4 * kBlock) {
            V v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * kBlock;
                if (e < count) v[u] = fetch(e);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * kBlock;
                if (e < count) put(e, v[u]);
            }
        }
    }
}

// Sum of p[i] over i = threadIdx.x, threadIdx.x + kBlock, ... < count, added
// in that order (the order of a plain strided loop); four loads in flight at
// a time.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int count) {
    double acc = 0.0;
    for (int i0 = threadIdx.x; i0 < count; i0 += 4 * kBlock) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * kBlock;
            v[u] = i < count ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u];
    }
    return acc;
}

template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int q) {
    const float2 w = tw[q];
    return DIR < 0 ? w : make_float2(w.x, -w.y);
}

// Table entries a radix-R butterfly reads: W^e, W^2e, W^4e, W^8e, the first
// tw_table_loads(R) of them.
__host__ __device__ constexpr int tw_table_loads(int R) {
    return R == 16 || R == 9 ? 4 : (R == 8 || R == 5 ? 3 : (R == 4 || R == 3 ? 2 : 1));
}

// w[r] = W^(r*e) for r = 1..R-1 from the table entries raw[t] = tw[2^t e]
// (W = exp(DIR 2 pi i / n), e = jm * step).  Powers 1, 2, 4, 8 come from the
// table; the others are one product away.
template <int R, int DIR>
__device__ __forceinline__ void twiddle_powers_raw(const float2* raw, float2* w) {
    auto pw = [&](int t) { return DIR < 0 ? raw[t] : make_float2(raw[t].x, -raw[t].y); };
    w[1] = pw(0);
    if constexpr (R >= 3) w[2] = pw(1);
    if constexpr (R >= 4) w[3] = cmul(w[1], w[2]);
    if constexpr (R == 5) w[4] = pw(2);
    if constexpr (R >= 8) {
        w[4] = pw(2);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
    }
    if constexpr (R == 9) w[8] = pw(3);
    if constexpr (R == 16) {
        w[8] = pw(3);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
    }
}

template <int R, int DIR>
__device__ __forceinline__ void twiddle_powers(const float2* __restrict__ tw, int e, int n, float2* w) {
    constexpr int T = tw_table_loads(R);
    float2 raw[T];
#pragma unroll
    for (int t = 0; t < T; ++t) raw[t] = tw[e << t];
    twiddle_powers_raw<R, DIR>(raw, w);
}

// a * (DIR i)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2* v) {
    const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const float2 s13 = cadd(v[1], v[3]), d13 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <int DIR>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
    const float s3 = 0.86602540378443865f;  // sqrt(3)/2
    const float2 t = cadd(b, c);
    const float2 d = cscale(mul_i<DIR>(csub(b, c)), s3);
    const float2 m = make_float2(a.x - 0.5f * t.x, a.y - 0.5f * t.y);
    a = cadd(a, t);
    b = cadd(m, d);
    c = csub(m, d);
}

// exp(DIR 2 pi i q / 16) and exp(DIR 2 pi i q / 9)
template <int DIR>
__device__ __forceinline__ float2 w16(int q) {
    const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    const float sg = (float)DIR;
    switch (q) {
        case 1: return make_float2(c1, sg * s1);
        case 2: return make_float2(h, sg * h);
        case 3: return make_float2(s1, sg * c1);
        case 4: return make_float2(0.0f, sg);
        case 6: return make_float2(-h, sg * h);
        default: return make_float2(-c1, -sg * s1);  // q == 9
    }
}

template <int DIR>
__device__ __forceinline__ float2 w9(int q) {
    const float sg = (float)DIR;
    switch (q) {
        case 1: return make_float2(0.76604444311897804f, sg * 0.64278760968653933f);
        case 2: return make_float2(0.17364817766693035f, sg * 0.98480775301220806f);
        default: return make_float2(-0.93969262078590838f, sg * 0.34202014332566873f);  // q == 4
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 16) {
        // 4 x 4: n = k1 + 4 n2, k = m + 4 j
        float2 y[4][4];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 t[4] = {v[k1], v[k1 + 4], v[k1 + 8], v[k1 + 12]};
            dft4<DIR>(t);
#pragma unroll
            for (int m = 0; m < 4; ++m) y[k1][m] = (k1 == 0 || m == 0) ? t[m] : cmul(t[m], w16<DIR>(k1 * m));
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            float2 t[4] = {y[0][m], y[1][m], y[2][m], y[3][m]};
            dft4<DIR>(t);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[m + 4 * j] = t[j];
        }
    } else if constexpr (R == 9) {
        // 3 x 3: n = k1 + 3 n2, k = m + 3 j
        float2 y[3][3];
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            float2 a = v[k1], b = v[k1 + 3], c = v[k1 + 6];
            dft3<DIR>(a, b, c);
            y[k1][0] = a;
            y[k1][1] = k1 == 0 ? b : cmul(b, w9<DIR>(k1));
            y[k1][2] = k1 == 0 ? c : cmul(c, w9<DIR>(2 * k1));
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float2 a = y[0][m], b = y[1][m], c = y[2][m];
            dft3<DIR>(a, b, c);
            v[m] = a;
            v[m + 3] = b;
            v[m + 6] = c;
        }
    } else if constexpr (R == 2) {
        const float2 t = v[0];
        v[0] = cadd(t, v[1]);
        v[1] = csub(t, v[1]);
    } else if constexpr (R == 3) {
        const float s3 = 0.86602540378443865f;  // sqrt(3)/2
        const float2 t = cadd(v[1], v[2]);
        const float2 d = cscale(mul_i<DIR>(csub(v[1], v[2])), s3);
        const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, d);
        v[2] = csub(m, d);
    } else if constexpr (R == 4) {
        dft4<DIR>(v);
    } else if constexpr (R == 5) {
        // X_k = sum_j x_j W^{jk}, W = exp(DIR 2 pi i / 5): pair the inputs j and
        // 5 - j (cosines on their sums, sines on their differences)
        const float c1 = 0.30901699437494742f, s1 = 0.95105651629515357f;   // cos, sin(2 pi / 5)
        const float c2 = -0.80901699437494742f, s2 = 0.58778525229247313f;  // cos, sin(4 pi / 5)
        const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        const float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        const float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        const float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        const float2 b1 = mul_i<DIR>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
        const float2 b2 = mul_i<DIR>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else {  // R == 8: two length-4 transforms and the eighth-root twiddles
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        dft4<DIR>(e);
        dft4<DIR>(o);
        const float h = 0.70710678118654752f;
        const float sg = (float)DIR;
        const float2 o1 = make_float2(h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x));
        const float2 o2 = mul_i<DIR>(o[2]);
        const float2 o3 = make_float2(h * (-o[3].x - sg * o[3].y), h * (-o[3].y + sg * o[3].x));
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
}

// One Stockham stage of radix R.  The workgroup holds up to kBlock >> seq_shift
// sequences of length n back to back in `buf`; sequence b is owned by the
// 2^seq_shift threads with threadIdx.x >> seq_shift == b (only the first nseq
// sequences are live).  Ns is the product of the radices already applied;
// ns_shift = log2(Ns) when Ns is a power of two (every radix-2/4/8 stage,
// since radix-3 and radix-5 stages run last), -1 otherwise.
template <int R, int DIR, int EPT = FFT_EPT>
__device__ __forceinline__ void stockham_stage(float2* buf, int n, int nseq, int seq_shift, int Ns,
                                               int ns_shift, const float2* __restrict__ tw) {
    constexpr int MAXB = (EPT + R - 1) / R;
    const int nb = n / R;
    const int nthr = 1 << seq_shift;
    const int b = threadIdx.x >> seq_shift;
    const int tl = threadIdx.x & (nthr - 1);
    const bool live = b < nseq;
    const int step = n / (Ns * R);
    const int base0 = b * n;
    float2 v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = tl + i * nthr;
        if (live && j < nb) {
            const int jm = ns_shift >= 0 ? (j & (Ns - 1)) : (j % Ns);
            // W^0 = 1 exactly, so butterflies with jm == 0 take the same
            // products (a per-lane skip would only add branches)
            float2 w[R];
            if (Ns > 1) twiddle_powers<R, DIR>(tw, jm * step, n, w);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = buf[lds_slot(base0 + j + r * nb)];
                if (r > 0 && Ns > 1) x = cmul(x, w[r]);
                v[i][r] = x;
            }
            dft<R, DIR>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = tl + i * nthr;
        if (live && j < nb) {
            const int jm = ns_shift >= 0 ? (j & (Ns - 1)) : (j % Ns);
            const int dst = base0 + (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[lds_slot(dst + r * Ns)] = v[i][r];
        }
    }
    __syncthreads();
}

// In-LDS transform of nseq sequences; DIR = -1 forward, +1 inverse
// (unnormalised).  Each sequence's 2^seq_shift threads carry at most EPT
// complex values per stage, so n <= EPT << seq_shift.  The caller synchronises
// before the call.
template <int DIR, int EPT = FFT_EPT>
__device__ __forceinline__ void lds_stockham(float2* buf, int len, const FftDesc& fd, int nseq, int seq_shift,
                             const float2* __restrict__ tw) {
    int Ns = 1, ns_shift = 0;
    for (int s = 0; s < fd.nst; ++s) {
        const int R = fd.radix[s];
        if (R == 8) stockham_stage<8, DIR, EPT>(buf, len, nseq, seq_shift, Ns, ns_shift, tw);
        else if (R == 4) stockham_stage<4, DIR, EPT>(buf, len, nseq, seq_shift, Ns, ns_shift, tw);
        else if (R == 2) stockham_stage<2, DIR, EPT>(buf, len, nseq, seq_shift, Ns, ns_shift, tw);
        else if (R == 3) stockham_stage<3, DIR, EPT>(buf, len, nseq, seq_shift, Ns, ns_shift, tw);
        else stockham_stage<5, DIR, EPT>(buf, len, nseq, seq_shift, Ns, ns_shift, tw);
        Ns *= R;
        ns_shift = (R == 3 || R == 5 || ns_shift < 0) ? -1 : ns_shift + (R == 8 ? 3 : (R == 4 ? 2 : 1));
    }
}

// Length-n DFT of the one sequence in buf[0, n) by Bluestein's identity
// jk = (j^2 + k^2 - (k - j)^2) / 2:
//   X_k = c_k sum_j (x_j c_j) conj(c_{k-j}),  c_k = exp(-i pi k^2 / n),
// the sum a circular convolution of length m >= 2n - 1 done with two m-point
// transforms and the stored spectrum of conj(c) (scaled by 1/m).  The inverse
// direction is conj(DFT(conj x)).  buf holds m slots; every thread of the
// workgroup takes part (m <= FFT_MAX_ELEMS).
template <int DIR, int EPT = FFT_EPT>
__device__ void lds_bluestein(float2* buf, const FftDesc& fd, const float2* __restrict__ tw) {
    constexpr int KE = FFT_MAX_ELEMS / kBlock;
    const int n = fd.n, m = fd.m;
    const float2* __restrict__ chirp = tw + m;
    const float2* __restrict__ bspec = tw + m + n;
    float2 a[KE];
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        a[j] = make_float2(0.0f, 0.0f);
        if (k < n) {
            float2 x = buf[lds_slot(k)];
            if (DIR > 0) x.y = -x.y;
            a[j] = cmul(x, chirp[k]);
        }
    }
    __syncthreads();  // every x read before the zero padding overwrites it
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        if (k < m) buf[lds_slot(k)] = a[j];
    }
    __syncthreads();
    lds_stockham<-1, EPT>(buf, m, fd, 1, 8, tw);
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        if (k < m) buf[lds_slot(k)] = cmul(buf[lds_slot(k)], bspec[k]);
    }
    __syncthreads();
    lds_stockham<1, EPT>(buf, m, fd, 1, 8, tw);
#pragma unroll
    for (int j = 0; j < KE; ++j) {
        const int k = (int)threadIdx.x + j * kBlock;
        if (k < n) {
            float2 v = cmul(buf[lds_slot(k)], chirp[k]);
            if (DIR > 0) v.y = -v.y;
            buf[lds_slot(k)] = v;
        }
    }
    __syncthreads();
}

// run-time 2/3/5-smooth lengths
template <int DIR, int EPT = FFT_EPT>
__device__ __forceinline__ void lds_fft(float2* buf, const FftDesc& fd, int nseq, int seq_shift, const float2* __restrict__ tw) {
    lds_stockham<DIR, EPT>(buf, fd.n, fd, nseq, seq_shift, tw);
}

// Template argument of the pass bodies and kernels for a run-time length that
// may take the Bluestein form (fd.m > 0); NT == 0 compiles the plain
// Stockham plan only, which keeps the Bluestein code (and its registers) out
// of the kernels that serve 2/3/5-smooth lengths.
constexpr int kAnyLen = -1;

// ---- fixed-size transforms ------------------------------------------------
// The same Stockham stages with the length known at compile time and one
// sequence per workgroup (kBlock threads): every index, stride and loop bound
// folds to a constant, and the plan may use radix-16 and radix-9 butterflies
// (fewer passes through LDS than the run-time plan's 8/4/2/3/5).
struct FixedPlan {
    int nst;
    int radix[24];
    int ns[24];
};

// Radices 16 (then 8, 4, 2) for the power of two and 9 (then 3) for the
// power of three: the fewest passes through LDS.
__host__ __device__ constexpr FixedPlan fixed_plan(int n) {
    FixedPlan p{};
    int a = 0, b = 0, m = n;
    while (m % 2 == 0) {
        m /= 2;
        ++a;
    }
    while (m % 3 == 0) {
        m /= 3;
        ++b;
    }
    while (a >= 4 && a != 5 && a != 6) {  // 32 = 8 4 and 64 = 8 8 keep two balanced stages
        p.radix[p.nst++] = 16;
        a -= 4;
    }
    while (a >= 3) {
        p.radix[p.nst++] = 8;
        a -= 3;
    }
    if (a == 2) p.radix[p.nst++] = 4;
    if (a == 1) p.radix[p.nst++] = 2;
    while (b >= 2) {
        p.radix[p.nst++] = 9;
        b -= 2;
    }
    if (b == 1) p.radix[p.nst++] = 3;
    int ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        p.ns[s] = ns;
        ns *= p.radix[s];
    }
    return p;
}

// The same radices in reverse order (the plan of the inverse transform in
// fixed_conv: its first butterflies take the forward transform's last
// outputs from registers).
__host__ __device__ constexpr FixedPlan fixed_plan(int n, bool rev) {
    const FixedPlan f = fixed_plan(n);
    if (!rev) return f;
    FixedPlan p{};
    p.nst = f.nst;
    int ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        p.radix[s] = f.radix[f.nst - 1 - s];
        p.ns[s] = ns;
        ns *= p.radix[s];
    }
    return p;
}

// Table entries of every stage of the fixed plan of length N, per thread:
// stage S (NS > 1) holds MAXB x tw_table_loads(R) of them from offset
// fixed_tw_offset(N, S).
__host__ __device__ constexpr int fixed_tw_offset(int N, int S, bool rev = false) {
    const FixedPlan P = fixed_plan(N, rev);
    int off = 0;
    for (int s = 0; s < S && s < P.nst; ++s)
        if (P.ns[s] > 1) off += ((N / P.radix[s] + kBlock - 1) / kBlock) * tw_table_loads(P.radix[s]);
    return off;
}

template <int N, bool REV = false>
struct FixedTw {
    static constexpr int kCount = fixed_tw_offset(N, 24, REV);
    float2 w[kCount > 0 ? kCount : 1];
};

// Loads the table entries of every stage (one batch, in flight with the
// pass's data loads); both directions use them (DIR +1 conjugates).
template <int N, int S = 0, bool REV = false>
__device__ __forceinline__ void fixed_tw_load(const float2* __restrict__ tw, float2* out, int tid = threadIdx.x) {
    constexpr FixedPlan P = fixed_plan(N, REV);
    if constexpr (S < P.nst) {
        constexpr int R = P.radix[S], NS = P.ns[S];
        if constexpr (NS > 1) {
            constexpr int nb = N / R, MAXB = (nb + kBlock - 1) / kBlock, T = tw_table_loads(R);
            constexpr int step = N / (NS * R), off = fixed_tw_offset(N, S, REV);
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                const int j = tid + i * kBlock;
                if (nb % kBlock == 0 || j < nb) {
                    const int e = (j % NS) * step;
#pragma unroll
                    for (int t = 0; t < T; ++t) out[off + i * T + t] = tw[e << t];
                }
            }
        }
        fixed_tw_load<N, S + 1, REV>(tw, out, tid);
    }
}

// pre: the stage's slice of fixed_tw_load's output, or null (table reads).
// LDS addresses: slot(i + c) = slot(i) + c + lds_pad_of(c) whenever c is a
// multiple of the padding period, so when the strides nb and NS are (or
// NS == 1 with R a multiple of it) each butterfly computes one base slot and
// reaches its R values at compile-time offsets (immediate offsets of the LDS
// instructions).
// tid: the thread's index inside the kBlock threads that own the sequence
template <int R, int DIR, int N, int NS>
__device__ __forceinline__ void stockham_stage_fixed(float2* buf, const float2* __restrict__ tw,
                                                     const float2* pre, int tid = threadIdx.x) {
    constexpr int nb = N / R;
    constexpr int MAXB = (nb + kBlock - 1) / kBlock;
    constexpr int step = N / (NS * R);
    constexpr int T = tw_table_loads(R);
    constexpr bool rd_off = lds_pad_aligned(nb);
    constexpr bool wr_off = lds_pad_aligned(NS) || (NS == 1 && lds_pad_aligned(R));
    float2 v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = tid + i * kBlock;
        if (nb % kBlock == 0 || j < nb) {
            const int jm = j % NS;
            float2 w[R];  // jm == 0 multiplies by W^0 = 1 exactly: no per-lane branch
            if constexpr (NS > 1) {
                if (pre) twiddle_powers_raw<R, DIR>(pre + i * T, w);
                else twiddle_powers<R, DIR>(tw, jm * step, N, w);
            }
            const int sb = lds_slot(j);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = rd_off ? buf[sb + r * (nb + lds_pad_of(nb))] : buf[lds_slot(j + r * nb)];
                if (NS > 1 && r > 0) x = cmul(x, w[r]);
                v[i][r] = x;
            }
            dft<R, DIR>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = tid + i * kBlock;
        if (nb % kBlock == 0 || j < nb) {
            const int jm = j % NS;
            const int dst = (j - jm) * R + jm;
            const int sb = lds_slot(dst);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (!wr_off) buf[lds_slot(dst + r * NS)] = v[i][r];
                else if constexpr (NS == 1) buf[sb + r + lds_pad_of(r)] = v[i][r];  // dst = j R, R aligned
                else buf[sb + r * (NS + lds_pad_of(NS))] = v[i][r];
            }
        }
    }
    __syncthreads();
}

// Stages [S, SEND) of the fixed plan (SEND < 0: to the end), LDS to LDS.
template <int DIR, int N, int S = 0, bool REV = false, int SEND = -1>
__device__ __forceinline__ void lds_fft_fixed(float2* buf, const float2* __restrict__ tw, const float2* pre,
                                              int tid = threadIdx.x) {
    constexpr FixedPlan P = fixed_plan(N, REV);
    if constexpr (S < (SEND < 0 ? P.nst : SEND)) {
        constexpr int off = fixed_tw_offset(N, S, REV);
        stockham_stage_fixed<P.radix[S], DIR, N, P.ns[S]>(buf, tw, pre ? pre + off : nullptr, tid);
        lds_fft_fixed<DIR, N, S + 1, REV, SEND>(buf, tw, pre, tid);
    }
}

// ---- transforms whose first and last stages skip LDS ----------------------
// A plan's first stage (NS = 1) reads elements j + r nb (nb = N / R) and
// writes j R + r; its last stage (NS = nb) reads j + r nb and writes
// j + r nb.  So the first stage can take its inputs straight from registers
// (loaded from global memory), and the last stage can leave its outputs in
// registers: thread j then holds the elements j + r nb, r < R.

// The first stage from registers for butterfly j (< nb): v[r] holds
// element j + r nb; DFT, then the write to LDS (j R + r).
template <int R, int DIR, int N>
__device__ __forceinline__ void stage_first_from_regs(float2 (&v)[R], float2* buf, int j) {
    dft<R, DIR>(v);
    const int sb = lds_slot(j * R);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (lds_pad_aligned(R)) buf[sb + r + lds_pad_of(r)] = v[r];
        else buf[lds_slot(j * R + r)] = v[r];
    }
}

// The last stage into registers for butterfly j (< nb): v[r] becomes
// output element j + r nb.  raw: the butterfly's table entries
// (fixed_tw_load), or null to read the table tw.
template <int R, int DIR, int N>
__device__ __forceinline__ void stage_last_to_regs(const float2* buf, const float2* __restrict__ tw,
                                                   const float2* raw, float2 (&v)[R], int j) {
    constexpr int nb = N / R;
    constexpr bool rd_off = lds_pad_aligned(nb);
    float2 w[R];  // twiddles W^(j r) of the length-N transform (W^0 = 1 exactly for j == 0)
    if (raw) twiddle_powers_raw<R, DIR>(raw, w);
    else twiddle_powers<R, DIR>(tw, j, N, w);
    const int sb = lds_slot(j);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float2 x = rd_off ? buf[sb + r * (nb + lds_pad_of(nb))] : buf[lds_slot(j + r * nb)];
        if (r > 0) x = cmul(x, w[r]);
        v[r] = x;
    }
    dft<R, DIR>(v);
}

// fixed_conv applies when the forward plan has two stages or more and its
// last stage has one butterfly per thread (N / R_last == kBlock), so that
// output element y = tid + r kBlock sits in slot r of every thread.
template <int N>
__host__ __device__ constexpr bool fixed_conv_ok() {
    constexpr FixedPlan P = fixed_plan(N);
    return P.nst >= 2 && N / P.radix[P.nst - 1] == kBlock;
}
template <int N>
__host__ __device__ constexpr int fixed_conv_slots() {
    return fixed_plan(N).radix[fixed_plan(N).nst - 1];
}

// Forward transform (DIR -1) of a length-N sequence read by load(y), a
// pointwise op on its spectrum in registers (op(r, y, v) returns the new
// value of element y = tid + r kBlock), and unless `forward_only` the inverse
// transform (DIR +1, the forward radices in reverse order) with each result
// passed to store(y, v); forward_only stores the spectrum after op.  LDS holds
// only the middle stages.  twf / twi: fixed_tw_load of the forward / reversed
// plan.  Every thread of the workgroup calls this (barriers inside).
template <int N, class Load, class Op, class Store>
__device__ __forceinline__ void fixed_conv(float2* buf, const float2* __restrict__ tw, const float2* twf,
                                           const float2* twi, Load load, Op op, Store store, bool forward_only,
                                           int tid = threadIdx.x) {
    static_assert(fixed_conv_ok<N>(), "fixed_conv: plan shape");
    constexpr FixedPlan F = fixed_plan(N), B = fixed_plan(N, true);
    constexpr int R0 = F.radix[0], RL = F.radix[F.nst - 1];
    constexpr int nb0 = N / R0;
    constexpr int offF = fixed_tw_offset(N, F.nst - 1), offB = fixed_tw_offset(N, B.nst - 1, true);
    static_assert(nb0 <= kBlock, "fixed_conv: one first-stage butterfly per thread");
    if (nb0 == kBlock || tid < nb0) {
        float2 v[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = load(tid + r * nb0);
        stage_first_from_regs<R0, -1, N>(v, buf, tid);
    }
    __syncthreads();
    lds_fft_fixed<-1, N, 1, false, F.nst - 1>(buf, tw, twf, tid);
    float2 u[RL];
    stage_last_to_regs<RL, -1, N>(buf, tw, twf ? twf + offF : nullptr, u, tid);
#pragma unroll
    for (int r = 0; r < RL; ++r) u[r] = op(r, tid + r * kBlock, u[r]);
    if (forward_only) {
#pragma unroll
        for (int r = 0; r < RL; ++r) store(tid + r * kBlock, u[r]);
        return;
    }
    __syncthreads();  // the last forward stage's reads before the inverse's writes
    stage_first_from_regs<RL, 1, N>(u, buf, tid);
    __syncthreads();
    lds_fft_fixed<1, N, 1, true, B.nst - 1>(buf, tw, twi, tid);
    if (nb0 == kBlock || tid < nb0) {
        float2 v[R0];
        stage_last_to_regs<R0, 1, N>(buf, tw, twi ? twi + offB : nullptr, v, tid);
#pragma unroll
        for (int r = 0; r < R0; ++r) store(tid + r * nb0, v[r]);
    }
}

// NT > 0: the fixed transform of length NT (one sequence per workgroup),
// with the twiddles of fixed_tw_load in `pre` when given; NT == 0: the
// run-time plan fd over nseq sequences; NT == kAnyLen: that, or the
// Bluestein form when fd.m > 0.
template <int DIR, int NT, int EPT = FFT_EPT>
__device__ __forceinline__ void lds_fft_any(float2* buf, const FftDesc& fd, int nseq, int seq_shift,
                                            const float2* __restrict__ tw, const float2* pre = nullptr) {
    if constexpr (NT > 0) {
        lds_fft_fixed<DIR, NT>(buf, tw, pre);
    } else if constexpr (NT == kAnyLen) {
        if (fd.m > 0) lds_bluestein<DIR, EPT>(buf, fd, tw);  // one sequence per workgroup
        else lds_fft<DIR, EPT>(buf, fd, nseq, seq_shift, tw);
    } else {
        lds_fft<DIR, EPT>(buf, fd, nseq, seq_shift, tw);
    }
}

}  // namespace mlba
