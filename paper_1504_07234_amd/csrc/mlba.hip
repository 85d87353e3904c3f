// C ABI of the MLBA library: plans, per-operator entry points and the
// restoration loop of eq. (MLBA2).  See include/mlba.h for the contract.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"
#include "mlba.h"
#include "plan.hpp"

using namespace mlba;

namespace {
thread_local int g_last_hip = 0;
}

int mlba_internal_last_hip() { return g_last_hip; }
void mlba_internal_set_hip(hipError_t e) { g_last_hip = (int)e; }

namespace {

// n = 2^a 3^b 5^c?
bool factor_235(int n, int* a, int* b, int* c) {
    *a = *b = *c = 0;
    if (n < 1) return false;
    for (; n % 2 == 0; n /= 2) ++*a;
    for (; n % 3 == 0; n /= 3) ++*b;
    for (; n % 5 == 0; n /= 5) ++*c;
    return n == 1;
}

// Run-time plan of a length-n transform (n = 2^a 3^b 5^c): radix 8 stages,
// one radix 4 or 2 stage, then the radix 3 and radix 5 stages.  (Radix 16 and
// 9 stages, as in the compiled plans, measured 3-6 % slower here: with
// several short sequences per workgroup half the threads idle in them and the
// larger butterflies cost occupancy.)
// Any other n takes the Bluestein form over m = bluestein_len(n) (stages of m).
FftDesc fft_desc(int n) {
    FftDesc d{};
    d.n = n;
    int a = 0, b = 0, c = 0;
    if (!factor_235(n, &a, &b, &c)) {
        d.m = bluestein_len(n);
        factor_235(d.m, &a, &b, &c);
    }
    for (; a >= 3; a -= 3) d.radix[d.nst++] = 8;
    if (a == 2) d.radix[d.nst++] = 4;
    if (a == 1) d.radix[d.nst++] = 2;
    for (int i = 0; i < b; ++i) d.radix[d.nst++] = 3;
    for (int i = 0; i < c; ++i) d.radix[d.nst++] = 5;
    return d;
}

// The device table of a run-time plan: exp(-2 pi i q / len) for q < len
// (len = n, or m in the Bluestein form), then for the Bluestein form the
// chirp c_k = exp(-i pi k^2 / n) (k < n) and the m-point DFT of the
// conjugate chirp wrapped onto the m-circle, divided by m; all in double,
// rounded once.
std::vector<float2> fft_table(const FftDesc& d) {
    const double pi = 3.14159265358979323846;
    const int len = d.m > 0 ? d.m : d.n;
    std::vector<float2> t((size_t)len + (d.m > 0 ? (size_t)d.n + d.m : 0));
    for (int q = 0; q < len; ++q) {
        const double ang = -2.0 * pi * (double)q / (double)len;
        t[q] = make_float2((float)cos(ang), (float)sin(ang));
    }
    if (d.m > 0) {
        const int n = d.n, m = d.m;
        std::vector<double> cr(n), ci(n);
        for (int k = 0; k < n; ++k) {  // k^2 mod 2n keeps the angle small
            const long long k2 = ((long long)k * k) % (2LL * n);
            const double ang = -pi * (double)k2 / (double)n;
            cr[k] = cos(ang);
            ci[k] = sin(ang);
            t[len + k] = make_float2((float)cr[k], (float)ci[k]);
        }
        // b_k = conj(c_k) at k and m - k (|k| < n), zero elsewhere
        for (int q = 0; q < m; ++q) {
            double sr = 0.0, si = 0.0;
            for (int k = -(n - 1); k <= n - 1; ++k) {
                const int kk = k < 0 ? -k : k;
                const long long e = ((long long)q * ((k + m) % m)) % m;
                const double ang = -2.0 * pi * (double)e / (double)m;
                const double wr = cos(ang), wi = sin(ang);
                sr += cr[kk] * wr + ci[kk] * wi;  // conj(c) * w
                si += cr[kk] * wi - ci[kk] * wr;
            }
            t[len + n + q] = make_float2((float)(sr / m), (float)(si / m));
        }
    }
    return t;
}

}  // namespace

FftDesc mlba_internal_fft_desc(int n) { return fft_desc(n); }

namespace {

int dalloc(mlba_plan_s* P, void** ptr, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        mlba_internal_set_hip(e);
        *ptr = nullptr;
        return MLBA_ENOMEM;
    }
    P->allocs.push_back(*ptr);
    return MLBA_OK;
}

template <class T>
int dalloc_t(mlba_plan_s* P, T** ptr, size_t count) {
    void* v = nullptr;
    int st = dalloc(P, &v, count * sizeof(T));
    *ptr = (T*)v;
    return st;
}

void release_events(mlba_plan_s* P) {
    for (hipEvent_t e : P->prof_ev) hipEventDestroy(e);
    P->prof_ev.clear();
    P->prof_phase.clear();
    P->prof_kernel.clear();
    P->prof_nl.clear();
    P->prof_nm.clear();
    P->prof_cap = P->prof_used = 0;
    P->prof_cur = -1;
}

constexpr int kMarks = mlba_plan_s::kMaxMarks;

// Start of a profiled iteration (while event slots remain).
int prof_iter_begin(mlba_plan_s* P, hipStream_t s) {
    P->prof_cur = -1;
    if (P->prof_used >= P->prof_cap) return MLBA_OK;
    if ((P->prof_seen++ % P->prof_stride) != 0) return MLBA_OK;
    const int it = P->prof_used++;
    P->prof_cur = it;
    P->prof_nm[it] = 1;
    HIPCHK(hipEventRecord(P->prof_ev[(size_t)it * kMarks], s));
    return MLBA_OK;
}

// The time since the previous event belongs to `launches` launches of `kernel`
// in `phase` (no-op outside a profiled iteration).
int prof_mark(mlba_plan_s* P, int phase, int kernel, int launches, hipStream_t s) {
    const int it = P->prof_cur;
    if (it < 0 || P->prof_nm[it] >= kMarks) return MLBA_OK;
    const size_t i = (size_t)it * kMarks + P->prof_nm[it]++;
    P->prof_phase[i] = phase;
    P->prof_kernel[i] = kernel;
    P->prof_nl[i] = launches;
    HIPCHK(hipEventRecord(P->prof_ev[i], s));
    return MLBA_OK;
}

#define MARK(ph, k) STCHK(prof_mark(P, MLBA_PHASE_##ph, MLBA_KERNEL_##k, 1, s))

// Records the plan's completion event on s after a call that enqueued work
// (mlba_plan_destroy waits for it instead of for the whole device).
int note_work(mlba_plan_s* P, int st, hipStream_t s) {
    if (st >= 0 && P->done) HIPCHK(hipEventRecord(P->done, s));
    return st;
}

void free_plan(mlba_plan_s* P) {
    if (P->done) (void)hipEventDestroy(P->done);
    release_events(P);
    for (void* a : P->allocs) hipFree(a);
    P->allocs.clear();
    delete P;
}

size_t NN(const mlba_plan_s* P) { return (size_t)P->N * P->N; }

// r = g - A u (g may be null: y = A u); partial sums of r^2 into P->partials
// The first two passes of A u on the FFT grid (section 2.1): the m x m grid
// (m = n + p - 1) holds the rectangular model's unknown at the origin, or a
// square model's image at (c, c) with its pad of Table 1 or section 2.2 around
// it (E u; the zero pad's rows are skipped); the column pass keeps the rows
// [p - 1, p - 1 + n) that the output crop reads.
int blur_grid_forward(mlba_plan_s* P, const float* u, hipStream_t s) {
    const int n = P->n, p = P->p, m = n + p - 1, c = P->c;
    int y_lo = 0, y_hi = m;
    if (P->bc == MLBA_BC_RECT) {
        HIPCHK(launch_fc_rows_fwd(P->fc, u, m, 0, 0, m, s));
    } else if (P->bc == MLBA_BC_ZERO) {
        y_lo = c;
        y_hi = c + n;
        HIPCHK(launch_fc_rows_fwd(P->fc, u, n, c, y_lo, y_hi, s));
    } else {
        HIPCHK(launch_fc_rows_fwd(P->fc, u, n, c, 0, m, s, ext_of_bc(P->bc)));
    }
    MARK(BLUR, FC_ROWS_FWD);
    HIPCHK(launch_fc_cols(P->fc, 0, y_lo, y_hi, 0, nullptr, s, p - 1, p - 1 + n + (n & 1)));
    MARK(BLUR, FC_COLS);
    return MLBA_OK;
}

int do_blur(mlba_plan_s* P, const float* u, const float* g, float* y, bool want_norm, int* nparts,
            hipStream_t s) {
    if (P->blur_fft) {
        const int n = P->n, p = P->p;
        STCHK(blur_grid_forward(P, u, s));
        HIPCHK(launch_fc_rows_inv(P->fc, p - 1, p - 1, n, y, g, 0, g && want_norm ? P->partials : nullptr, nparts,
                                  s));
        MARK(BLUR, FC_ROWS_INV);
        return MLBA_OK;
    }
    BatchImage d = plan_desc(P);
    d.u = const_cast<float*>(u);
    d.g = g;
    d.r = y;
    HIPCHK(launch_conv_job(blur_job(d), P->p, 1, P->conv_rows[0], want_norm ? P->partials : nullptr, nparts, s));
    MARK(BLUR, CONV_BLUR);
    return MLBA_OK;
}

// The preconditioner's transposed workspace and transform plan (BCCB: the
// half spectrum; DCT: the real coefficients and the DCT twiddles).
PrecondRows precond_rows(const mlba_plan_s* P) {
    PrecondRows pr{};
    pr.T = (float2*)P->swork;
    pr.ts = P->ts;
    pr.fd = P->fd;
    pr.tw = P->tw;
    pr.dtw = P->precond == MLBA_PRECOND_DCT ? P->dtw : nullptr;
    return pr;
}

// FFT blur with the BCCB or DCT preconditioner: the residual's inverse row
// pass and the preconditioner's forward row pass run as one launch (as do the
// preconditioner's inverse row pass and the forward row pass of A^T).
bool fused_fft_path(const mlba_plan_s* P) {
    return P->blur_fft && P->bc != MLBA_BC_ANTIREFLECT &&
           (P->precond == MLBA_PRECOND_BCCB || P->precond == MLBA_PRECOND_DCT) &&
           fftconv_fusable(P->fc, P->n, precond_rows(P));
}

// FFT blur of the antireflective model with the antireflective transform: the
// residual's inverse row pass runs with the transform's forward row pass.
bool fused_ar_path(const mlba_plan_s* P) {
    return P->blur_fft && P->bc == MLBA_BC_ANTIREFLECT && P->precond == MLBA_PRECOND_AR &&
           fftconv_ar_fusable(P->fc, P->n, P->fd);
}

// r = g - A u with its partials and the preconditioner's forward row pass of r
int do_blur_residual_precond_rows(mlba_plan_s* P, const float* u, const float* g, int* nparts, hipStream_t s) {
    const int n = P->n, p = P->p;
    STCHK(blur_grid_forward(P, u, s));
    HIPCHK(launch_fc_residual_precond_rows(P->fc, n, p, g, nullptr, P->partials, nparts, precond_rows(P), s));
    MARK(BLUR, FC_RESIDUAL_PRECOND_ROWS);
    return MLBA_OK;
}

// The last two passes of w (+)= A^T y on the FFT grid, after the forward rows
// of y placed at (p - 1, p - 1): the column pass with the conjugate spectrum,
// then the inverse rows; the circular correlation cropped to [0, m)^2
// (rectangular model), or folded back onto the n x n image by E^T, the
// transpose of the square model's pad (zero: the crop at (c, c)).
int blurT_grid_finish(mlba_plan_s* P, float* w, int accum, hipStream_t s) {
    const int n = P->n, p = P->p, m = n + p - 1;
    if (P->bc == MLBA_BC_RECT) {
        HIPCHK(launch_fc_cols(P->fc, 1, p - 1, m, 0, nullptr, s, 0, m + (m & 1)));
        MARK(BLUR_T, FC_COLS);
        HIPCHK(launch_fc_rows_inv(P->fc, 0, 0, m, w, nullptr, accum, nullptr, nullptr, s));
    } else {
        const int fold = ext_of_bc(P->bc);
        HIPCHK(launch_fc_cols(P->fc, 1, p - 1, m, 0, nullptr, s, 0, 0, fold, n, P->c));
        MARK(BLUR_T, FC_COLS);
        HIPCHK(launch_fc_rows_inv(P->fc, 0, 0, n, w, nullptr, accum, nullptr, nullptr, s, fold, P->c));
    }
    MARK(BLUR_T, FC_ROWS_INV);
    return MLBA_OK;
}

// the preconditioner's inverse row pass, then w (+)= A^T t
int do_precond_rows_blurT(mlba_plan_s* P, float* w, int accum, hipStream_t s) {
    HIPCHK(launch_precond_rows_fc_fwd(P->fc, P->n, P->p, precond_rows(P), nullptr, s));
    MARK(BLUR_T, PRECOND_ROWS_FC_FWD);
    return blurT_grid_finish(P, w, accum, s);
}

// w (+)= A^T y on the FFT grid: the circular correlation of y placed at
// (p-1, p-1), cropped to [0, m)^2 (rectangular model) or folded by E^T (square
// models); antireflective model: the reblur A' y, the circular correlation of
// y's antireflective extension (m x m at the origin) cropped to [0, n)^2 (the
// valid part of its convolution with the rotated PSF)
int do_blurT_fft(mlba_plan_s* P, const float* y, float* w, int accum, hipStream_t s) {
    const int n = P->n, p = P->p, N = n + p - 1;
    if (P->bc == MLBA_BC_ANTIREFLECT) {
        HIPCHK(launch_fc_rows_fwd(P->fc, y, n, P->c, 0, N, s, EXT_ANTIREFLECT));
        MARK(BLUR_T, FC_ROWS_FWD);
        HIPCHK(launch_fc_cols(P->fc, 1, 0, N, 0, nullptr, s, 0, n + (n & 1)));
        MARK(BLUR_T, FC_COLS);
        HIPCHK(launch_fc_rows_inv(P->fc, 0, 0, n, w, nullptr, accum, nullptr, nullptr, s));
        MARK(BLUR_T, FC_ROWS_INV);
        return MLBA_OK;
    }
    HIPCHK(launch_fc_rows_fwd(P->fc, y, n, p - 1, p - 1, N, s));
    MARK(BLUR_T, FC_ROWS_FWD);
    return blurT_grid_finish(P, w, accum, s);
}

int do_blurT(mlba_plan_s* P, const float* y, float* w, hipStream_t s) {
    if (P->blur_fft) return do_blurT_fft(P, y, w, 0, s);
    BatchImage d = plan_desc(P);
    d.t = const_cast<float*>(y);
    d.w = w;
    HIPCHK(launch_conv_job(blurT_job(d), P->p, 0, P->conv_rows[1], nullptr, nullptr, s));
    MARK(BLUR_T, CONV_BLUR_T);
    if (P->bc == MLBA_BC_REFLECT) {
        HIPCHK(launch_fold_reflect(P->wext, P->n + P->p - 1, w, P->n, P->c, s));
        MARK(BLUR_T, FOLD_REFLECT);
    }
    return MLBA_OK;
}

int do_precond(mlba_plan_s* P, const float* r, float* t, double alpha, hipStream_t s) {
    const int n = P->n;
    const float inv = (float)(1.0 / ((double)n * (double)n));
    if (P->precond == MLBA_PRECOND_BCCB) {
        float2* T = (float2*)P->swork;
        HIPCHK(launch_fft_rows_r2c(r, n, T, P->ts, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_fft_cols_filter(T, n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_fft_rows_c2r(T, n, P->ts, t, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_INV);
    } else if (P->precond == MLBA_PRECOND_DCT) {
        float* Tr = (float*)P->swork;
        HIPCHK(launch_dct_rows_fwd(r, n, Tr, P->ts, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_dct_cols_filter(Tr, n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_dct_rows_inv(Tr, n, P->ts, t, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_ROWS_INV);
    } else if (P->precond == MLBA_PRECOND_AR) {
        float* Tr = (float*)P->swork;
        HIPCHK(launch_ar_rows_fwd(r, n, Tr, P->ts, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_ar_cols_filter(Tr, n, P->ts, P->spec, (float)alpha, nullptr, P->fd, P->tw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_ar_rows_inv(Tr, n, P->ts, t, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_INV);
    } else if (r != t) {
        HIPCHK(hipMemcpyAsync(t, r, (size_t)n * n * sizeof(float), hipMemcpyDeviceToDevice, s));
        MARK(PRECOND, OTHER);
    }
    return MLBA_OK;
}

int compute_spectrum(mlba_plan_s* P, hipStream_t s) {
    const int n = P->n;
    if (P->precond == MLBA_PRECOND_BCCB) {
        HIPCHK(launch_pad_psf(P->psf, P->p, P->r, n, s));
        HIPCHK(launch_fft_rows_r2c(P->r, n, (float2*)P->swork, P->ts, P->fd, P->tw, s));
        HIPCHK(launch_fft_cols_power((const float2*)P->swork, n, P->ts, P->spec, P->fd, P->tw, s));
        if (P->lamc) {  // Algorithm 4: eigenvalues of the periodic blur (PSF centred at the origin)
            HIPCHK(launch_pad_psf_centred(P->psf, P->p, P->r, n, s));
            HIPCHK(launch_fft_rows_r2c(P->r, n, (float2*)P->swork, P->ts, P->fd, P->tw, s));
            HIPCHK(launch_fft_cols_complex((const float2*)P->swork, n, P->ts, P->lamc, P->fd, P->tw, s));
        }
    } else if (P->precond == MLBA_PRECOND_DCT) {
        HIPCHK(launch_cos_spectrum(P->psf, P->p, n, n, 0, P->costab, P->r, P->spec, P->lamr, s));
    } else if (P->precond == MLBA_PRECOND_AR) {
        HIPCHK(launch_cos_spectrum(P->psf, P->p, n, n - 1, 1, P->costab, P->r, P->spec, P->lamr, s));
    }
    return MLBA_OK;
}

// t = C^T (C C^T + alpha I)^{-1} r (Algorithm 4), or accumulated into t (accum)
int do_ct_precond(mlba_plan_s* P, const float* r, float* t, double alpha, int accum, hipStream_t s) {
    const int n = P->n;
    const float inv = (float)(1.0 / ((double)n * (double)n));
    if (P->precond == MLBA_PRECOND_BCCB) {
        float2* T = (float2*)P->swork;
        HIPCHK(launch_fft_rows_r2c(r, n, T, P->ts, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_fft_cols_filter(T, n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, s, P->lamc));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_fft_rows_c2r(T, n, P->ts, t, P->fd, P->tw, s, accum));
        MARK(PRECOND, FFT_ROWS_INV);
    } else if (P->precond == MLBA_PRECOND_AR) {
        float* Tr = (float*)P->swork;
        HIPCHK(launch_ar_rows_fwd(r, n, Tr, P->ts, P->fd, P->tw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_ar_cols_filter(Tr, n, P->ts, P->spec, (float)alpha, P->lamr, P->fd, P->tw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_ar_rows_inv(Tr, n, P->ts, t, P->fd, P->tw, s, accum));
        MARK(PRECOND, FFT_ROWS_INV);
    } else {
        float* Tr = (float*)P->swork;
        HIPCHK(launch_dct_rows_fwd(r, n, Tr, P->ts, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_dct_cols_filter(Tr, n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, P->dtw, s, P->lamr));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_dct_rows_inv(Tr, n, P->ts, t, P->fd, P->tw, P->dtw, s, accum));
        MARK(PRECOND, FFT_ROWS_INV);
    }
    return MLBA_OK;
}

// Algorithm 4-NS step (BCCB or DCT plan): alpha_n solved on the device from
// the spectrum (or the DCT coefficients) of r (rn_sq = ||r||^2 on the device),
// then t (+)= C^T (C C^T + alpha_n I)^{-1} r
int do_ct_precond_ns(mlba_plan_s* P, const float* r, float* t, const double* rn_sq, double noise, double q,
                     double rho, double alpha_first, int first, double* hist, int accum, hipStream_t s) {
    const int n = P->n;
    const float inv = (float)(1.0 / ((double)n * (double)n));
    if (P->precond == MLBA_PRECOND_DCT) {  // the same steps on the 2-D DCT-II coefficients
        float* Tr = (float*)P->swork;
        HIPCHK(launch_dct_rows_fwd(r, n, Tr, P->ts, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_ROWS_FWD);
        HIPCHK(launch_dct_cols_forward(Tr, n, P->ts, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_ns_alpha(Tr, 1, n, P->ts, P->spec, P->ns, P->partials, rn_sq, noise, q, rho,
                               alpha_first, first, kNsSteps, hist, s));
        STCHK(prof_mark(P, MLBA_PHASE_PRECOND, MLBA_KERNEL_OTHER, ns_alpha_launches(kNsSteps), s));
        HIPCHK(launch_dct_cols_filter_inverse(Tr, n, P->ts, P->spec, P->ns, inv, P->lamr, P->fd, P->tw, P->dtw, s));
        MARK(PRECOND, FFT_COLS);
        HIPCHK(launch_dct_rows_inv(Tr, n, P->ts, t, P->fd, P->tw, P->dtw, s, accum));
        MARK(PRECOND, FFT_ROWS_INV);
        return MLBA_OK;
    }
    float2* T = (float2*)P->swork;
    HIPCHK(launch_fft_rows_r2c(r, n, T, P->ts, P->fd, P->tw, s));
    MARK(PRECOND, FFT_ROWS_FWD);
    HIPCHK(launch_fft_cols_forward(T, n, P->ts, P->fd, P->tw, s));
    MARK(PRECOND, FFT_COLS);
    HIPCHK(launch_ns_alpha(T, 0, n, P->ts, P->spec, P->ns, P->partials, rn_sq, noise, q, rho,
                           alpha_first, first, kNsSteps, hist, s));
    STCHK(prof_mark(P, MLBA_PHASE_PRECOND, MLBA_KERNEL_OTHER, ns_alpha_launches(kNsSteps), s));
    HIPCHK(launch_fft_cols_filter_inverse(T, n, P->ts, P->spec, P->ns, inv, P->lamc, P->fd, P->tw, s));
    MARK(PRECOND, FFT_COLS);
    HIPCHK(launch_fft_rows_c2r(T, n, P->ts, t, P->fd, P->tw, s, accum));
    MARK(PRECOND, FFT_ROWS_INV);
    return MLBA_OK;
}

LevelMu level_mu(const float* mub, int lev) {
    LevelMu m;
    m.low = mub[0];
    for (int q = 0; q < 8; ++q) m.band[q] = mub[1 + 8 * (lev - 1) + q];
    return m;
}

// z (+)= W v over all levels
int do_analysis(mlba_plan_s* P, const float* v, float* z, bool accum, hipStream_t s) {
    const size_t nn = NN(P);
    const float* in = v;
    for (int lev = 1; lev <= P->levels; ++lev) {
        const int d = 1 << (lev - 1);
        float* zlev = z + (size_t)(1 + 8 * (lev - 1)) * nn;
        const bool last = lev == P->levels;
        float* low = last ? z : P->tmp[lev & 1];
        HIPCHK(launch_analysis_level(in, P->N, d, zlev, low, accum ? 1 : 0, (accum && last) ? 1 : 0, s));
        MARK(ANALYSIS, ANALYSIS_LEVEL);
        in = low;
    }
    return MLBA_OK;
}

// f = W^T (delta S_mu(z)) (thr) or W^T z
int do_synthesis(mlba_plan_s* P, const float* z, float* f, bool thr, const float* mub, float delta,
                 hipStream_t s) {
    const size_t nn = NN(P);
    static const float zeros[64] = {0};
    const float* mu = thr ? mub : zeros;
    const float* low = z;
    for (int lev = P->levels; lev >= 1; --lev) {
        const int d = 1 << (lev - 1);
        const float* zlev = z + (size_t)(1 + 8 * (lev - 1)) * nn;
        float* out = lev == 1 ? f : P->tmp[lev & 1];
        const bool top = lev == P->levels;
        HIPCHK(launch_synthesis_level(zlev, low, P->N, d, out, level_mu(mu, lev), thr ? delta : 1.0f,
                                      (thr && top) ? 1 : 0, thr ? 1 : 0, s));
        MARK(SYNTHESIS, SYNTHESIS_LEVEL);
        low = out;
    }
    return MLBA_OK;
}

// f = W^T (delta S_mu(W omega)) (implicit state): low-pass chain, then one
// shrink-synthesis launch per level from the top
int do_shrink_synthesis(mlba_plan_s* P, const float* omega, float* f, const float* mub, float delta,
                        hipStream_t s) {
    const float* low[4] = {omega, P->lows[0], P->lows[1], P->lows[2]};
    int l = 1;
    if (P->levels >= 3) {  // the first two levels of the chain in one pass
        HIPCHK(launch_lowpass_two_levels(omega, P->N, P->lows[0], P->lows[1], s));
        MARK(SYNTHESIS, LOWPASS_LEVEL);
        l = 3;
    }
    for (; l < P->levels; ++l) {
        HIPCHK(launch_lowpass_level(low[l - 1], P->N, 1 << (l - 1), P->lows[l - 1], s));
        MARK(SYNTHESIS, LOWPASS_LEVEL);
    }
    const float* s_in = nullptr;
    for (int lev = P->levels; lev >= 1; --lev) {
        float* out = lev == 1 ? f : P->tmp[lev & 1];
        HIPCHK(launch_shrink_synthesis_level(low[lev - 1], s_in, P->N, 1 << (lev - 1), out, level_mu(mub, lev),
                                             delta, s));
        MARK(SYNTHESIS, SHRINK_SYNTHESIS);
        s_in = out;
    }
    return MLBA_OK;
}

// omega += A^T y (implicit state: the Bregman update of eq. (MLBA2) before W)
int do_blurT_acc(mlba_plan_s* P, const float* y, float* omega, hipStream_t s) {
    if (P->blur_fft) return do_blurT_fft(P, y, omega, 1, s);
    BatchImage d = plan_desc(P);
    d.t = const_cast<float*>(y);
    d.w = omega;
    ConvJob j = blurT_job(d);
    const bool fold = P->bc == MLBA_BC_REFLECT;
    j.acc = fold ? 0 : 1;
    HIPCHK(launch_conv_job(j, P->p, 0, P->conv_rows[1], nullptr, nullptr, s));
    MARK(BLUR_T, CONV_BLUR_T);
    if (fold) {
        HIPCHK(launch_fold_reflect(P->wext, P->n + P->p - 1, omega, P->n, P->c, s, 1));
        MARK(BLUR_T, FOLD_REFLECT);
    }
    return MLBA_OK;
}

// Algorithm 2: P->pcg[0 .. n^2) <- t ~ (A A^T + alpha I)^{-1} r (r = P->r, used
// as the CG residual and overwritten) by preconditioned CG from t = 0, at most
// max_steps steps, stopping at the first step with sqrt(rho_j / rho_0) <= tol,
// rho_j = res_j^T M^{-1} res_j (eq. bet).  The test runs on the device: all
// max_steps steps are enqueued, and once the CG has stopped the updates of
// t, res and d are skipped; *hist (device) receives beta_n.  No host round trip.
// q = (A A^T + alpha I) d with the partials of d . q (np of them).  The
// rectangular model on the FFT grid takes one transform pair with |H|^2:
// the correlation A^T d of d placed at (p-1, p-1) vanishes outside
// [0, m)^2, and M >= m, so the crop between A^T and A changes nothing.
// dir (optional): first update d = z + b d in the same pass (FFT grid) or as
// a separate pass.
bool gram_on_grid(const mlba_plan_s* P) { return P->blur_fft && P->bc == MLBA_BC_RECT; }

int do_gram(mlba_plan_s* P, float* d, float* q, double alpha, int* np, const PcgDir* dir, hipStream_t s) {
    const int n = P->n, p = P->p, m = n + p - 1;
    const size_t nn = (size_t)n * n;
    if (dir && !gram_on_grid(P)) {
        if (dir->rho_new) HIPCHK(launch_pcg_dir(d, dir->z, nn, dir->rho_new, dir->rho, dir->act, s));
        else HIPCHK(hipMemcpyAsync(d, dir->z, nn * sizeof(float), hipMemcpyDeviceToDevice, s));
        dir = nullptr;
    }
    if (gram_on_grid(P)) {
        HIPCHK(launch_fc_rows_fwd(P->fc, d, n, p - 1, p - 1, m, s, EXT_ZERO, dir));
        MARK(BLUR_T, FC_ROWS_FWD);
        HIPCHK(launch_fc_cols(P->fc, 2, p - 1, m, 0, nullptr, s, p - 1, p - 1 + n + (n & 1)));
        MARK(BLUR, FC_COLS);
        HIPCHK(launch_fc_rows_inv(P->fc, p - 1, p - 1, n, q, nullptr, 0, P->partials, np, s, -1, 0, d,
                                  (float)alpha));
        MARK(BLUR, FC_ROWS_INV);
        return MLBA_OK;
    }
    STCHK(do_blurT(P, d, P->w, s));
    STCHK(do_blur(P, P->w, nullptr, q, false, nullptr, s));
    HIPCHK(launch_axpy(q, d, nn, (float)alpha, s));
    HIPCHK(launch_dot_partials(d, q, nn, P->partials, np, s));
    return MLBA_OK;
}

// The PCG's start through the fused row kernels: BCCB plan, the partials of
// the c2r pass fit, and (for the residual's fused row pass) the fused FFT path.
bool pcg_fused_rows(const mlba_plan_s* P) {
    return P->precond == MLBA_PRECOND_BCCB && pcg_rows_c2r_partials(P->n) <= P->partials_cap;
}
bool pcg_fused_start(const mlba_plan_s* P) { return pcg_fused_rows(P) && fused_fft_path(P); }

// rows_ready: P's forward row pass of res is already in the plan's workspace
int do_pcg(mlba_plan_s* P, double alpha, int max_steps, double tol, int* hist, bool rows_ready, hipStream_t s) {
    const size_t nn = (size_t)P->n * P->n;
    float* t = P->pcg;
    float* zc = P->pcg + nn;
    float* d = P->pcg + 2 * nn;
    float* q = P->pcg + 3 * nn;
    float* res = P->r;
    double* st = P->pcgs;
    double* rho[2] = {st, st + 1};
    double* pq = st + 2;
    const double* act = st + 4;
    int np = 0;
    // BCCB plan: the update t += a d, res -= a q runs inside P's forward row
    // pass and the dot product res . z inside its inverse row pass; the first
    // direction d = z is copied by the first Gram product's forward row pass
    const bool fused = pcg_fused_rows(P);
    const float inv = (float)(1.0 / ((double)P->n * (double)P->n));
    HIPCHK(launch_fill(t, nn, 0.0f, s));
    if (fused) {
        if (!rows_ready) HIPCHK(launch_fft_rows_r2c(res, P->n, (float2*)P->swork, P->ts, P->fd, P->tw, s));
        HIPCHK(launch_fft_cols_filter((float2*)P->swork, P->n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, s));
        HIPCHK(launch_pcg_rows_c2r((const float2*)P->swork, P->n, P->ts, zc, res, P->fd, P->tw, P->partials, &np, s));
        HIPCHK(launch_pcg_begin_sum(st, P->partials, np, hist, s));
    } else {
        STCHK(do_precond(P, res, zc, alpha, s));
        HIPCHK(hipMemcpyAsync(d, zc, nn * sizeof(float), hipMemcpyDeviceToDevice, s));
        HIPCHK(launch_dot_partials(res, zc, nn, P->partials, &np, s));
        HIPCHK(launch_sum_partials(P->partials, np, rho[0], s));
        HIPCHK(launch_pcg_begin(st, hist, s));
    }
    for (int j = 1; j <= max_steps; ++j) {
        double* rc = rho[(j - 1) & 1];
        double* rn = rho[j & 1];
        // q = (A A^T + alpha I) d, d . q; from the second step on, first the
        // direction d = z + (rho_{j-1} / rho_{j-2}) d of the previous step
        // (fused start: at the first step the copy d = z, rho_new null)
        const PcgDir dir{d, zc, j > 1 ? rc : nullptr, rn, act};
        STCHK(do_gram(P, d, q, alpha, &np, (j > 1 || fused) ? &dir : nullptr, s));
        HIPCHK(launch_sum_partials(P->partials, np, pq, s));
        if (fused) {
            const PcgVec v{t, res, d, q, rc, pq, act};
            HIPCHK(launch_pcg_rows_r2c(P->n, (float2*)P->swork, P->ts, P->fd, P->tw, v, s));
            HIPCHK(launch_fft_cols_filter((float2*)P->swork, P->n, P->ts, P->spec, (float)alpha, inv, P->fd, P->tw, s));
            HIPCHK(launch_pcg_rows_c2r((const float2*)P->swork, P->n, P->ts, zc, res, P->fd, P->tw, P->partials, &np,
                                       s));
            HIPCHK(launch_pcg_check_sum(st, P->partials, np, rn, j, max_steps, tol, hist, s));
        } else {
            HIPCHK(launch_pcg_update(t, res, d, q, nn, rc, pq, act, s));
            STCHK(do_precond(P, res, zc, alpha, s));
            HIPCHK(launch_dot_partials(res, zc, nn, P->partials, &np, s));
            HIPCHK(launch_sum_partials(P->partials, np, rn, s));
            HIPCHK(launch_pcg_check(st, rn, j, max_steps, tol, hist, s));
        }
    }
    return MLBA_OK;
}

int expand_mu(const mlba_plan_s* P, const double* mu, int n_mu, float* out) {
    if (!mu || (n_mu != 1 && n_mu != P->bands)) return MLBA_EINVAL;
    for (int b = 0; b < P->bands; ++b) {
        const double v = mu[n_mu == 1 ? 0 : b];
        if (!(v >= 0.0) || !isfinite(v)) return MLBA_EINVAL;
        out[b] = (float)v;
    }
    return MLBA_OK;
}

}  // namespace

namespace {

// y = A^T P_alpha A v (A' P_alpha A for antireflective conditions)
int normal_matvec(mlba_plan_s* P, const float* v, float* y, double alpha, hipStream_t s) {
    STCHK(do_blur(P, v, nullptr, P->r, false, nullptr, s));
    STCHK(do_precond(P, P->r, P->t, alpha, s));
    return do_blurT(P, P->t, y, s);
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..k)
// and off-diagonal b[1..k) (b[j] couples rows j-1 and j), by bisection on the
// Sturm count (the number of negative pivots of T - xI is the number of
// eigenvalues below x).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < k ? fabs(b[i + 1]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    auto below = [&](double x) {
        int c = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = a[i] - x - (i > 0 ? b[i] * b[i] / d : 0.0);
            if (fabs(d) < 1e-300) d = -1e-300;
            if (d < 0.0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 400 && hi - lo > 1e-16 * fmax(fabs(hi), fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (below(mid) == k) hi = mid;
        else lo = mid;
    }
    return hi;
}

// Lanczos on the symmetric operator A^T P A (no reorthogonalisation: lost
// orthogonality duplicates converged Ritz values but leaves the largest one
// converging to the largest eigenvalue).  The tridiagonal entries are device
// doubles in the plan's norm ring (hist[2k] = alpha_k, hist[2k+1] =
// beta_{k+1}^2), read back every kBatch steps; the largest Ritz value grows
// monotonically with k (interlacing), and the run stops once it has changed
// by at most tol (relative) over kBatch steps, at an invariant subspace
// (beta ~ 0) or after max_steps.
int lanczos_norm(mlba_plan_s* P, double alpha, int max_steps, double tol, double* out, int* steps_out,
                 hipStream_t s) {
    constexpr int kBatch = 8;
    const size_t nn = NN(P);
    if (max_steps > P->rn_cap / 2) max_steps = P->rn_cap / 2;
    float* v = P->pv;
    float* vp = P->tmp[0];
    float* w = P->u;  // the synthesis buffer is free while estimating
    double* hist = P->rn;
    HIPCHK(launch_fill_hash(v, nn, 7u, s));
    int np = 0;
    HIPCHK(launch_dot_partials(v, v, nn, P->partials, &np, s));
    HIPCHK(launch_sum_partials(P->partials, np, P->scal, s));
    HIPCHK(launch_scale(v, nn, P->scal, 1.0f, s));
    std::vector<double> a, b(1, 0.0), theta, buf(2 * kBatch);
    int k = 0;
    bool done = false;
    while (!done && k < max_steps) {
        const int k1 = k + kBatch < max_steps ? k + kBatch : max_steps;
        for (int j = k; j < k1; ++j) {
            STCHK(normal_matvec(P, v, w, alpha, s));
            HIPCHK(launch_dot_partials(v, w, nn, P->partials, &np, s));
            HIPCHK(launch_sum_partials(P->partials, np, hist + 2 * j, s));
            HIPCHK(launch_lanczos_step(w, v, j ? vp : nullptr, nn, hist + 2 * j, j ? hist + 2 * j - 1 : nullptr,
                                       P->partials, &np, s));
            HIPCHK(launch_sum_partials(P->partials, np, hist + 2 * j + 1, s));
            HIPCHK(launch_scale(w, nn, hist + 2 * j + 1, 1.0f, s));
            float* x = vp;
            vp = v;
            v = w;
            w = x;
        }
        HIPCHK(hipMemcpyAsync(buf.data(), hist + 2 * k, 2 * (k1 - k) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int j = k; j < k1 && !done; ++j) {
            const double aj = buf[2 * (j - k)], b2 = buf[2 * (j - k) + 1];
            if (!isfinite(aj)) {
                done = true;
                break;
            }
            a.push_back(aj);
            theta.push_back(tridiag_max_eig(a, b, (int)a.size()));
            const double th = theta.back();
            if (!isfinite(b2) || b2 <= 1e-24 * th * th) done = true;  // invariant subspace
            else b.push_back(sqrt(b2));
        }
        k = (int)a.size();
        if (k > kBatch && fabs(theta[k - 1] - theta[k - 1 - kBatch]) <= tol * fabs(theta[k - 1])) done = true;
        if ((int)a.size() < k1) done = true;
    }
    if (a.empty()) return MLBA_EHIP;
    *out = theta.back();
    if (steps_out) *steps_out = (int)a.size();
    return MLBA_OK;
}

// The antireflective model's A' P A is not symmetric: power iteration on it,
// ||M v|| / ||v|| after `iters` steps.
int power_norm(mlba_plan_s* P, double alpha, int iters, double* out, hipStream_t s) {
    const size_t nn = NN(P);
    float* v = P->pv;
    float* w = P->u;
    HIPCHK(launch_fill_hash(v, nn, 7u, s));
    int np = 0;
    HIPCHK(launch_dot_partials(v, v, nn, P->partials, &np, s));
    HIPCHK(launch_sum_partials(P->partials, np, P->scal, s));
    HIPCHK(launch_scale(v, nn, P->scal, 1.0f, s));
    for (int it = 0; it < iters; ++it) {
        STCHK(normal_matvec(P, v, w, alpha, s));
        HIPCHK(launch_dot_partials(v, w, nn, P->partials, &np, s));
        HIPCHK(launch_sum_partials(P->partials, np, P->scal + 1, s));
        HIPCHK(launch_dot_partials(w, w, nn, P->partials, &np, s));
        HIPCHK(launch_sum_partials(P->partials, np, P->scal, s));
        HIPCHK(launch_scale(w, nn, P->scal, 1.0f, s));
        float* x = v;
        v = w;
        w = x;
    }
    double host[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(host, P->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = host[1];
    return MLBA_OK;
}

}  // namespace

int mlba_internal_opnorm(mlba_plan_s* P, double alpha, int iters, double tol, double* out, int* steps_out,
                         hipStream_t s) {
    if (P->bc == MLBA_BC_ANTIREFLECT) {
        if (steps_out) *steps_out = iters;
        return power_norm(P, alpha, iters, out, s);
    }
    return lanczos_norm(P, alpha, iters, tol, out, steps_out, s);
}

int mlba_internal_auto_delta(mlba_plan_s* P, double alpha, double* delta, hipStream_t s) {
    double nrm = 0.0;
    if (P->bc == MLBA_BC_ANTIREFLECT) STCHK(mlba_internal_opnorm(P, alpha, kAutoPowerSteps, 0.0, &nrm, nullptr, s));
    else STCHK(mlba_internal_opnorm(P, alpha, kAutoLanczosSteps, kAutoLanczosTol, &nrm, nullptr, s));
    *delta = 0.9 / (nrm > 0.9 ? nrm : 0.9);
    return MLBA_OK;
}

namespace {

double alpha_at(const mlba_alpha_schedule& a, int k) {
    switch (a.kind) {
        case MLBA_ALPHA_GEOMETRIC: {
            const double v = a.alpha0 * pow(a.ratio, (double)k);
            return v > a.alpha_floor ? v : a.alpha_floor;
        }
        case MLBA_ALPHA_TABLE:
            return a.table[k];
        default:
            return a.alpha0;
    }
}

}  // namespace

extern "C" {

const char* mlba_status_string(int status) {
    switch (status) {
        case MLBA_OK: return "ok";
        case MLBA_WARN_DIVERGED: return "warning: residual diverged";
        case MLBA_EINVAL: return "invalid argument";
        case MLBA_EUNSUPPORTED: return "unsupported size";
        case MLBA_EHIP: return "HIP runtime error";
        case MLBA_ENOMEM: return "device allocation failed";
        default: return "unknown status";
    }
}

int mlba_last_hip_error(void) { return mlba_internal_last_hip(); }

int mlba_version(void) { return 1; }

int mlba_plan_create(mlba_plan_t* plan, int n, int p, int bc, int precond, int levels, const float* psf,
                     hipStream_t s) {
    if (!plan || !psf) return MLBA_EINVAL;
    *plan = nullptr;
    if (n < 2 || p < 1 || (p % 2) == 0 || p > n) return MLBA_EINVAL;
    if (p > 49) return MLBA_EUNSUPPORTED;  // the blur's LDS window
    if (bc < MLBA_BC_RECT || bc > MLBA_BC_ANTIREFLECT) return MLBA_EINVAL;
    if (precond < MLBA_PRECOND_BCCB || precond > MLBA_PRECOND_AR) return MLBA_EINVAL;
    if (levels < 1 || levels > 4) return MLBA_EINVAL;
    const int N = bc == MLBA_BC_RECT ? n + p - 1 : n;
    if ((1 << (levels - 1)) >= N) return MLBA_EINVAL;
    if (precond == MLBA_PRECOND_AR) {  // complex FFTs of length 2(n - 1); Q antireflective like A
        if (bc != MLBA_BC_ANTIREFLECT || !ar_transform_supported(n)) return MLBA_EUNSUPPORTED;
    } else if (precond != MLBA_PRECOND_NONE) {  // row pairs: n even
        if (n % 2 != 0 || n < 8 || !fft_length_supported(n)) return MLBA_EUNSUPPORTED;
    }

    mlba_plan_s* P = new (std::nothrow) mlba_plan_s();
    if (!P) return MLBA_ENOMEM;
    P->n = n;
    P->p = p;
    P->c = (p - 1) / 2;
    P->N = N;
    P->bc = bc;
    P->precond = precond;
    P->levels = levels;
    P->bands = 8 * levels + 1;

    int st = MLBA_OK;
    const size_t nn = (size_t)N * N, obs = (size_t)n * n;
    const int m = n + p - 1;
    P->partials_cap = conv_partials_count(n);
    if (P->partials_cap < reduce_partials_cap()) P->partials_cap = reduce_partials_cap();
    if (P->partials_cap < ns_partials_needed()) P->partials_cap = ns_partials_needed();
    P->rn_cap = 1 << 16;
#define ALLOC(ptr, count)                                  \
    do {                                                   \
        st = dalloc_t(P, &(ptr), (count));                 \
        if (st) {                                          \
            free_plan(P);                                  \
            return st;                                     \
        }                                                  \
    } while (0)
    ALLOC(P->psf, (size_t)p * p);
    ALLOC(P->u, nn);
    ALLOC(P->r, obs);
    ALLOC(P->t, obs);
    ALLOC(P->w, nn);
    ALLOC(P->tmp[0], nn);
    ALLOC(P->tmp[1], nn);
    ALLOC(P->pv, nn);
    ALLOC(P->z, nn * P->bands);
    ALLOC(P->omega, nn);
    for (int l = 0; l < levels - 1; ++l) ALLOC(P->lows[l], nn);
    ALLOC(P->partials, (size_t)P->partials_cap);
    ALLOC(P->scal, 8);
    ALLOC(P->rn, (size_t)P->rn_cap);
    ALLOC(P->ahist, (size_t)P->rn_cap);
    if (precond != MLBA_PRECOND_NONE) {
        ALLOC(P->pcg, 4 * obs);
        ALLOC(P->pcgs, 8);
        ALLOC(P->pcgh, (size_t)P->rn_cap);
    }
    if (bc == MLBA_BC_REFLECT) ALLOC(P->wext, (size_t)m * m);

    if (precond != MLBA_PRECOND_NONE) {
        const int L = precond == MLBA_PRECOND_AR ? 2 * (n - 1) : n;  // transform length
        P->fd = fft_desc(L);

        // the cosine table serves the eigenvalues: angles pi q / n (DCT) or
        // pi q / (n - 1) (antireflective transform); BCCB does not read it
        const int CN = precond == MLBA_PRECOND_AR ? n - 1 : n;
        const std::vector<float2> tw = fft_table(P->fd);
        std::vector<float2> dtw(n);
        std::vector<float> cost(2 * CN);
        const double pi = 3.14159265358979323846;
        for (int q = 0; q < n; ++q) {
            const double ang2 = -pi * (double)q / (2.0 * (double)n);
            dtw[q] = make_float2((float)cos(ang2), (float)sin(ang2));
        }
        for (int q = 0; q < 2 * CN; ++q) cost[q] = (float)cos(pi * (double)q / (double)CN);
        ALLOC(P->tw, tw.size());
        ALLOC(P->dtw, (size_t)n);
        ALLOC(P->costab, (size_t)2 * CN);
        ALLOC(P->ns, (size_t)ns_state_doubles());
        if (hipMemsetAsync(P->ns, 0, (size_t)ns_state_doubles() * sizeof(double), s) != hipSuccess) {
            free_plan(P);
            return MLBA_EHIP;
        }
        if (precond == MLBA_PRECOND_AR) {
            P->ts = ar_workspace_stride(n);
            ALLOC(P->spec, obs);
            if (bc != MLBA_BC_RECT) ALLOC(P->lamr, obs);
            float* Tr = nullptr;
            ALLOC(Tr, (size_t)n * P->ts);
            P->swork = Tr;
        } else if (precond == MLBA_PRECOND_BCCB) {
            P->ts = n + 16;
            ALLOC(P->spec, (size_t)(n / 2 + 1) * n);
            if (bc != MLBA_BC_RECT) ALLOC(P->lamc, (size_t)(n / 2 + 1) * n);
            if (bc == MLBA_BC_PERIODIC) ALLOC(P->ghat, (size_t)(n / 2 + 1) * n);  // the spectral residual: F g
            float2* T = nullptr;
            ALLOC(T, (size_t)(n / 2 + 1) * P->ts);
            P->swork = T;
        } else {
            P->ts = n + 32;
            ALLOC(P->spec, obs);
            if (bc != MLBA_BC_RECT) ALLOC(P->lamr, obs);
            float* Tr = nullptr;
            ALLOC(Tr, (size_t)n * P->ts);
            P->swork = Tr;
        }
#undef ALLOC
        hipError_t e = hipMemcpyAsync(P->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(P->dtw, dtw.data(), n * sizeof(float2), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P->costab, cost.data(), 2 * CN * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // host tables go out of scope
        if (e != hipSuccess) {
            mlba_internal_set_hip(e);
            free_plan(P);
            return MLBA_EHIP;
        }
    }
    {
        const hipError_t e = hipEventCreateWithFlags(&P->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            P->done = nullptr;
            mlba_internal_set_hip(e);
            free_plan(P);
            return MLBA_EHIP;
        }
    }
    st = mlba_plan_set_psf(P, psf, s);
    if (st < 0) {
        free_plan(P);
        return st;
    }
    *plan = P;
    return MLBA_OK;
}

int mlba_plan_set_psf(mlba_plan_t P, const float* psf, hipStream_t s) {
    if (!P || !psf) return MLBA_EINVAL;
    HIPCHK(hipMemcpyAsync(P->psf, psf, (size_t)P->p * P->p * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (P->fc.H) HIPCHK(launch_fftconv_spectrum(P->fc, P->psf, P->p, s));
    if (P->ns) HIPCHK(launch_ns_psf_l1(P->psf, P->p, P->ns, s));
    return note_work(P, compute_spectrum(P, s), s);
}

}  // extern "C"

namespace {

// Smallest M = 2^a 3^b (a >= 1) with M >= N, or 0 above the transform limit.
int fft_grid_size(int N) {
    int best = 0;
    for (int a = 1; (1 << a) <= fftconv_max_size(); ++a)
        for (long m = 1L << a; m <= fftconv_max_size(); m *= 3)
            if (m >= N && (best == 0 || m < best)) best = (int)m;
    return best;
}

// Allocates the FFT blur of a rectangular or antireflective plan (first use)
// and computes the PSF spectrum on that grid.
int ensure_fftconv(mlba_plan_s* P, hipStream_t s) {
    if (P->fc.H) return MLBA_OK;
    const int M = fft_grid_size(P->n + P->p - 1);  // the (extended) unknown, m x m
    if (M == 0) return MLBA_EUNSUPPORTED;
    if (fftconv_partials_count(M, P->n) > P->partials_cap) return MLBA_EUNSUPPORTED;
    FftConv c{};
    c.M = M;
    c.ts = M + 16;
    c.fd = fft_desc(M);
    std::vector<float2> tw(M);
    const double pi = 3.14159265358979323846;
    for (int q = 0; q < M; ++q) {
        const double ang = -2.0 * pi * (double)q / (double)M;
        tw[q] = make_float2((float)cos(ang), (float)sin(ang));
    }
    float2 *twd = nullptr, *T = nullptr, *H = nullptr, *G = nullptr;
    STCHK(dalloc_t(P, &twd, (size_t)M));
    STCHK(dalloc_t(P, &T, (size_t)(M / 2 + 1) * c.ts));
    STCHK(dalloc_t(P, &H, (size_t)(M / 2 + 1) * M));
    if (fftconv_direct_taps(P->p)) {
        STCHK(dalloc_t(P, &G, (size_t)(M / 2 + 1) * P->p));
        c.G = G;
        c.p = P->p;
    }
    HIPCHK(hipMemcpyAsync(twd, tw.data(), M * sizeof(float2), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // the host table goes out of scope
    c.tw = twd;
    c.T = T;
    c.H = H;
    HIPCHK(launch_fftconv_spectrum(c, P->psf, P->p, s));
    P->fc = c;
    return MLBA_OK;
}

// mean ms of `reps` calls of f after one untimed call
template <class F>
int time_ms(F f, int reps, hipStream_t s, double* ms) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        mlba_internal_set_hip(err);
        return MLBA_EHIP;
    }
    int st = f();
    if (st >= 0) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st >= 0; ++r) st = f();
        (void)hipEventRecord(e1, s);
        err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) {
            mlba_internal_set_hip(err);
            st = MLBA_EHIP;
        }
        *ms = (double)t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" {

int mlba_plan_set_blur(mlba_plan_t P, int mode, hipStream_t s) {
    if (!P || mode < MLBA_BLUR_DIRECT || mode > MLBA_BLUR_FFT) return MLBA_EINVAL;
    if (mode == MLBA_BLUR_FFT) STCHK(ensure_fftconv(P, s));
    P->blur_fft = mode == MLBA_BLUR_FFT ? 1 : 0;
    return MLBA_OK;
}

int mlba_plan_autotune(mlba_plan_t P, int reps, double* ms_out, hipStream_t s) {
    if (!P || reps < 1) return MLBA_EINVAL;
    double t[2][2] = {{0.0, 0.0}, {-1.0, -1.0}};  // [direct / fft][A / A^T]
    const int keep = P->blur_fft;
    const int have_fft = ensure_fftconv(P, s);
    if (have_fft < 0 && have_fft != MLBA_EUNSUPPORTED) return have_fft;
    for (int mode = 0; mode < (have_fft == MLBA_OK ? 2 : 1); ++mode) {
        P->blur_fft = mode;
        // scratch only: u -> r and t -> w of the plan
        int st = time_ms([&]() { return do_blur(P, P->u, nullptr, P->r, false, nullptr, s); }, reps, s, &t[mode][0]);
        if (st >= 0) st = time_ms([&]() { return do_blurT(P, P->t, P->w, s); }, reps, s, &t[mode][1]);
        if (st < 0) {
            P->blur_fft = keep;
            return st;
        }
    }
    P->blur_fft = (have_fft == MLBA_OK && t[1][0] + t[1][1] < t[0][0] + t[0][1]) ? 1 : 0;
    if (ms_out)
        for (int i = 0; i < 4; ++i) ms_out[i] = t[i / 2][i % 2];
    return P->blur_fft ? MLBA_BLUR_FFT : MLBA_BLUR_DIRECT;
}

int mlba_plan_destroy(mlba_plan_t P) {
    if (!P) return MLBA_EINVAL;
    if (P->done) (void)hipEventSynchronize(P->done);  // the plan's last enqueued work
    free_plan(P);
    return MLBA_OK;
}

int mlba_plan_dims(mlba_plan_t P, int* n, int* p, int* N, int* bands) {
    if (!P) return MLBA_EINVAL;
    if (n) *n = P->n;
    if (p) *p = P->p;
    if (N) *N = P->N;
    if (bands) *bands = P->bands;
    return MLBA_OK;
}

int mlba_plan_opnorm(mlba_plan_t P, double alpha, int iters, double* out, hipStream_t s) {
    if (!P || !out || iters < 1 || !(alpha > 0.0 || P->precond == MLBA_PRECOND_NONE)) return MLBA_EINVAL;
    return note_work(P, mlba_internal_opnorm(P, alpha, iters, kAutoLanczosTol, out, nullptr, s), s);
}

int mlba_apply_A(mlba_plan_t P, const float* u, float* y, hipStream_t s) {
    if (!P || !u || !y) return MLBA_EINVAL;
    return note_work(P, do_blur(P, u, nullptr, y, false, nullptr, s), s);
}

int mlba_residual(mlba_plan_t P, const float* g, const float* u, float* r, hipStream_t s) {
    if (!P || !g || !u || !r) return MLBA_EINVAL;
    return note_work(P, do_blur(P, u, g, r, false, nullptr, s), s);
}

int mlba_apply_At(mlba_plan_t P, const float* y, float* w, hipStream_t s) {
    if (!P || !y || !w) return MLBA_EINVAL;
    return note_work(P, do_blurT(P, y, w, s), s);
}

int mlba_apply_P(mlba_plan_t P, const float* r, float* t, double alpha, hipStream_t s) {
    if (!P || !r || !t) return MLBA_EINVAL;
    if (P->precond != MLBA_PRECOND_NONE && !(alpha > 0.0)) return MLBA_EINVAL;
    return note_work(P, do_precond(P, r, t, alpha, s), s);
}

int mlba_apply_CtP(mlba_plan_t P, const float* r, float* t, double alpha, hipStream_t s) {
    if (!P || !r || !t || r == t || !(alpha > 0.0)) return MLBA_EINVAL;
    if (P->bc == MLBA_BC_RECT || P->precond == MLBA_PRECOND_NONE) return MLBA_EUNSUPPORTED;
    return note_work(P, do_ct_precond(P, r, t, alpha, 0, s), s);
}

int mlba_framelet_analysis(mlba_plan_t P, const float* f, float* z, hipStream_t s) {
    if (!P || !f || !z) return MLBA_EINVAL;
    return note_work(P, do_analysis(P, f, z, false, s), s);
}

int mlba_analysis_update(mlba_plan_t P, const float* w, float* z, hipStream_t s) {
    if (!P || !w || !z) return MLBA_EINVAL;
    return note_work(P, do_analysis(P, w, z, true, s), s);
}

int mlba_framelet_synthesis(mlba_plan_t P, const float* z, float* f, hipStream_t s) {
    if (!P || !z || !f) return MLBA_EINVAL;
    return note_work(P, do_synthesis(P, z, f, false, nullptr, 1.0f, s), s);
}

int mlba_threshold_synthesis(mlba_plan_t P, const float* z, const double* mu, int n_mu, double delta, float* f,
                             hipStream_t s) {
    if (!P || !z || !f || !isfinite(delta)) return MLBA_EINVAL;
    float mub[64];
    STCHK(expand_mu(P, mu, n_mu, mub));
    return note_work(P, do_synthesis(P, z, f, true, mub, (float)delta, s), s);
}

int mlba_shrink_synthesis(mlba_plan_t P, const float* omega, const double* mu, int n_mu, double delta, float* f,
                          hipStream_t s) {
    if (!P || !omega || !f || omega == f || !isfinite(delta)) return MLBA_EINVAL;
    float mub[64];
    STCHK(expand_mu(P, mu, n_mu, mub));
    return note_work(P, do_shrink_synthesis(P, omega, f, mub, (float)delta, s), s);
}

int mlba_soft_threshold(const float* z, float* x, int bands, size_t band_elems, const double* mu, int n_mu,
                        double delta, hipStream_t s) {
    if (!z || !x || !mu || bands < 1 || bands > 64 || (n_mu != 1 && n_mu != bands) || !isfinite(delta))
        return MLBA_EINVAL;
    BandMu m;
    for (int b = 0; b < bands; ++b) {
        const double v = mu[n_mu == 1 ? 0 : b];
        if (!(v >= 0.0) || !isfinite(v)) return MLBA_EINVAL;
        m.v[b] = (float)v;
    }
    HIPCHK(launch_soft_threshold(z, x, bands, band_elems, m, (float)delta, s));
    return MLBA_OK;
}

int mlba_restore(mlba_plan_t P, const float* g, const mlba_params* prm, float* f_out, float* z_state,
                 double* rnorm_out, int* iters_done, hipStream_t s) {
    if (!P || !g || !prm || !f_out) return MLBA_EINVAL;
    const int iters = prm->iters, k0 = prm->k0;
    if (iters < 0 || k0 < 0) return MLBA_EINVAL;
    const mlba_alpha_schedule& as = prm->alpha;
    if (as.kind < MLBA_ALPHA_CONST || as.kind > MLBA_ALPHA_NS) return MLBA_EINVAL;
    if (as.kind == MLBA_ALPHA_TABLE && (!as.table || as.table_len < k0 + iters)) return MLBA_EINVAL;
    if (as.kind == MLBA_ALPHA_GEOMETRIC && !(as.ratio > 0.0)) return MLBA_EINVAL;
    if (prm->delta_table && prm->delta_table_len < k0 + iters + 1) return MLBA_EINVAL;
    const mlba_stop* stop = prm->stop;
    if (stop && (stop->check_every < 1 || !(stop->noise_norm >= 0.0))) return MLBA_EINVAL;
    if (prm->state != MLBA_STATE_EXPLICIT && prm->state != MLBA_STATE_IMPLICIT) return MLBA_EINVAL;
    const bool implicit = prm->state == MLBA_STATE_IMPLICIT;
    if (prm->method < MLBA_METHOD_MLBA || prm->method > MLBA_METHOD_ALG2) return MLBA_EINVAL;
    const bool alg4 = prm->method == MLBA_METHOD_ALG4;
    const bool alg2 = prm->method == MLBA_METHOD_ALG2;
    if (alg2 && P->precond == MLBA_PRECOND_NONE) return MLBA_EUNSUPPORTED;
    const int pcg_max = prm->pcg_max > 0 ? prm->pcg_max : 5;
    const double pcg_tol = prm->pcg_tol > 0.0 ? prm->pcg_tol : 1e-3;
    if (alg2 && (pcg_max > 1000 || !isfinite(pcg_tol) || iters > P->rn_cap)) return MLBA_EINVAL;
    if (alg4 && (P->bc == MLBA_BC_RECT || P->precond == MLBA_PRECOND_NONE)) return MLBA_EUNSUPPORTED;
    const bool ns = as.kind == MLBA_ALPHA_NS;
    mlba_stop ns_stop{};
    if (ns) {
        if (prm->alpha_out && iters > P->rn_cap) return MLBA_EINVAL;  // the device history is one ring
        if (!alg4 || (P->precond != MLBA_PRECOND_BCCB && P->precond != MLBA_PRECOND_DCT)) return MLBA_EUNSUPPORTED;
        if (!stop || !(stop->noise_norm > 0.0) || !(as.ns_rho > 0.0 && as.ns_rho < 0.5) ||
            !(as.ns_q > 2.0 * as.ns_rho && as.ns_q < 1.0) || !(as.alpha0 > 0.0))
            return MLBA_EINVAL;
        ns_stop.noise_norm = stop->noise_norm;
        ns_stop.gamma = (1.0 + 2.0 * as.ns_rho) / (1.0 - 2.0 * as.ns_rho);  // tau of eq. (Alg4_rev_12)
        ns_stop.check_every = 1;
        stop = &ns_stop;
    }
    float mub[64];
    STCHK(expand_mu(P, prm->mu, prm->n_mu, mub));

    // schedules for k = k0 .. k0 + iters (the last entry scales the output)
    std::vector<double> alpha(iters + 1), delta(iters + 1);
    for (int i = 0; i <= iters; ++i) {
        alpha[i] = alpha_at(as, k0 + (i < iters ? i : (iters > 0 ? iters - 1 : 0)));
        if (P->precond != MLBA_PRECOND_NONE && !(alpha[i] > 0.0)) return MLBA_EINVAL;
    }
    if (prm->delta_table) {
        for (int i = 0; i <= iters; ++i) delta[i] = prm->delta_table[k0 + i];
    } else if (prm->delta > 0.0) {
        for (int i = 0; i <= iters; ++i) delta[i] = prm->delta;
    } else if (alg4) {
        for (int i = 0; i <= iters; ++i) delta[i] = 1.0;  // eq. (Alg4) uses the unit step
    } else {
        std::vector<double> seen_a, seen_d;
        for (int i = 0; i <= iters; ++i) {
            size_t j = 0;
            while (j < seen_a.size() && seen_a[j] != alpha[i]) ++j;
            if (j == seen_a.size()) {
                double dl = 0.0;
                STCHK(mlba_internal_auto_delta(P, alpha[i], &dl, s));
                seen_a.push_back(alpha[i]);
                seen_d.push_back(dl);
            }
            delta[i] = seen_d[j];
        }
    }
    for (int i = 0; i <= iters; ++i)
        if (!isfinite(delta[i])) return MLBA_EINVAL;

    const size_t nn = NN(P);
    float* z = z_state ? z_state : (implicit ? P->omega : P->z);
    if (!z_state) HIPCHK(launch_fill(z, implicit ? nn : nn * P->bands, 0.0f, s));

    const bool track = rnorm_out || iters_done || stop;
    std::vector<double> rn_host;
    if (track) rn_host.reserve(iters);
    int done = 0;
    bool stopped = false;
    int ring_base = 0;  // iteration index stored at rn[0]
    auto drain = [&](int upto) -> int {  // copy rn[ring] for iterations [rn_host.size(), upto)
        const int from = (int)rn_host.size();
        if (upto <= from) return MLBA_OK;
        std::vector<double> buf(upto - from);
        HIPCHK(hipMemcpyAsync(buf.data(), P->rn + (from - ring_base), (upto - from) * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (double v : buf) rn_host.push_back(v);
        return MLBA_OK;
    };

    // marks are recorded only inside profiled iterations; every exit path clears them
    struct ProfGuard {
        mlba_plan_s* P;
        ~ProfGuard() { P->prof_cur = -1; }
    } prof_guard{P};
    // The periodic model with the BCCB matrix: A = C, so A^T P_alpha r is
    // Algorithm 4's direction C^T (C C^T + alpha I)^{-1} r; for Algorithm 4,
    // and for MLBA with the blur evaluated by FFTs, the residual is formed in
    // the spectrum (F g computed once here) and an iteration is the synthesis
    // and one 2-D transform pair
    const bool fold4 = (alg4 || (!alg2 && P->blur_fft)) && P->bc == MLBA_BC_PERIODIC &&
                       P->precond == MLBA_PRECOND_BCCB && P->ghat && (P->n / 2 + 1) <= P->partials_cap;
    const bool fused = !fold4 && !alg4 && !alg2 && fused_fft_path(P);
    if (fold4 && iters > 0) {
        HIPCHK(launch_fft_rows_r2c(g, P->n, (float2*)P->swork, P->ts, P->fd, P->tw, s));
        HIPCHK(launch_fft_cols_complex((const float2*)P->swork, P->n, P->ts, P->ghat, P->fd, P->tw, s));
    }
    const bool fused_ar = !ns && !alg2 && fused_ar_path(P);  // MLBA or Algorithm 4
    for (int i = 0; i < iters; ++i) {
        if (i - ring_base >= P->rn_cap) {
            if (track) STCHK(drain(i));
            ring_base = i;
        }
        STCHK(prof_iter_begin(P, s));
        if (implicit) STCHK(do_shrink_synthesis(P, z, P->u, mub, (float)delta[i], s));
        else STCHK(do_synthesis(P, z, P->u, true, mub, (float)delta[i], s));
        int np = 0;
        // the discrepancy stop after ||r^k||^2 is on the device: returns W^T x^k when it holds
        auto check_stop = [&](bool* hit) -> int {
            *hit = false;
            if (!stop || (i % stop->check_every) != 0) return MLBA_OK;
            STCHK(drain(i + 1));
            if (sqrt(rn_host.back()) <= stop->gamma * stop->noise_norm) {
                rn_host.pop_back();
                HIPCHK(hipMemcpyAsync(f_out, P->u, nn * sizeof(float), hipMemcpyDeviceToDevice, s));
                *hit = true;
            }
            return MLBA_OK;
        };
        bool hit = false;
        if (fused) {
            // r = g - A u with P's forward row pass; the partials are summed by P's column pass
            STCHK(do_blur_residual_precond_rows(P, P->u, g, &np, s));
            const float inv = (float)(1.0 / ((double)P->n * (double)P->n));
            if (P->precond == MLBA_PRECOND_DCT) {
                HIPCHK(launch_sum_partials(P->partials, np, P->rn + (i - ring_base), s));
                MARK(BLUR, REDUCE);
                HIPCHK(launch_dct_cols_filter((float*)P->swork, P->n, P->ts, P->spec, (float)alpha[i], inv, P->fd,
                                              P->tw, P->dtw, s, nullptr));
            } else {
                HIPCHK(launch_fft_cols_filter((float2*)P->swork, P->n, P->ts, P->spec, (float)alpha[i], inv, P->fd,
                                              P->tw, s, nullptr, P->partials, np, P->rn + (i - ring_base)));
            }
            MARK(PRECOND, FFT_COLS);
            STCHK(check_stop(&hit));
            if (hit) {
                stopped = true;
                break;
            }
            // P's inverse row pass runs with A^T's forward one
            STCHK(do_precond_rows_blurT(P, implicit ? z : P->w, implicit ? 1 : 0, s));
            if (!implicit) STCHK(do_analysis(P, P->w, z, true, s));
            P->prof_cur = -1;
            done = i + 1;
            continue;
        }
        if (fused_ar) {
            // r = g - A u on the grid; its inverse row pass also runs the
            // transform's forward row pass, and the transform's column pass
            // sums the residual partials
            const int n = P->n, p = P->p, m = n + p - 1;
            float* Tr = (float*)P->swork;
            HIPCHK(launch_fc_rows_fwd(P->fc, P->u, n, P->c, 0, m, s, EXT_ANTIREFLECT));
            MARK(BLUR, FC_ROWS_FWD);
            HIPCHK(launch_fc_cols(P->fc, 0, 0, m, 0, nullptr, s, p - 1, p - 1 + n + (n & 1)));
            MARK(BLUR, FC_COLS);
            HIPCHK(launch_fc_residual_ar_rows(P->fc, n, p, g, P->partials, &np, Tr, P->ts, P->fd, P->tw, s));
            MARK(BLUR, FC_RESIDUAL_PRECOND_ROWS);
            // Algorithm 4: the filter carries lambda (Q' (Q Q' + alpha I)^{-1}) and
            // the direction goes straight into the state, no A' product
            HIPCHK(launch_ar_cols_filter(Tr, n, P->ts, P->spec, (float)alpha[i], alg4 ? P->lamr : nullptr, P->fd,
                                         P->tw, s, P->partials, np, P->rn + (i - ring_base)));
            MARK(PRECOND, FFT_COLS);
            STCHK(check_stop(&hit));
            if (hit) {
                stopped = true;
                break;
            }
            if (alg4) {
                HIPCHK(launch_ar_rows_inv(Tr, n, P->ts, implicit ? z : P->t, P->fd, P->tw, s, implicit ? 1 : 0));
                MARK(PRECOND, FFT_ROWS_INV);
                if (!implicit) STCHK(do_analysis(P, P->t, z, true, s));
                P->prof_cur = -1;
                done = i + 1;
                continue;
            }
            HIPCHK(launch_ar_rows_inv(Tr, n, P->ts, P->t, P->fd, P->tw, s));
            MARK(PRECOND, FFT_ROWS_INV);
            if (implicit) {
                STCHK(do_blurT_acc(P, P->t, z, s));
            } else {
                STCHK(do_blurT(P, P->t, P->w, s));
                STCHK(do_analysis(P, P->w, z, true, s));
            }
            P->prof_cur = -1;
            done = i + 1;
            continue;
        }
        if (fold4) {
            const int n = P->n;
            const float inv = (float)(1.0 / ((double)n * (double)n));
            float2* T = (float2*)P->swork;
            HIPCHK(launch_fft_rows_r2c(P->u, n, T, P->ts, P->fd, P->tw, s));
            MARK(BLUR, FFT_ROWS_FWD);
            HIPCHK(launch_fft_cols_residual(T, n, P->ts, P->ghat, P->lamc, P->spec, (float)alpha[i], inv, P->fd,
                                            P->tw, ns ? 1 : 0, P->partials, &np, s));
            MARK(PRECOND, FFT_COLS);
            HIPCHK(launch_sum_partials(P->partials, np, P->rn + (i - ring_base), s));
            MARK(BLUR, REDUCE);
            STCHK(check_stop(&hit));
            if (hit) {
                stopped = true;
                break;
            }
            if (ns) {  // T holds F r: alpha_n, then the filter and the inverse column transform
                HIPCHK(launch_ns_alpha(T, 0, n, P->ts, P->spec, P->ns, P->partials, P->rn + (i - ring_base),
                                       stop->noise_norm, as.ns_q, as.ns_rho, as.alpha0, i == 0 ? 1 : 0,
                                       kNsSteps, P->ahist + (i - ring_base), s));
                STCHK(prof_mark(P, MLBA_PHASE_PRECOND, MLBA_KERNEL_OTHER, ns_alpha_launches(kNsSteps), s));
                HIPCHK(launch_fft_cols_filter_inverse(T, n, P->ts, P->spec, P->ns, inv, P->lamc, P->fd, P->tw, s));
                MARK(PRECOND, FFT_COLS);
            }
            HIPCHK(launch_fft_rows_c2r(T, n, P->ts, implicit ? z : P->t, P->fd, P->tw, s, implicit ? 1 : 0));
            MARK(PRECOND, FFT_ROWS_INV);
            if (!implicit) STCHK(do_analysis(P, P->t, z, true, s));
            P->prof_cur = -1;
            done = i + 1;
            continue;
        }
        // Algorithm 2 on the fused FFT path: the residual's inverse row pass
        // also runs P's forward row pass of r (the PCG's first P application)
        const bool pcg_rows = alg2 && pcg_fused_start(P);
        if (pcg_rows) {
            STCHK(blur_grid_forward(P, P->u, s));
            HIPCHK(launch_fc_residual_precond_rows(P->fc, P->n, P->p, g, P->r, P->partials, &np, precond_rows(P), s));
            MARK(BLUR, FC_RESIDUAL_PRECOND_ROWS);
        } else {
            STCHK(do_blur(P, P->u, g, P->r, true, &np, s));
        }
        HIPCHK(launch_sum_partials(P->partials, np, P->rn + (i - ring_base), s));
        MARK(BLUR, REDUCE);
        STCHK(check_stop(&hit));
        if (hit) {
            stopped = true;
            break;
        }
        if (alg4) {
            // eq. (Alg4): the direction C^T (C C^T + alpha I)^{-1} r, no A^T product
            float* dst = implicit ? z : P->t;
            if (ns) {
                STCHK(do_ct_precond_ns(P, P->r, dst, P->rn + (i - ring_base), stop->noise_norm, as.ns_q,
                                       as.ns_rho, as.alpha0, i == 0 ? 1 : 0, P->ahist + (i - ring_base),
                                       implicit ? 1 : 0, s));
            } else {
                STCHK(do_ct_precond(P, P->r, dst, alpha[i], implicit ? 1 : 0, s));
            }
            if (!implicit) STCHK(do_analysis(P, P->t, z, true, s));
            P->prof_cur = -1;
            done = i + 1;
            continue;
        }
        if (alg2) {
            const int cur = P->prof_cur;  // the PCG is timed as one sequence
            P->prof_cur = -1;
            STCHK(do_pcg(P, alpha[i], pcg_max, pcg_tol, P->pcgh + i, pcg_rows, s));
            P->prof_cur = cur;
            STCHK(prof_mark(P, MLBA_PHASE_PRECOND, MLBA_KERNEL_OTHER, 1, s));
            float* tsol = P->pcg;  // the CG solution t
            if (implicit) {
                STCHK(do_blurT_acc(P, tsol, z, s));
            } else {
                STCHK(do_blurT(P, tsol, P->w, s));
                STCHK(do_analysis(P, P->w, z, true, s));
            }
            P->prof_cur = -1;
            done = i + 1;
            continue;
        }
        STCHK(do_precond(P, P->r, P->t, alpha[i], s));
        if (implicit) {
            STCHK(do_blurT_acc(P, P->t, z, s));
        } else {
            STCHK(do_blurT(P, P->t, P->w, s));
            STCHK(do_analysis(P, P->w, z, true, s));
        }
        P->prof_cur = -1;
        done = i + 1;
    }
    P->prof_cur = -1;
    if (!stopped) {
        if (implicit) STCHK(do_shrink_synthesis(P, z, f_out, mub, (float)delta[done], s));
        else STCHK(do_synthesis(P, z, f_out, true, mub, (float)delta[done], s));
    }

    if (prm->delta_out)
        for (int i = 0; i <= done; ++i) prm->delta_out[i] = delta[i];
    if (alg2 && prm->pcg_steps_out && done > 0) {
        HIPCHK(hipMemcpyAsync(prm->pcg_steps_out, P->pcgh, (size_t)done * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (prm->alpha_out && done > 0) {
        if (ns) {
            HIPCHK(hipMemcpyAsync(prm->alpha_out, P->ahist, (size_t)done * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            for (int i = 0; i < done; ++i) prm->alpha_out[i] = alpha[i];
        }
    }
    int status = MLBA_OK;
    if (track) {
        STCHK(drain(done));
        rn_host.resize(done);
        double first = -1.0;
        for (int i = 0; i < done; ++i) {
            const double v = sqrt(rn_host[i]);
            if (rnorm_out) rnorm_out[i] = v;
            if (first < 0.0) first = v;
            if (!isfinite(v) || v > 1e3 * first) status = MLBA_WARN_DIVERGED;
        }
        if (iters_done) *iters_done = done;
    }
    return note_work(P, status, s);
}

int mlba_profile_begin(mlba_plan_t P, int max_iters) {
    if (!P || max_iters < 1 || max_iters > (1 << 16)) return MLBA_EINVAL;
    release_events(P);
    const size_t count = (size_t)max_iters * kMarks;
    P->prof_ev.reserve(count);
    for (size_t i = 0; i < count; ++i) {
        hipEvent_t e;
        // timestamps only: no system-scope fence when the event completes
        hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        if (err != hipSuccess) {
            mlba_internal_set_hip(err);
            release_events(P);
            return MLBA_EHIP;
        }
        P->prof_ev.push_back(e);
    }
    P->prof_phase.assign(count, 0);
    P->prof_kernel.assign(count, 0);
    P->prof_nl.assign(count, 0);
    P->prof_nm.assign((size_t)max_iters, 0);
    P->prof_cap = max_iters;
    P->prof_used = 0;
    P->prof_cur = -1;
    P->prof_seen = 0;
    P->prof_stride = 1;
    return MLBA_OK;
}

int mlba_profile_every(mlba_plan_t P, int stride) {
    if (!P || stride < 1) return MLBA_EINVAL;
    P->prof_stride = stride;
    P->prof_seen = 0;
    return MLBA_OK;
}

int mlba_profile_end(mlba_plan_t P, double* ms, int* launches, int* iters) {
    if (!P || !ms) return MLBA_EINVAL;
    for (int q = 0; q < MLBA_NPHASES; ++q) {
        ms[q] = 0.0;
        if (launches) launches[q] = 0;
    }
    for (int k = 0; k < MLBA_NKERNELS; ++k) {
        P->prof_kms[k] = 0.0;
        P->prof_kl[k] = 0;
    }
    for (int it = 0; it < P->prof_used; ++it) {
        const size_t b = (size_t)it * kMarks;
        const int nm = P->prof_nm[it];
        if (nm < 2) continue;
        HIPCHK(hipEventSynchronize(P->prof_ev[b + nm - 1]));
        for (int m = 1; m < nm; ++m) {
            float t = 0.0f;
            HIPCHK(hipEventElapsedTime(&t, P->prof_ev[b + m - 1], P->prof_ev[b + m]));
            const int ph = P->prof_phase[b + m], k = P->prof_kernel[b + m], nl = P->prof_nl[b + m];
            ms[ph] += (double)t;
            if (launches) launches[ph] += nl;
            P->prof_kms[k] += (double)t;
            P->prof_kl[k] += nl;
        }
    }
    if (iters) *iters = P->prof_used;
    release_events(P);
    return MLBA_OK;
}

int mlba_profile_kernels(mlba_plan_t P, double* ms, int* launches) {
    if (!P || !ms) return MLBA_EINVAL;
    for (int k = 0; k < MLBA_NKERNELS; ++k) {
        ms[k] = P->prof_kms[k];
        if (launches) launches[k] = P->prof_kl[k];
    }
    return MLBA_OK;
}

}  // extern "C"
