// Internal plan layout shared by the library's host translation units.
#pragma once

#include <vector>

#include "kernels.hpp"
#include "mlba.h"

int mlba_internal_last_hip();
// Run-time transform plan of length n (mixed radix, or the Bluestein form).
mlba::FftDesc mlba_internal_fft_desc(int n);
void mlba_internal_set_hip(hipError_t e);

#define HIPCHK(expr)                         \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) {              \
            mlba_internal_set_hip(e_);       \
            return MLBA_EHIP;                \
        }                                    \
    } while (0)

#define STCHK(expr)              \
    do {                         \
        int st_ = (expr);        \
        if (st_ < 0) return st_; \
    } while (0)

struct mlba_plan_s {
    int n = 0, p = 0, c = 0, N = 0, bc = 0, precond = 0, levels = 0, bands = 0;
    mlba::FftDesc fd{};
    int ts = 0;                // row stride of the transposed spectral workspace
    int conv_rows[2] = {0, 0}; // output rows per thread of the A / A^T blur (0: by occupancy)
    int blur_fft = 0;          // rectangular model: A and A^T by FFTs of an M x M grid
    mlba::FftConv fc{};        // its plan and buffers (allocated on first use)
    float* psf = nullptr;
    float* spec = nullptr;     // BCCB: [n/2+1][n] |Lambda|^2 (transposed); DCT, AR: [n][n] lambda^2
    float2* lamc = nullptr;    // square models, BCCB: Lambda_c of the centred PSF (layout of spec)
    float2* ghat = nullptr;    // periodic model, BCCB: F g of the current restoration (layout of spec)
    float* lamr = nullptr;     // square models, DCT and AR: lambda (layout of spec)
    double* ns = nullptr;      // Algorithm 4-NS device state
    double* ahist = nullptr;   // alpha_k used (ring like rn)
    float* pcg = nullptr;      // Algorithm 2: t, z, d, q (n x n each)
    double* pcgs = nullptr;    // Algorithm 2 scalars: rho (two slots), pq, rho0, running flag
    int* pcgh = nullptr;       // Algorithm 2: beta_n of each iteration (rn_cap entries)
    float2* tw = nullptr;      // exp(-2 pi i q / L), L = fd.n (n; 2(n-1) for AR)
    float2* dtw = nullptr;     // exp(-i pi k / (2n))
    float* costab = nullptr;   // cos(pi q / n), q < 2n (AR: cos(pi q / (n-1)), q < 2(n-1))
    void* swork = nullptr;     // spectral workspace
    float* u = nullptr;        // N x N synthesis output
    float* r = nullptr;        // n x n residual
    float* t = nullptr;        // n x n preconditioned residual
    float* w = nullptr;        // N x N A^T t
    float* wext = nullptr;     // m x m full correlation (reflective boundary)
    float* tmp[2] = {nullptr, nullptr};  // N x N level intermediates
    float* pv = nullptr;       // N x N power-iteration vector
    float* z = nullptr;        // [bands][N][N] state when the caller passes none
    float* omega = nullptr;    // N x N implicit state (z = W omega) when the caller passes none
    float* lows[3] = {nullptr, nullptr, nullptr};  // low-pass chain low_1 .. low_{levels-1} (N x N)
    double* partials = nullptr;
    int partials_cap = 0;
    double* scal = nullptr;    // device scalars
    double* rn = nullptr;      // ||r^k||^2 history ring
    int rn_cap = 0;
    std::vector<void*> allocs;
    hipEvent_t done = nullptr;  // recorded after every call that enqueues work
    // kernel timing (mlba_profile_begin / end): per profiled iteration one
    // start event and up to kMaxMarks - 1 marks, each an event recorded after
    // a launch (or a launch sequence) and labelled with the phase and kernel
    // whose time since the previous event it measures
    static constexpr int kMaxMarks = 48;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_phase, prof_kernel, prof_nl, prof_nm;
    int prof_cap = 0, prof_used = 0, prof_cur = -1;
    int prof_stride = 1, prof_seen = 0;  // record every prof_stride-th iteration
    double prof_kms[MLBA_NKERNELS] = {};  // per kernel, from the last mlba_profile_end
    int prof_kl[MLBA_NKERNELS] = {};
};

// ||A^T P_alpha A||: Lanczos (at most `iters` steps, stopping once the largest
// Ritz value changes by at most `tol` relative over 8 steps) for the
// symmetric models; power iteration (`iters` steps) on A' P_alpha A for the
// antireflective model.
int mlba_internal_opnorm(mlba_plan_s* P, double alpha, int iters, double tol, double* out, int* steps_out,
                         hipStream_t s);
// The automatic step of the convergence theorem of section 3:
// delta = 0.9 / max(||A^T P_alpha A||, 0.9).
constexpr int kAutoLanczosSteps = 1000;
constexpr double kAutoLanczosTol = 1e-9;
constexpr int kAutoPowerSteps = 50;
int mlba_internal_auto_delta(mlba_plan_s* P, double alpha, double* delta, hipStream_t s);
// Newton steps for alpha_n of Algorithm 4-NS in every iteration.
constexpr int kNsSteps = 12;

// Descriptor of a plan's sizes and buffers (the per-image record of a batch;
// the single-image path builds the same record so both run identical jobs).
inline mlba::BatchImage plan_desc(const mlba_plan_s* P) {
    mlba::BatchImage d{};
    d.n = P->n;
    d.p = P->p;
    d.c = P->c;
    d.N = P->N;
    d.bc = P->bc;
    d.precond = P->precond;
    d.levels = P->levels;
    d.bands = P->bands;
    d.ts = P->ts;
    d.u = P->u;
    d.r = P->r;
    d.t = P->precond == MLBA_PRECOND_NONE ? P->r : P->t;
    d.w = P->w;
    d.wext = P->wext;
    d.tmp0 = P->tmp[0];
    d.tmp1 = P->tmp[1];
    d.z = P->z;
    d.zin = P->z;
    d.psf = P->psf;
    d.spec = P->spec;
    d.swork = P->swork;
    d.tw = P->tw;
    d.dtw = P->dtw;
    d.fd = P->fd;
    d.state_planes = P->bands;
    d.blur_acc = 0;
    for (int l = 0; l < 3; ++l) d.lows[l] = P->lows[l];
    if (P->precond == MLBA_PRECOND_AR) {  // one row pair per workgroup
        d.fft_rows_g = d.fft_cols_c = 1;
        d.fft_rows_shift = d.fft_cols_shift = mlba::fft_seq_shift(1);
    } else if (P->precond != MLBA_PRECOND_NONE) {
        d.fft_rows_g = mlba::fft_rows_batch(P->n);
        d.fft_cols_c = mlba::fft_cols_batch(P->n);
        d.fft_rows_shift = mlba::fft_seq_shift(d.fft_rows_g);
        d.fft_cols_shift = mlba::fft_seq_shift(d.fft_cols_c);
    }
    return d;
}
