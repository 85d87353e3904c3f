// Internal launcher interface between the kernel translation units and the
// C ABI implementation.  Every launcher enqueues on `s` and returns the
// hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace mlba {

// Mixed-radix plan of a length-n complex FFT (n = 2^a 3^b 5^c).
// Run-time transform plan of length n.  m == 0: Stockham stages of radix
// radix[0..nst) over n itself (n = 2^a 3^b 5^c).  m > 0 (any other n): the
// Bluestein form, a circular convolution of length m >= 2n - 1 (m 5-smooth),
// and radix[] are the stages of m; the table then holds the m twiddles, the
// chirp exp(-i pi k^2 / n) (k < n) and the spectrum of the conjugate chirp
// divided by m (m values), in that order.
struct FftDesc {
    int n;
    int nst;
    int radix[24];
    int m;
};

// Soft-threshold parameters of one framelet level: mu of the low-pass input
// (used when it is thresholded) and mu of the eight detail bands.
struct LevelMu {
    float low;
    float band[8];
};

struct BandMu {
    float v[64];
};

// Shrink-synthesis coefficients of one level (implicit state): per band (i, j)
// the threshold of the coefficient computed with the unnormalised masks and
// its synthesis weight (see shrink.hip).
struct SsCoef {
    float thr[3][3];
    float wgt[3][3];
};
// The coefficients of a level from its thresholds and the step; from_above:
// the (0, 0) input is the output of the level above (unthresholded).
SsCoef ss_coef(const LevelMu& mu, float delta, bool from_above);

// One blur: dst[y][x] = (g ? g[y][x] - s : (acc ? dst[y][x] + s : s)) over D x D
// outputs, s = sum_{a,b} K[a][b] src_ext[y+org+a][x+org+b] (src S x S, extension ext).
struct ConvJob {
    const float* src;
    int S, ext, org;
    float* dst;
    int D;
    const float* g;
    const float* psf;
    int acc;
};

// Per-image descriptor of a batch (device memory): sizes, model, parameters
// and the plan's buffers.  All images of a batch share the framelet depth.
struct BatchImage {
    int n, p, c, N, bc, precond, levels, bands, ts;
    int fft_rows_g, fft_cols_c, fft_rows_shift, fft_cols_shift;  // transform batching
    int pbase;  // first residual-norm partial of this image
    float alpha, delta;
    float mu[33];
    const float* g;
    float* f;
    float* z;          // state written by the analysis update
    const float* zin;  // state read by the synthesis and by the update (z unless a step writes a new slot)
    float* u;
    float* r;
    float* t;
    float* w;
    float* wext;
    float* tmp0;
    float* tmp1;
    const float* psf;
    const float* spec;
    void* swork;
    const float2* tw;
    const float2* dtw;
    double* rn;  // ||r^k||^2 per iteration
    // implicit state (z = W omega): z holds omega (state_planes = 1, else
    // bands); the A^T blur accumulates into w (= omega) when blur_acc; the
    // low-pass chain low_1 .. low_{levels-1}; the shrink-synthesis
    // coefficients of levels 1 .. levels
    int state_planes;
    int blur_acc;
    float* lows[3];
    SsCoef ss[4];
    // reverse sweep of unrolled iterations (null elsewhere)
    float2* sstore;      // the preconditioner's filtered spectrum is stored here ([n/2+1][n])
    const float2* sfwd;  // filtered spectrum of the forward step being reversed
    float* eacc;         // += Re(conj(filtered) * sfwd), dense [n/2+1][n]
    const float* zk;     // forward state z_k: its active set masks the cotangent update
    float* zbar;         // state cotangent [bands][N][N]
    const float* tk;     // forward t_k = P r_k (n x n)
    const float* uk;     // forward u_k = W^T(delta S_mu(z_k)) (N x N)
    float* dg;           // gradient of the observation (n x n)
    FftDesc fd;
};

__host__ __device__ inline int ext_of_bc(int bc) {  // REFLECT, PERIODIC, ANTIREFLECT, else zero
    return bc == 1 ? EXT_REFLECT : (bc == 2 ? EXT_PERIODIC : (bc == 4 ? EXT_ANTIREFLECT : EXT_ZERO));
}

// r = g - A u  (section 2: valid convolution of the (extended) unknown)
__host__ __device__ inline ConvJob blur_job(const BatchImage& I) {
    ConvJob j;
    j.src = I.u;
    j.S = I.N;
    j.ext = ext_of_bc(I.bc);
    j.org = I.bc == 0 ? 0 : -I.c;
    j.dst = I.r;
    j.D = I.n;
    j.g = I.g;
    j.psf = I.psf;
    j.acc = 0;
    return j;
}

// w = A^T t (full correlation; the reflective model writes the padded grid
// wext, folded afterwards).  Zero and periodic models: the correlation of the
// extended t, which is their exact transpose.  Antireflective model: the same
// correlation of the antireflected t, i.e. the reblurring A' (the blur with
// the PSF rotated by 180 degrees, section 2.2) that replaces A^T there.
__host__ __device__ inline ConvJob blurT_job(const BatchImage& I) {
    ConvJob j;
    j.src = I.t;
    j.S = I.n;
    j.g = nullptr;
    j.psf = I.psf;
    j.acc = 0;
    if (I.bc == 0 || I.bc == 1) {
        j.ext = EXT_ZERO;
        j.org = -(I.p - 1);
        j.dst = I.bc == 0 ? I.w : I.wext;
        j.D = I.n + I.p - 1;
    } else {
        j.ext = ext_of_bc(I.bc);
        j.org = -I.c;
        j.dst = I.w;
        j.D = I.n;
    }
    if (j.dst == I.w) j.acc = I.blur_acc;  // the reflective model accumulates in its fold
    return j;
}

// ---- blur (direct convolution) -------------------------------------------
// dst[y][x] = (g ? g[y][x] - s : s),  s = sum_{a,b} K[a][b] src_ext[y+org+a][x+org+b]
// with K = H rotated by 180 degrees (flip = 1, the blur A) or K = H
// (flip = 0, the correlation of A^T).  src is S x S, dst is D x D.
// partials (optional, needs g): one double per workgroup with sum of dst^2.
hipError_t launch_conv(const float* src, int S, int ext, int org, float* dst, int D,
                       const float* g, const float* psf, int p, int flip, double* partials,
                       int* n_partials, hipStream_t s);
// ry: output rows per thread (1 or 2; other values pick by occupancy)
hipError_t launch_conv_job(const ConvJob& j, int p, int flip, int ry, double* partials, int* n_partials,
                           hipStream_t s);
int conv_partials_count(int D);
int conv_default_rows(int D, int p);
int conv_tiles(int D, int ry);
// batched: tiles of every image in one launch (flip = 1: residual, 0: A^T);
// ry = output rows per thread (1 or 2) of the images with p <= 33
int conv_batched_tiles(const BatchImage& I, int flip, int ry = 1);
hipError_t launch_conv_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                               int flip, int pmax, double* partials, hipStream_t s, int ry = 1);
hipError_t launch_fold_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                               hipStream_t s);

// Transpose of the reflective padding: w[y][x] = sum of wext over the
// positions of the (n+2c)^2 padded grid that copy pixel (y, x).
hipError_t launch_fold_reflect(const float* wext, int m, float* w, int n, int c, hipStream_t s, int accum = 0);

// ---- blur by FFTs (rectangular model) -------------------------------------
// M x M grid, M >= N = n + p - 1, M = 2^a 3^b <= fftconv_max_size(); T: half
// spectrum workspace [M/2+1][ts], H: spectrum of the PSF at the origin
// (dense [M/2+1][M]).
struct FftConv {
    int M, ts;
    FftDesc fd;
    const float2* tw;
    float2* T;
    float2* H;
    // the PSF's rows transformed along x on the grid, G[k * p + a] for the
    // half-spectrum column k and PSF row a (null: the column pass always
    // transforms)
    float2* G;
    int p;
};
int fftconv_max_size();
int fftconv_partials_count(int M, int n);
// PSF sizes with a compiled direct column pass (FftConv::G)
bool fftconv_direct_taps(int p);
hipError_t launch_fftconv_spectrum(const FftConv& c, const float* psf, int p, hipStream_t s);

// The transposed half spectrum of the BCCB preconditioner (n x n, row stride
// ts complex) and its transform plan, for the passes fused with the FFT blur.
struct PrecondRows {
    float2* T;            // BCCB: the transposed half spectrum; DCT: the real coefficients (float)
    int ts;
    FftDesc fd;
    const float2* tw;
    const float2* dtw;    // DCT plan: the DCT twiddles (null: BCCB)
};
// The three passes of the FFT blur, one launch each: forward rows of the
// S x S image placed at (off, off) (rows outside [y_lo, y_hi) are zero; `ext`
// other than EXT_ZERO: with its pad of width off around it under that
// extension, i.e. E src E^T at 0), columns (mode 0: product with the PSF
// spectrum or its conjugate and the inverse, stored for the rows
// [o_lo, o_hi) only, whole row pairs; mode 1: forward only into cspec),
// inverse rows cropped to the D x D window at (oy, ox) with the epilogue
// g - . (partials) / plain / +=.  fold >= 0 (an Ext of a square model, fn x fn
// image, pad fcn): the column pass stores E^T along the columns in rows
// [0, fn + (fn & 1)) and the row pass (oy = ox = 0, D = fn) applies E^T along
// the rows.  conj_h: the column product with H (0), conj(H) (1) or |H|^2 (2).
// axd: the row pass writes v + axa axd with the partials of sum axd (v + axa axd).
// Algorithm 2's direction update folded into a forward row pass (src == d):
// d = z + (*rho_new / *rho) d while *act != 0; rho_new null: d = z
struct PcgDir {
    float* d;
    const float* z;
    const double* rho_new;
    const double* rho;
    const double* act;
};
hipError_t launch_fc_rows_fwd(const FftConv& c, const float* src, int S, int off, int y_lo, int y_hi, hipStream_t s,
                              int ext = EXT_ZERO, const PcgDir* dir = nullptr);
hipError_t launch_fc_cols(const FftConv& c, int conj_h, int y_lo, int y_hi, int mode, float2* cspec, hipStream_t s,
                          int o_lo, int o_hi, int fold = -1, int fn = 0, int fcn = 0);
hipError_t launch_fc_rows_inv(const FftConv& c, int oy, int ox, int D, float* dst, const float* g, int accum,
                              double* partials, int* n_partials, hipStream_t s, int fold = -1, int fcn = 0,
                              const float* axd = nullptr, float axa = 0.0f);
// Row passes fused with the preconditioner's (n even, n <= 2048):
// the residual rows r = g - A u (after launch_fc_cols of u) with their
// squared-norm partials, then the preconditioner's forward row transform of r
// into pr.T (r written only when r_out is given);
hipError_t launch_fc_residual_precond_rows(const FftConv& c, int n, int p, const float* g, float* r_out,
                                           double* partials, int* n_partials, const PrecondRows& pr, hipStream_t s);
// the preconditioner's inverse row transform of pr.T (t = P r, written to
// t_out when given), then the forward rows of A^T t on the grid (followed by
// launch_fc_cols with the conjugate spectrum and launch_fc_rows_inv).
hipError_t launch_precond_rows_fc_fwd(const FftConv& c, int n, int p, const PrecondRows& pr, float* t_out,
                                      hipStream_t s);
bool fftconv_fusable(const FftConv& c, int n, const PrecondRows& pr);
// Antireflective model with the antireflective transform: the residual's
// inverse row pass and the transform's forward row pass in one launch (one
// observed row pair per workgroup, (n + 1) / 2 partials of ||r||^2); fdl / twl
// describe the transform's length 2(n - 1), Tr its workspace (row stride tsr).
bool fftconv_ar_fusable(const FftConv& c, int n, const FftDesc& fdl);
hipError_t launch_fc_residual_ar_rows(const FftConv& c, int n, int p, const float* g, double* partials,
                                     int* n_partials, float* Tr, int tsr, const FftDesc& fdl, const float2* twl,
                                     hipStream_t s);

// ---- framelet -----------------------------------------------------------
// analysis level with dilation d: bands (+)= B_i B_j v, low (+)= B_0 B_0 v
hipError_t launch_analysis_level(const float* v, int N, int d, float* zlev, float* low,
                                 int accum_bands, int accum_low, hipStream_t s);
// synthesis level with dilation d (transpose), optional threshold of inputs
hipError_t launch_synthesis_level(const float* zlev, const float* low, int N, int d, float* out,
                                  LevelMu mu, float delta, int thr_low, int thr_bands,
                                  hipStream_t s);
hipError_t launch_soft_threshold(const float* z, float* x, int bands, size_t band_elems,
                                 BandMu mu, float delta, hipStream_t s);
// implicit state (z = W omega): low-pass of one level, out = (b0 x b0) v
hipError_t launch_lowpass_level(const float* v, int N, int d, float* out, hipStream_t s);
// one level of W^T(delta S_mu(W omega)) from low = low_{l-1}; s_in = output of
// the level above, or null at the top level (thresholded low-pass)
// low1 = (b0 x b0) v, low2 = (b0 x b0) low1 (dilations 1 and 2) in one pass
hipError_t launch_lowpass_two_levels(const float* v, int N, float* low1, float* low2, hipStream_t s);
// batched implicit state: level `lev` of the low-pass chain (low_lev from
// low_{lev-1}, dilation d = 2^(lev-1)) and the shrink-synthesis of level lev
// (final_out: level 1 writes f instead of u), over the tiles of all images
int lowpass_level_tiles(int N);
int shrink_level_tiles(int N, int d);
hipError_t launch_lowpass_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks, int lev,
                                  int d, hipStream_t s);
hipError_t launch_shrink_synthesis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                           int lev, int d, int top, int final_out, hipStream_t s);
hipError_t launch_shrink_synthesis_level(const float* low, const float* s_in, int N, int d, float* out,
                                         LevelMu mu, float delta, hipStream_t s);
// batched framelet levels (all images share `levels`); tiles per image:
int synthesis_level_tiles(int N, int d);
int analysis_level_tiles(int N, int d);
// synthesis of level `lev` (thresholded input when thr, else plain W^T); final_out:
// level 1 writes f, else u
hipError_t launch_synthesis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                    int lev, int d, int final_out, hipStream_t s, int thr = 1);
// z += W w, level `lev`
hipError_t launch_analysis_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                   int lev, int d, hipStream_t s);
hipError_t launch_fill_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                               hipStream_t s);  // z = 0, 256 * 1024 elements per workgroup
int fill_tiles(const BatchImage& I);
// Reverse sweep, level `lev` of v = W w with the cotangent update applied to
// every band it produces (the low-pass of inner levels goes to tmp as usual):
//   init:  zbar_b  = delta 1{|zk_b| > mu_b} v_b,  part += -delta sgn(zk) 1{..} v
//   else:  zbar_b -= delta 1{|zk_b| > mu_b} v_b,  part += +delta sgn(zk) 1{..} v
// Input: w (level 1), else the previous level's low-pass.
// part: running per-workgroup band sums [nblocks][9] (slot 8 = low-pass).
int analysis_adjoint_tiles(int N, int d);
hipError_t launch_analysis_adjoint_batched(const BatchImage* imgs, const int* bmap, const int* bfirst,
                                           int nblocks, int lev, int d, int init, double* part, hipStream_t s);

// ---- spectral preconditioner --------------------------------------------
// BCCB: rows r2c -> T (half spectrum, transposed [n/2+1][ts] complex; the row
// stride ts = n + 16 keeps the transposed accesses off a single memory channel)
hipError_t launch_fft_rows_r2c(const float* src, int n, float2* T, int ts, const FftDesc& fd,
                               const float2* tw, hipStream_t s);
// columns: forward FFT, scale by inv / (spec + alpha) (times conj(lamc) when
// given: the C^T (C C^T + alpha I)^{-1} of Algorithm 4), inverse FFT (in place);
// red_out (optional): the first workgroup also writes the sum of red_count
// partials (the previous launch's) to *red_out
hipError_t launch_fft_cols_filter(float2* T, int n, int ts, const float* spec, float alpha, float inv,
                                  const FftDesc& fd, const float2* tw, hipStream_t s, const float2* lamc = nullptr,
                                  const double* red_in = nullptr, int red_count = 0, double* red_out = nullptr);
// columns, Algorithm 4 with the periodic model (A = C): forward FFT, R = ghat -
// lamc * (F u) with the partial of ||r||^2 = sum |R|^2 / n^2 per workgroup
// into part (*n_part partials), then the direction conj(lamc) R inv /
// (spec + alpha) and the inverse FFT, or (store_r) R itself
hipError_t launch_fft_cols_residual(float2* T, int n, int ts, const float2* ghat, const float2* lamc,
                                    const float* spec, float alpha, float inv, const FftDesc& fd, const float2* tw,
                                    int store_r, double* part, int* n_part, hipStream_t s);
// columns: forward FFT only (T then holds the 2-D half spectrum)
hipError_t launch_fft_cols_forward(float2* T, int n, int ts, const FftDesc& fd, const float2* tw, hipStream_t s);
// columns: the filter of launch_fft_cols_filter with alpha read on the device, inverse FFT
hipError_t launch_fft_cols_filter_inverse(float2* T, int n, int ts, const float* spec, const double* alpha_dev,
                                          float inv, const float2* lamc, const FftDesc& fd, const float2* tw,
                                          hipStream_t s);
// columns: forward FFT, complex values into cspec (dense [n/2+1][n])
hipError_t launch_fft_cols_complex(const float2* T, int n, int ts, float2* cspec, const FftDesc& fd,
                                   const float2* tw, hipStream_t s);
// Algorithm 2's PCG vectors (device): t += a d and res -= a q with
// a = *rho / *pq while *act != 0
struct PcgVec {
    float* t;
    float* res;
    const float* d;
    const float* q;
    const double* rho;
    const double* pq;
    const double* act;
};
// BCCB plan: P's forward row pass with the step's update applied to res (and
// t) first; P's inverse row pass writing z with the partials of res . z
// (pcg_rows_c2r_partials(n) of them)
hipError_t launch_pcg_rows_r2c(int n, float2* T, int ts, const FftDesc& fd, const float2* tw, const PcgVec& v,
                               hipStream_t s);
hipError_t launch_pcg_rows_c2r(const float2* T, int n, int ts, float* z, const float* res, const FftDesc& fd,
                               const float2* tw, double* part, int* n_part, hipStream_t s);
int pcg_rows_c2r_partials(int n);
// pcg_begin after summing the np partials of rho_0 into st[0] (one workgroup)
hipError_t launch_pcg_begin_sum(double* st, const double* part, int np, int* hist, hipStream_t s);
// pcg_check after summing the np partials of rho_j into *rn (one workgroup)
hipError_t launch_pcg_check_sum(double* st, const double* part, int np, double* rn, int j, int max_steps,
                                double tol, int* hist, hipStream_t s);
// Algorithm 4-NS: alpha_n on the device from the BCCB half spectrum T
// (float2, real = 0) or the DCT coefficients (float, real = 1); state:
// ns_state_doubles() device doubles (launch_ns_psf_l1 after every PSF
// change), alpha_n at state[0]; hist: a device double or null; part: at
// least ns_partials_needed() device doubles
hipError_t launch_ns_alpha(const void* T, int real, int n, int ts, const float* spec, double* state, double* part,
                           const double* rn_sq, double noise, double q, double rho, double alpha_first, int first,
                           int steps, double* hist, hipStream_t s);
hipError_t launch_ns_psf_l1(const float* psf, int p, double* state, hipStream_t s);
int ns_partials_needed();
int ns_state_doubles();
int ns_alpha_launches(int steps);  // kernels launch_ns_alpha enqueues
// columns: forward FFT, write spec = |.|^2 (same transposed layout)
hipError_t launch_fft_cols_power(const float2* T, int n, int ts, float* spec, const FftDesc& fd,
                                 const float2* tw, hipStream_t s);
hipError_t launch_fft_rows_c2r(const float2* T, int n, int ts, float* dst, const FftDesc& fd,
                               const float2* tw, hipStream_t s, int accum = 0);  // accum: dst +=
// DCT: rows DCT-II -> Tr (transposed, real [n][n]); columns DCT-II, filter,
// DCT-III; rows DCT-III -> dst.  Unnormalised transforms; `inv` carries 1/n^2.
hipError_t launch_dct_rows_fwd(const float* src, int n, float* Tr, int ts, const FftDesc& fd,
                               const float2* tw, const float2* dtw, hipStream_t s);
hipError_t launch_dct_cols_filter(float* Tr, int n, int ts, const float* spec, float alpha, float inv,
                                  const FftDesc& fd, const float2* tw, const float2* dtw,
                                  hipStream_t s, const float* lamr = nullptr);  // lamr: times lambda (Alg. 4)
hipError_t launch_dct_rows_inv(const float* Tr, int n, int ts, float* dst, const FftDesc& fd,
                               const float2* tw, const float2* dtw, hipStream_t s, int accum = 0);
// columns: DCT-II only (Tr then holds the 2-D coefficients), and the filter
// inv lamr / (spec + alpha_dev[0]) with the DCT-III from those coefficients (Algorithm 4-NS)
hipError_t launch_dct_cols_forward(float* Tr, int n, int ts, const FftDesc& fd, const float2* tw, const float2* dtw,
                                   hipStream_t s);
hipError_t launch_dct_cols_filter_inverse(float* Tr, int n, int ts, const float* spec, const double* alpha_dev,
                                          float inv, const float* lamr, const FftDesc& fd, const float2* tw,
                                          const float2* dtw, hipStream_t s);
// spec[kx][ky] = lambda[ky][kx]^2 of the symmetrised PSF's cosine spectrum,
// lambda itself into lam when given: K = n with costab[q] = cos(pi q / n)
// for the reflective blur (Algorithm 3); K = n - 1, costab[q] = cos(pi q /
// (n-1)) and lin_last = 1 for the antireflective blur.  tmp: p x n floats.
hipError_t launch_cos_spectrum(const float* psf, int p, int n, int K, int lin_last, const float* costab, float* tmp,
                               float* spec, float* lam, hipStream_t s);
// Antireflective transform (Algorithm 3 with antireflective boundaries): rows
// T^-1 -> Tr (transposed, real, row stride ts = ar_workspace_stride(n), n
// rows); columns T^-1, filter 1/(spec + alpha) (times lamr), T; rows T -> dst.
// fd / tw describe the complex FFT of length 2(n - 1).
bool ar_transform_supported(int n);
int ar_workspace_stride(int n);
hipError_t launch_ar_rows_fwd(const float* src, int n, float* Tr, int ts, const FftDesc& fd, const float2* tw,
                              hipStream_t s);
hipError_t launch_ar_cols_filter(float* Tr, int n, int ts, const float* spec, float alpha, const float* lamr,
                                 const FftDesc& fd, const float2* tw, hipStream_t s, const double* red_in = nullptr,
                                 int red_count = 0, double* red_out = nullptr);  // red_*: see fft_cols
hipError_t launch_ar_rows_inv(const float* Tr, int n, int ts, float* dst, const FftDesc& fd, const float2* tw,
                              hipStream_t s, int accum = 0);
// place the PSF in the top-left corner of a zeroed n x n image
hipError_t launch_pad_psf(const float* psf, int p, float* dst, int n, hipStream_t s);
// the PSF centred at the origin (kernel of the periodic-boundary blur)
hipError_t launch_pad_psf_centred(const float* psf, int p, float* dst, int n, hipStream_t s);
// transform batching chosen for size n (row pairs / columns per workgroup)
int fft_rows_batch(int n);
// a run-time transform of length n fits one workgroup's LDS (directly or in
// the Bluestein form)
bool fft_length_supported(int n);
int fft_cols_batch(int n);
int fft_seq_shift(int batch);
// the largest valid batching <= want (a power of two) for size n
int fft_rows_batch_at_most(int n, int want);
int fft_cols_batch_at_most(int n, int want);
// batched preconditioner passes: pass 0 rows forward, 1 columns, 2 rows inverse
int precond_pass_tiles(const BatchImage& I, int pass);
// pass 3: columns, inverse FFT only, of the real dense spectrum I.eacc (into swork)
hipError_t launch_precond_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                  int pass, int precond, int nmax, hipStream_t s,
                                  int any_len = 0);

// ---- PSF correlations of the reverse sweep ---------------------------------
// Per tile of the n x n grid, running sums over the steps of
//   part[b][a*p+q] += sum_{y,x} tk[y][x] u[y+p-1-a][x+p-1-q] - t[y][x] uk[y+p-1-a][x+p-1-q]
//   apart[b]       -= sum_{y,x} t[y][x] tk[y][x]
//   dg             (+)= t   (written at the first step)
// with u = W^T zbar and t = rbar of the descriptor.
int psf_corr_tiles(const BatchImage& I);
hipError_t launch_psf_corr_batched(const BatchImage* imgs, const int* bmap, const int* bfirst, int nblocks,
                                   int p, int first, double* part, double* apart, hipStream_t s);
// spec[i][a*p+q] = -2 n^2 sum_{a',q'} H[a'][q'] e[(a'-a) mod n][(q'-q) mod n], e = I.t (one workgroup per image)
hipError_t launch_psf_spectral_batched(const BatchImage* imgs, int count, int p, double* spec, hipStream_t s);
// Running partials of the reverse sweep and their final reduction into
// dmu[bands], dalpha and dpsf[p*p] (all device doubles, written).
struct UnrolledSums {
    int bands, levels, p, count, corr_blocks;
    int mu_blocks[4];
    const double* mu_part[4];  // per level [blocks][9]
    const double* alpha_part;  // [corr_blocks]
    const double* corr_part;   // [corr_blocks][p*p]
    const double* spec;        // [count][p*p]
};
hipError_t launch_unrolled_reduce(const UnrolledSums& S, double* dmu, double* dalpha, double* dpsf, hipStream_t s);

// ---- reductions and small helpers ---------------------------------------
// out[0] = sum of partials[0..count) in a fixed order (double)
hipError_t launch_sum_partials(const double* partials, int count, double* out, hipStream_t s);
// partial sums of a*b over `count` floats (one double per workgroup); returns #partials
hipError_t launch_dot_partials(const float* a, const float* b, size_t count, double* partials,
                               int* n_partials, hipStream_t s);
hipError_t launch_scale(float* x, size_t count, const double* inv_norm_sq_or_null, float factor,
                        hipStream_t s);
hipError_t launch_fill_hash(float* x, size_t count, unsigned seed, hipStream_t s);
hipError_t launch_fill(float* x, size_t count, float value, hipStream_t s);
int reduce_partials_cap();
// preconditioned CG of Algorithm 2: t += a d, res -= a q with a = *rho / *pq
hipError_t launch_pcg_update(float* t, float* res, const float* d, const float* q, size_t count, const double* rho,
                             const double* pq, const double* act, hipStream_t s);
// d = z + (*rho_new / *rho) d; both skipped once *act == 0
hipError_t launch_pcg_dir(float* d, const float* z, size_t count, const double* rho_new, const double* rho,
                          const double* act, hipStream_t s);
// CG state st[] (see reduce.hip): begin after rho_0 is in st[0]; check after step j
hipError_t launch_pcg_begin(double* st, int* hist, hipStream_t s);
hipError_t launch_pcg_check(double* st, const double* rn, int j, int max_steps, double tol, int* hist,
                            hipStream_t s);
hipError_t launch_axpy(float* y, const float* x, size_t count, float a, hipStream_t s);  // y += a x
// w -= ab[0] v + sqrt(*beta2) vprev (vprev may be null), partial sums of w^2
hipError_t launch_lanczos_step(float* w, const float* v, const float* vprev, size_t count, const double* ab,
                               const double* beta2, double* partials, int* n_partials, hipStream_t s);
// rn[image][k] = sum of that image's residual-norm partials (one workgroup per image)
hipError_t launch_sum_partials_batched(const BatchImage* imgs, const double* partials, const int* pcount,
                                       int count, int k, hipStream_t s);

}  // namespace mlba
