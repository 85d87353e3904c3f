// mlba_apply_P_static: the spectral preconditioner of Algorithm 1 (BCCB) or
// Algorithm 3 (DCT of the symmetrised PSF) without a plan and without any
// device allocation.  The transform tables, the spectrum of the PSF and the
// transposed spectral workspace live in one file-scope device array; every
// call rebuilds the tables and the spectrum there from the PSF it is given,
// then runs the same three transform passes as mlba_apply_P.
#include <math.h>

#include <mutex>

#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"
#include "mlba.h"
#include "plan.hpp"

using namespace mlba;

namespace {

constexpr int kStaticMaxN = MLBA_STATIC_MAX_N;

// Float offsets of the scratch regions for a transform length n (each
// region starts on a 256-byte boundary).
struct StaticLayout {
    size_t tw, dtw, costab, tmp, spec, swork, total;
};

constexpr size_t round64(size_t v) { return (v + 63) / 64 * 64; }

constexpr StaticLayout static_layout(int n, int precond) {
    StaticLayout L{};
    const size_t nn = (size_t)n * n;
    L.tw = 0;
    L.dtw = L.tw + round64(2 * (size_t)n);
    L.costab = L.dtw + round64(2 * (size_t)n);
    L.tmp = L.costab + round64(2 * (size_t)n);
    L.spec = L.tmp + round64(nn);
    const size_t spec = precond == MLBA_PRECOND_BCCB ? (size_t)(n / 2 + 1) * n : nn;
    L.swork = L.spec + round64(spec);
    const size_t work = precond == MLBA_PRECOND_BCCB ? (size_t)(n / 2 + 1) * (n + 16) * 2 : (size_t)n * (n + 32);
    L.total = L.swork + round64(work);
    return L;
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kScratchFloats =
    cmax(static_layout(kStaticMaxN, MLBA_PRECOND_BCCB).total, static_layout(kStaticMaxN, MLBA_PRECOND_DCT).total);

}  // namespace

// The scratch memory of mlba_apply_P_static: one copy per device, held until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

// Twiddle and cosine tables of the transforms, in double, rounded once:
// tw[q] = exp(-2 pi i q / n), dtw[q] = exp(-i pi q / (2n)) (q < n),
// costab[q] = cos(pi q / n) (q < 2n).
__global__ __launch_bounds__(kBlock) void static_tables_kernel(int n, float2* __restrict__ tw,
                                                               float2* __restrict__ dtw, float* __restrict__ costab) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q < n) {
        double sn, cs;
        sincospi(-2.0 * (double)q / (double)n, &sn, &cs);
        tw[q] = make_float2((float)cs, (float)sn);
        sincospi(-(double)q / (2.0 * (double)n), &sn, &cs);
        dtw[q] = make_float2((float)cs, (float)sn);
    }
    if (q < 2 * n) costab[q] = (float)cospi((double)q / (double)n);
}

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
float* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device).
int scratch_address(float** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MLBA_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return MLBA_EHIP;
        g_scratch[dev] = (float*)ptr;
    }
    *out = g_scratch[dev];
    return MLBA_OK;
}

}  // namespace

extern "C" int mlba_apply_P_static(const float* psf, int n, int p, int precond, const float* r, float* t,
                                   double alpha, hipStream_t s) {
    if (!psf || !r || !t || !(alpha > 0.0) || !isfinite(alpha)) return MLBA_EINVAL;
    if (p < 1 || p % 2 == 0 || p > n) return MLBA_EINVAL;
    if (precond != MLBA_PRECOND_BCCB && precond != MLBA_PRECOND_DCT) return MLBA_EUNSUPPORTED;
    if (n % 2 != 0 || n < 8 || n > kStaticMaxN || !fft_length_supported(n)) return MLBA_EUNSUPPORTED;
    const FftDesc fd = mlba_internal_fft_desc(n);
    if (fd.m > 0) return MLBA_EUNSUPPORTED;  // only 2^a 3^b 5^c lengths
    float* base = nullptr;
    STCHK(scratch_address(&base));
    const StaticLayout L = static_layout(n, precond);
    if (L.total > kScratchFloats) return MLBA_EUNSUPPORTED;
    float2* tw = (float2*)(base + L.tw);
    float2* dtw = (float2*)(base + L.dtw);
    float* costab = base + L.costab;
    float* tmp = base + L.tmp;
    float* spec = base + L.spec;
    const float inv = (float)(1.0 / ((double)n * (double)n));
    hipLaunchKernelGGL(static_tables_kernel, dim3((2 * n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, tw, dtw,
                       costab);
    HIPCHK(hipGetLastError());
    if (precond == MLBA_PRECOND_BCCB) {
        const int ts = n + 16;
        float2* T = (float2*)(base + L.swork);
        // |Lambda|^2 of the BCCB matrix (section 4.1), then the filter
        HIPCHK(launch_pad_psf(psf, p, tmp, n, s));
        HIPCHK(launch_fft_rows_r2c(tmp, n, T, ts, fd, tw, s));
        HIPCHK(launch_fft_cols_power(T, n, ts, spec, fd, tw, s));
        HIPCHK(launch_fft_rows_r2c(r, n, T, ts, fd, tw, s));
        HIPCHK(launch_fft_cols_filter(T, n, ts, spec, (float)alpha, inv, fd, tw, s));
        HIPCHK(launch_fft_rows_c2r(T, n, ts, t, fd, tw, s));
    } else {
        const int ts = n + 32;
        float* Tr = base + L.swork;
        // lambda^2 of the reflective blur of the symmetrised PSF (section 4.3)
        HIPCHK(launch_cos_spectrum(psf, p, n, n, 0, costab, tmp, spec, nullptr, s));
        HIPCHK(launch_dct_rows_fwd(r, n, Tr, ts, fd, tw, dtw, s));
        HIPCHK(launch_dct_cols_filter(Tr, n, ts, spec, (float)alpha, inv, fd, tw, dtw, s));
        HIPCHK(launch_dct_rows_inv(Tr, n, ts, t, fd, tw, dtw, s));
    }
    return MLBA_OK;
}
